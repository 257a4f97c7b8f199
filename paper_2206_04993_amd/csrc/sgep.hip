// sgep.hip -- host side of the C ABI declared in include/sgep.h.
//
// Owns the device state of one solver, validates arguments synchronously,
// chooses launch shapes once at init, and enqueues the two kernels of an
// iteration (sgep_kernels.hpp) on the handle's stream.  sgep_step performs
// no allocation, no synchronisation and no host copy, so it can be captured
// in a hipGraph.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <new>
#include <vector>

#include "../../include/sgep.h"
#include "sgep_kernels.hpp"
#include "sgep_wide.hpp"

using sgep::Coef;
using sgep::StepArgs;
using sgep::wide::WideArgs;

namespace {

constexpr uint32_t kStateMagic = 0x53474550u; // "SGEP"
constexpr uint32_t kStateVersion = 1u;

struct StateHeader {
    uint32_t magic, version;
    uint64_t cfg_hash;
    int64_t d, kp;
    int64_t elem;
    int64_t adam;
};

} // namespace

struct sgep_handle_s {
    sgep_config cfg;
    int64_t d = 0;
    int kp = 0, mb = 0, ft = 0;
    size_t esz = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    void *V = nullptr, *G = nullptr, *Am = nullptr, *As = nullptr;
    void *P = nullptr, *Q = nullptr;
    double *gram_part = nullptr, *stat_part = nullptr, *stat_tot = nullptr, *readout = nullptr;
    Coef *coef = nullptr;
    int n_tx = 0, n_ty = 0, n_tiles = 0;
    int ldg = 0, lds = 0;   // leading dimensions of the partial arrays
    int64_t W = 0;          // partial width: KP (KP + 1) / 2 + KP
    int64_t ldv = 0;        // player row length of V, G, Adam moments (padded views)
    int64_t dxp = 0;        // storage offset of view y in a player row (CCA)
    int64_t ldp = 0;        // player row length of P^T, Q^T
    int64_t fwd_blocks_max = 0;
    bool poisoned = false;
    // BF16 / FP8 path (sgep_wide.hpp): argument block with every field that
    // does not change between iterations, and its extra buffers
    bool wide = false;
    WideArgs wa;
    void *Vh = nullptr, *Vl = nullptr, *colscale = nullptr, *Ppart = nullptr;
    void *Wh = nullptr, *Wl = nullptr, *Mcls = nullptr, *Mbar = nullptr, *prior = nullptr;
};

namespace {

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull)
{
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t config_hash(const sgep_config &c)
{
    // hash every field explicitly (no struct padding in the digest)
    uint64_t h = 1469598103934665603ull;
    const int32_t ints[] = {c.kind, c.dtype, c.k, c.optimizer, c.schedule, c.n_classes};
    const int64_t dims[] = {c.dx, c.dy, c.b_max};
    const double reals[] = {c.eta0, c.eta_T, c.t0, c.t_c, c.T, c.gamma, c.rho, c.eps_reg,
                            c.adam_b1, c.adam_b2, c.adam_eps};
    h = fnv1a(ints, sizeof(ints), h);
    h = fnv1a(dims, sizeof(dims), h);
    h = fnv1a(reals, sizeof(reals), h);
    return h;
}

// feature-tile height of the backward pass: 16 features (MB = 1) keeps the
// tile count up for small d; wide problems use MB = 4 (2 when the LDS tiles of
// KP * sizeof(T) > 128 bytes per row would not fit) to cut the re-reads of P, Q
template <typename T> constexpr int mb_wide(int kp) { return (kp * (int)sizeof(T) <= 128) ? 4 : 2; }
constexpr int64_t kWideD = 8192;

void free_all(sgep_handle *h)
{
    void *ptrs[] = {h->V,  h->G,        h->Am,      h->As,    h->P,  h->Q,    h->gram_part,
                    h->stat_part, h->stat_tot, h->readout, h->coef, h->Vh, h->Vl, h->colscale,
                    h->Ppart, h->Wh, h->Wl, h->Mcls, h->Mbar, h->prior};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
}

sgep_status check_cfg(const sgep_config *c)
{
    if (!c)
        return SGEP_EINVAL;
    if (c->kind != SGEP_KIND_CCA && c->kind != SGEP_KIND_GENERAL && c->kind != SGEP_KIND_LDA)
        return SGEP_EINVAL;
    if (c->dtype < SGEP_F64 || c->dtype > SGEP_FP8_E4M3)
        return SGEP_EINVAL;
    const bool narrow = c->dtype == SGEP_BF16 || c->dtype == SGEP_FP8_E4M3;
    const bool lda = c->kind == SGEP_KIND_LDA;
    // LDA runs on the BF16 path only; GENERAL on the F64 / F32 path only
    if ((lda && c->dtype != SGEP_BF16) || (narrow && c->kind == SGEP_KIND_GENERAL))
        return SGEP_EUNSUPPORTED;
    if (c->k < 1)
        return SGEP_EINVAL;
    if (c->k > 64 || ((c->dtype == SGEP_F64 || (narrow && !lda)) && c->k > 32))
        return SGEP_EUNSUPPORTED;
    if (c->optimizer != SGEP_SGD && c->optimizer != SGEP_ADAM)
        return SGEP_EINVAL;
    if (c->schedule < SGEP_SCHED_CONST || c->schedule > SGEP_SCHED_WARMUP_HARMONIC)
        return SGEP_EINVAL;
    if (lda) {
        if (c->n_classes < 2 || c->n_classes > sgep::wide::kMaxCls)
            return SGEP_EINVAL;
        if (c->dx < 1 || c->dy != 0 || c->b_max < 1)
            return SGEP_ESHAPE;
    } else if (c->dx < 1 || c->dy < 1 || c->b_max < 1) {
        return SGEP_ESHAPE;
    }
    if (c->kind == SGEP_KIND_GENERAL && c->dx != c->dy)
        return SGEP_ESHAPE;
    if (narrow && (c->dx % 8 != 0 || c->dy % 8 != 0))
        return SGEP_ESHAPE;
    const int64_t d = c->kind == SGEP_KIND_CCA ? c->dx + c->dy : c->dx;
    if (c->k > d)
        return SGEP_ESHAPE;
    // partial reductions are sized for at most 2^19 rows / features
    if (c->b_max > (int64_t)1 << 19 || d > (int64_t)1 << 19)
        return SGEP_EUNSUPPORTED;
    if (!(c->eta0 >= 0.0) || !(c->gamma > 0.0 && c->gamma <= 1.0) || !(c->rho >= 0.0))
        return SGEP_EINVAL;
    if (c->kind == SGEP_KIND_CCA && c->eps_reg != 0.0)
        return SGEP_EINVAL;
    if (!(c->eps_reg >= 0.0))
        return SGEP_EINVAL;
    if (c->schedule == SGEP_SCHED_INV && !(c->t0 > 0.0))
        return SGEP_EINVAL;
    if (c->schedule == SGEP_SCHED_WARMUP_HARMONIC &&
        (!(c->t_c > 0.0) || !(c->T > c->t_c) || !(c->eta0 > c->eta_T) || !(c->eta_T > 0.0)))
        return SGEP_EINVAL;
    if (c->optimizer == SGEP_ADAM &&
        (!(c->adam_b1 >= 0.0 && c->adam_b1 < 1.0) || !(c->adam_b2 >= 0.0 && c->adam_b2 < 1.0) ||
         !(c->adam_eps > 0.0)))
        return SGEP_EINVAL;
    return SGEP_OK;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        if ((x) != hipSuccess)                                                             \
            return SGEP_EDEVICE;                                                           \
    } while (0)

template <typename T, int KP>
sgep_status launch_init(sgep_handle *h)
{
    hipLaunchKernelGGL((sgep::k_init<T, KP>), dim3(1), dim3(sgep::kNT), 0, h->stream, (T *)h->V,
                       (T *)h->G, h->ldv, h->cfg.k, h->stat_part, h->lds, h->coef);
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

// One launch of a step kernel.  With timing events the launch goes through
// hipExtLaunchKernelGGL, which stamps e0 / e1 with the start and end of the
// kernel's own dispatch (no launch gaps), the same interval a kernel trace
// reports.
template <typename K>
void launch_timed(K kernel, dim3 grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                  const StepArgs &a)
{
    if (e0)
        hipExtLaunchKernelGGL(kernel, grid, dim3(sgep::kNT), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(kernel, grid, dim3(sgep::kNT), 0, s, a);
}

template <typename T, int KP, int MB>
void launch_bwd(sgep_handle *h, const StepArgs &a, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 gb(h->n_tiles);
    const bool cca = h->cfg.kind == SGEP_KIND_CCA;
    const bool adam = h->cfg.optimizer == SGEP_ADAM;
    if (cca && !adam)
        launch_timed(sgep::k_bwd<T, KP, MB, sgep::kKindCCA, sgep::kOptSGD>, gb, h->stream, e0, e1, a);
    else if (cca && adam)
        launch_timed(sgep::k_bwd<T, KP, MB, sgep::kKindCCA, sgep::kOptAdam>, gb, h->stream, e0, e1, a);
    else if (!adam)
        launch_timed(sgep::k_bwd<T, KP, MB, sgep::kKindGeneral, sgep::kOptSGD>, gb, h->stream, e0, e1,
                     a);
    else
        launch_timed(sgep::k_bwd<T, KP, MB, sgep::kKindGeneral, sgep::kOptAdam>, gb, h->stream, e0,
                     e1, a);
}

template <typename T, int KP>
sgep_status launch_step(sgep_handle *h, const StepArgs &a, void *const *events)
{
    const dim3 gf(a.n_fwd + 1); // + the norm-totals workgroup
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (events)
        for (int i = 0; i < 4; ++i)
            ev[i] = (hipEvent_t)events[i];
    if (h->cfg.kind == SGEP_KIND_CCA)
        launch_timed(sgep::k_fwd<T, KP, sgep::kKindCCA>, gf, h->stream, ev[0], ev[1], a);
    else
        launch_timed(sgep::k_fwd<T, KP, sgep::kKindGeneral>, gf, h->stream, ev[0], ev[1], a);
    if (h->mb == 1)
        launch_bwd<T, KP, 1>(h, a, ev[2], ev[3]);
    else
        launch_bwd<T, KP, mb_wide<T>(KP)>(h, a, ev[2], ev[3]);
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

template <typename T, int KP>
sgep_status launch_readout(sgep_handle *h, const void *S, int mode)
{
    const int64_t dx = h->cfg.kind == SGEP_KIND_CCA ? h->cfg.dx : h->d;
    hipLaunchKernelGGL((sgep::k_readout<T, KP>), dim3(1), dim3(sgep::kNT), 0, h->stream,
                       (const T *)S, h->d, dx, h->dxp, h->ldv, h->cfg.k, h->stat_part, h->n_tiles,
                       h->lds, h->cfg.rho, h->coef, mode, h->readout);
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

// ---------------------------------------------------------------------------
// BF16 / FP8 path
// ---------------------------------------------------------------------------
template <typename K, typename... Args>
void launch_k(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
              Args... args)
{
    if (e0)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

int wide_stat_blocks(const WideArgs &a)
{
    return (a.Ws + sgep::wide::kStatCols - 1) / sgep::wide::kStatCols;
}

template <int KP, int IN, int KIND>
sgep_status wide_step_t(sgep_handle *h, const WideArgs &a, const hipEvent_t *ev)
{
    using namespace sgep::wide;
    const dim3 blk(kWT);
    const bool adam = h->cfg.optimizer == SGEP_ADAM;
    // forward workgroups, then the statistics reductions
    launch_k(k_wfwd<KP, IN>, dim3(a.n_rb * a.nview * a.n_split + wide_stat_blocks(a)), blk,
             h->stream, ev[0], ev[1], a);
    launch_k(k_wmid<KP, KIND>, dim3(a.nA), blk, h->stream, ev[2], ev[3], a);
    const dim3 bblk(kBT);
    if (adam)
        launch_k(k_wbwd<KP, IN, KIND, sgep::kOptAdam>, dim3(a.nwg), bblk, h->stream, ev[4], ev[5], a);
    else
        launch_k(k_wbwd<KP, IN, KIND, sgep::kOptSGD>, dim3(a.nwg), bblk, h->stream, ev[4], ev[5], a);
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

template <int KP, int IN, int KIND>
sgep_status wide_init_t(sgep_handle *h, const WideArgs &a, const hipEvent_t *)
{
    hipLaunchKernelGGL((sgep::wide::k_winit<KP, IN, KIND>), dim3(a.nwg), dim3(sgep::wide::kBT), 0,
                       h->stream, a);
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

// reduce the latest statistics, then scale the state rows into h->readout
template <int KP, int IN, int KIND>
sgep_status wide_readout_t(sgep_handle *h, const WideArgs &a, const void *S, int mode)
{
    using namespace sgep::wide;
    hipLaunchKernelGGL(k_wstats, dim3(wide_stat_blocks(a)), dim3(kWT), 0, h->stream, a);
    const int64_t n = h->d * (int64_t)h->cfg.k;
    int64_t nb = (n + 255) / 256;
    if (nb > 1024)
        nb = 1024;
    const int64_t dx = h->cfg.kind == SGEP_KIND_CCA ? h->cfg.dx : h->d;
    hipLaunchKernelGGL((k_wreadout<KP>), dim3((unsigned)nb), dim3(256), 0, h->stream,
                       (const float *)S, (const double *)a.stot, h->d, dx, a.off[1], h->cfg.k,
                       h->cfg.rho, h->coef, mode, h->readout);
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

// dispatch on (input format, kind, KP) for the BF16 / FP8 path
#define WIDE_DISPATCH(h, FN, ...)                                                          \
    ([&]() -> sgep_status {                                                                \
        using namespace sgep::wide;                                                        \
        if ((h)->cfg.kind == SGEP_KIND_LDA) {                                              \
            if ((h)->kp == 16) return FN<16, kInBF16, kKindLDA>(__VA_ARGS__);              \
            if ((h)->kp == 32) return FN<32, kInBF16, kKindLDA>(__VA_ARGS__);              \
            if ((h)->kp == 64) return FN<64, kInBF16, kKindLDA>(__VA_ARGS__);              \
        } else if ((h)->cfg.dtype == SGEP_FP8_E4M3) {                                      \
            if ((h)->kp == 16) return FN<16, kInFP8, sgep::kKindCCA>(__VA_ARGS__);         \
            if ((h)->kp == 32) return FN<32, kInFP8, sgep::kKindCCA>(__VA_ARGS__);         \
        } else {                                                                           \
            if ((h)->kp == 16) return FN<16, kInBF16, sgep::kKindCCA>(__VA_ARGS__);        \
            if ((h)->kp == 32) return FN<32, kInBF16, sgep::kKindCCA>(__VA_ARGS__);        \
        }                                                                                  \
        return SGEP_EUNSUPPORTED;                                                          \
    }())

// dispatch on (dtype, KP)
#define SGEP_DISPATCH(h, FN, ...)                                                          \
    ([&]() -> sgep_status {                                                                \
        if ((h)->cfg.dtype == SGEP_F64) {                                                  \
            if ((h)->kp == 16) return FN<double, 16>(__VA_ARGS__);                         \
            if ((h)->kp == 32) return FN<double, 32>(__VA_ARGS__);                         \
        } else {                                                                           \
            if ((h)->kp == 16) return FN<float, 16>(__VA_ARGS__);                          \
            if ((h)->kp == 32) return FN<float, 32>(__VA_ARGS__);                          \
            if ((h)->kp == 64) return FN<float, 64>(__VA_ARGS__);                          \
        }                                                                                  \
        return SGEP_EUNSUPPORTED;                                                          \
    }())

sgep_status latch_status(sgep_handle *h)
{
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, &h->coef->status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (st != 0) {
        h->poisoned = true;
        return SGEP_ENONFINITE;
    }
    return SGEP_OK;
}

sgep_status check_aux(const sgep_config *c, const sgep_init_aux *aux)
{
    const bool fp8 = c->dtype == SGEP_FP8_E4M3, lda = c->kind == SGEP_KIND_LDA;
    const bool has_scale = aux && (aux->x_col_scale || aux->y_col_scale);
    const bool has_cls = aux && (aux->class_means || aux->class_priors);
    if (has_scale != fp8 || has_cls != lda)
        return SGEP_EINVAL;
    if (fp8) {
        if (!aux->x_col_scale || !aux->y_col_scale)
            return SGEP_EINVAL;
        for (int64_t f = 0; f < c->dx; ++f)
            if (!(aux->x_col_scale[f] > 0.f) || !std::isfinite(aux->x_col_scale[f]))
                return SGEP_EINVAL;
        for (int64_t f = 0; f < c->dy; ++f)
            if (!(aux->y_col_scale[f] > 0.f) || !std::isfinite(aux->y_col_scale[f]))
                return SGEP_EINVAL;
    }
    if (lda) {
        if (!aux->class_means || !aux->class_priors)
            return SGEP_EINVAL;
        for (int cc = 0; cc < c->n_classes; ++cc)
            if (!(aux->class_priors[cc] > 0.0) || !std::isfinite(aux->class_priors[cc]))
                return SGEP_EINVAL;
        for (int64_t e = 0; e < (int64_t)c->n_classes * c->dx; ++e)
            if (!std::isfinite(aux->class_means[e]))
                return SGEP_EINVAL;
    }
    return SGEP_OK;
}

// Set up the BF16 / FP8 path: launch geometry, buffers, starting state (unit
// columns of V0, normalised here in FP64; [Bv] = V, the BF16 operand and the
// first statistics are written by k_winit).
sgep_status init_wide(sgep_handle *h, const double *V0, const sgep_init_aux *aux)
{
    using namespace sgep::wide;
    const sgep_config &c = h->cfg;
    const bool lda = c.kind == SGEP_KIND_LDA, fp8 = c.dtype == SGEP_FP8_E4M3;
    const int64_t KP = h->kp, d = h->d;
    auto r64 = [](int64_t x) { return (x + 63) / 64 * 64; };
    WideArgs &a = h->wa;
    memset(&a, 0, sizeof(a));
    h->esz = fp8 ? 1 : 2; // element size of the minibatch (checkpoint header)
    a.nview = lda ? 1 : 2;
    a.dv[0] = c.dx;
    a.dv[1] = lda ? 0 : c.dy;
    a.off[0] = 0;
    a.off[1] = r64(c.dx);
    a.dtot = lda ? r64(c.dx) : r64(c.dx) + r64(c.dy);
    a.k = c.k;
    a.ncls = lda ? c.n_classes : 0;
    a.ldr = r64(c.b_max);
    // forward: aim at >= 512 workgroups at b_max, each wave >= one 64-feature step
    const int64_t nrb = a.ldr / kRB;
    const int64_t dvmax = a.dv[0] > a.dv[1] ? a.dv[0] : a.dv[1];
    const int64_t nf64 = (dvmax + 63) / 64;
    int64_t ns = (512 + nrb * a.nview - 1) / (nrb * a.nview);
    const int64_t ns_max = (nf64 + kNW - 1) / kNW;
    if (ns > ns_max)
        ns = ns_max;
    if (ns < 1)
        ns = 1;
    a.fw = 64 * ((nf64 + kNW * ns - 1) / (kNW * ns));
    a.fs = kNW * a.fw;
    a.n_split = (int32_t)((dvmax + a.fs - 1) / a.fs);
    // backward: 64-feature subtiles, about 256 workgroups
    a.nsubv[0] = (int32_t)((a.dv[0] + kFT - 1) / kFT);
    a.nsubv[1] = (int32_t)((a.dv[1] + kFT - 1) / kFT);
    const int nsubt = a.nsubv[0] + a.nsubv[1];
    a.nsub = nsubt / 256 > 1 ? nsubt / 256 : 1;
    a.nwg0 = (a.nsubv[0] + a.nsub - 1) / a.nsub;
    a.nwg = a.nwg0 + (a.nsubv[1] + a.nsub - 1) / a.nsub;
    a.lds = (a.nwg + 1) / 2 * 2;
    a.Ws = (int32_t)(KP * (KP + 1) / 2 + KP + (lda ? a.ncls * KP : 0));
    const int64_t MW = lda ? KP + 16 : 2 * KP;

    bool ok = true;
    auto alloc = [&](void **p, size_t n) {
        if (ok && hipMalloc(p, n < 256 ? 256 : n) != hipSuccess) {
            *p = nullptr;
            ok = false;
        }
    };
    const size_t st = (size_t)a.dtot * KP * sizeof(float);
    const size_t op = (size_t)KP * a.dtot * sizeof(uint16_t);
    const size_t wbytes = (size_t)MW * a.ldr * sizeof(uint16_t);
    const size_t spb = (size_t)a.Ws * a.lds * sizeof(double);
    alloc(&h->V, st);
    alloc(&h->G, st);
    if (c.optimizer == SGEP_ADAM) {
        alloc(&h->Am, st);
        alloc(&h->As, st);
    }
    alloc(&h->Vh, op);
    alloc(&h->Vl, op);
    if (fp8)
        alloc(&h->colscale, (size_t)a.dtot * sizeof(float));
    alloc(&h->Ppart, (size_t)a.n_split * a.nview * a.ldr * KP * sizeof(float));
    alloc(&h->Wh, wbytes);
    alloc(&h->Wl, wbytes);
    if (lda) {
        alloc(&h->Mcls, (size_t)a.ncls * a.dtot * sizeof(float));
        alloc(&h->Mbar, (size_t)a.dtot * sizeof(float));
        alloc(&h->prior, (size_t)a.ncls * sizeof(double));
    }
    alloc((void **)&h->stat_part, spb);
    alloc((void **)&h->stat_tot, (size_t)a.Ws * sizeof(double));
    alloc((void **)&h->readout, (size_t)d * c.k * sizeof(double));
    alloc((void **)&h->coef, sizeof(Coef));
    if (!ok)
        return SGEP_ENOMEM;
    a.V = (float *)h->V;
    a.G = (float *)h->G;
    a.Am = (float *)h->Am;
    a.As = (float *)h->As;
    a.Vh = (uint16_t *)h->Vh;
    a.Vl = (uint16_t *)h->Vl;
    a.colscale = (const float *)h->colscale;
    a.Ppart = (float *)h->Ppart;
    a.Wh = (uint16_t *)h->Wh;
    a.Wl = (uint16_t *)h->Wl;
    a.M = (const float *)h->Mcls;
    a.Mbar = (const float *)h->Mbar;
    a.prior = (const double *)h->prior;
    a.spart = h->stat_part;
    a.stot = h->stat_tot;
    a.coef = h->coef;
    a.schedule = c.schedule;
    a.eta0 = c.eta0;
    a.eta_T = c.eta_T;
    a.t0 = c.t0;
    a.t_c = c.t_c;
    a.T = c.T;
    a.gamma = c.gamma;
    a.rho = c.rho;
    a.eps_reg = c.eps_reg;
    a.adam_b1 = c.adam_b1;
    a.adam_b2 = c.adam_b2;
    a.adam_eps = c.adam_eps;

    // starting players: unit columns (FP64 norms), FP32, state rows of the views
    auto row_of = [&](int64_t f) { return f < c.dx ? f : a.off[1] + (f - c.dx); };
    std::vector<float> hv((size_t)a.dtot * KP, 0.f);
    for (int i = 0; i < c.k; ++i) {
        double n2 = 0.0;
        for (int64_t f = 0; f < d; ++f)
            n2 += V0[(size_t)i * d + f] * V0[(size_t)i * d + f];
        if (!(n2 > 0.0) || !std::isfinite(n2))
            return SGEP_EINVAL; // zero or non-finite starting column
        const double inv = 1.0 / sqrt(n2);
        for (int64_t f = 0; f < d; ++f)
            hv[(size_t)row_of(f) * KP + i] = (float)(V0[(size_t)i * d + f] * inv);
    }
    std::vector<float> hs, hm, hmb;
    std::vector<double> hp;
    bool hok = hipMemsetAsync(h->coef, 0, sizeof(Coef), h->stream) == hipSuccess &&
               hipMemsetAsync(h->stat_part, 0, spb, h->stream) == hipSuccess &&
               hipMemsetAsync(h->Vh, 0, op, h->stream) == hipSuccess &&
               hipMemsetAsync(h->Vl, 0, op, h->stream) == hipSuccess &&
               hipMemsetAsync(h->Wh, 0, wbytes, h->stream) == hipSuccess &&
               hipMemsetAsync(h->Wl, 0, wbytes, h->stream) == hipSuccess &&
               hipMemcpyAsync(h->V, hv.data(), st, hipMemcpyHostToDevice, h->stream) == hipSuccess;
    if (h->Am)
        hok = hok && hipMemsetAsync(h->Am, 0, st, h->stream) == hipSuccess &&
              hipMemsetAsync(h->As, 0, st, h->stream) == hipSuccess;
    if (fp8) {
        hs.assign((size_t)a.dtot, 0.f);
        for (int64_t f = 0; f < d; ++f)
            hs[(size_t)row_of(f)] = f < c.dx ? aux->x_col_scale[f] : aux->y_col_scale[f - c.dx];
        hok = hok && hipMemcpyAsync(h->colscale, hs.data(), hs.size() * sizeof(float),
                                    hipMemcpyHostToDevice, h->stream) == hipSuccess;
    }
    if (lda) {
        hm.assign((size_t)a.ncls * a.dtot, 0.f);
        hmb.assign((size_t)a.dtot, 0.f);
        hp.assign(aux->class_priors, aux->class_priors + a.ncls);
        for (int64_t f = 0; f < d; ++f) {
            double mb = 0.0;
            for (int cc = 0; cc < a.ncls; ++cc) {
                const double m = aux->class_means[(size_t)cc * d + f];
                hm[(size_t)cc * a.dtot + f] = (float)m;
                mb += hp[cc] * m;
            }
            hmb[(size_t)f] = (float)mb;
        }
        hok = hok &&
              hipMemcpyAsync(h->Mcls, hm.data(), hm.size() * sizeof(float), hipMemcpyHostToDevice,
                             h->stream) == hipSuccess &&
              hipMemcpyAsync(h->Mbar, hmb.data(), hmb.size() * sizeof(float),
                             hipMemcpyHostToDevice, h->stream) == hipSuccess &&
              hipMemcpyAsync(h->prior, hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice,
                             h->stream) == hipSuccess;
    }
    if (!hok)
        return SGEP_EDEVICE;
    sgep_status rc = WIDE_DISPATCH(h, wide_init_t, h, a, nullptr);
    if (rc != SGEP_OK)
        return rc;
    // waits for the uploads from the host vectors above
    if (hipStreamSynchronize(h->stream) != hipSuccess)
        return SGEP_EDEVICE;
    return SGEP_OK;
}

sgep_status step_wide(sgep_handle *h, const void *X, int64_t ldx, const void *Y, int64_t ldy,
                      const int32_t *labels, int64_t b, void *const *events)
{
    const sgep_config &c = h->cfg;
    const bool lda = c.kind == SGEP_KIND_LDA;
    if (!X || (lda ? !labels : (!Y || labels != nullptr)))
        return SGEP_EINVAL;
    if (b < 1 || b > c.b_max)
        return SGEP_ESHAPE;
    if (ldx < c.dx || ldx % 8 != 0 || ((uintptr_t)X & 15u) != 0)
        return SGEP_ESHAPE;
    if (!lda && (ldy < c.dy || ldy % 8 != 0 || ((uintptr_t)Y & 15u) != 0))
        return SGEP_ESHAPE;
    WideArgs a = h->wa;
    a.X = X;
    a.Y = lda ? nullptr : Y;
    a.labels = labels;
    a.ldx = ldx;
    a.ldy = lda ? 0 : ldy;
    a.b = b;
    a.n_rb = (int32_t)((b + sgep::wide::kRB - 1) / sgep::wide::kRB);
    a.nA = 4 * a.n_rb;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (events)
        for (int i = 0; i < 6; ++i)
            ev[i] = (hipEvent_t)events[i];
    return WIDE_DISPATCH(h, wide_step_t, h, a, ev);
}

// device arrays of a checkpoint after the header and the coefficient block
struct StateLayout {
    int n = 0;
    void *ptr[8];
    size_t bytes[8];
    void add(void *p, size_t b)
    {
        if (p) {
            ptr[n] = p;
            bytes[n] = b;
            ++n;
        }
    }
};

StateLayout state_layout(const sgep_handle *h)
{
    StateLayout L;
    if (h->wide) {
        const size_t st = (size_t)h->wa.dtot * h->kp * sizeof(float);
        const size_t op = (size_t)h->kp * h->wa.dtot * sizeof(uint16_t);
        L.add(h->V, st);
        L.add(h->G, st);
        L.add(h->Am, st);
        L.add(h->As, st);
        L.add(h->Vh, op);
        L.add(h->Vl, op);
        L.add(h->stat_part, (size_t)h->wa.Ws * h->wa.lds * sizeof(double));
    } else {
        const size_t st = (size_t)h->ldv * h->kp * h->esz;
        L.add(h->V, st);
        L.add(h->G, st);
        L.add(h->Am, st);
        L.add(h->As, st);
        L.add(h->stat_part, (size_t)h->W * h->lds * sizeof(double));
    }
    return L;
}

} // namespace

extern "C" {

int32_t sgep_version(void) { return 110; }

const char *sgep_status_string(sgep_status s)
{
    switch (s) {
    case SGEP_OK: return "ok";
    case SGEP_EINVAL: return "invalid argument";
    case SGEP_ESHAPE: return "inconsistent shape, leading dimension or alignment";
    case SGEP_ENOMEM: return "device allocation failed";
    case SGEP_EDEVICE: return "HIP runtime error";
    case SGEP_ENONFINITE: return "non-finite or zero norm / Gram term in a step";
    case SGEP_EUNSUPPORTED: return "not supported by this build";
    case SGEP_EPOISONED: return "handle poisoned by an earlier fault";
    default: return "unknown status";
    }
}

sgep_status sgep_init(sgep_handle **out, const sgep_config *cfg, const double *V0, void *hip_stream)
{
    return sgep_init_ex(out, cfg, V0, nullptr, hip_stream);
}

sgep_status sgep_init_ex(sgep_handle **out, const sgep_config *cfg, const double *V0,
                         const sgep_init_aux *aux, void *hip_stream)
{
    if (!out)
        return SGEP_EINVAL;
    *out = nullptr;
    sgep_status rc = check_cfg(cfg);
    if (rc != SGEP_OK)
        return rc;
    if (!V0)
        return SGEP_EINVAL;
    rc = check_aux(cfg, aux);
    if (rc != SGEP_OK)
        return rc;
    sgep_handle *h = new (std::nothrow) sgep_handle_s();
    if (!h)
        return SGEP_ENOMEM;
    h->cfg = *cfg;
    h->stream = (hipStream_t)hip_stream;
    h->d = cfg->kind == SGEP_KIND_CCA ? cfg->dx + cfg->dy : cfg->dx;
    h->kp = cfg->k <= 16 ? 16 : (cfg->k <= 32 ? 32 : 64);
    if (cfg->dtype == SGEP_BF16 || cfg->dtype == SGEP_FP8_E4M3) {
        h->wide = true;
        if (hipGetDevice(&h->device) != hipSuccess) {
            delete h;
            return SGEP_EDEVICE;
        }
        rc = init_wide(h, V0, aux);
        if (rc != SGEP_OK) {
            free_all(h);
            delete h;
            return rc;
        }
        *out = h;
        return SGEP_OK;
    }
    h->esz = cfg->dtype == SGEP_F64 ? sizeof(double) : sizeof(float);
    const bool wide = h->d >= kWideD;
    h->mb = !wide ? 1 : (cfg->dtype == SGEP_F64 ? mb_wide<double>(h->kp) : mb_wide<float>(h->kp));
    h->ft = 16 * h->mb;
    if (cfg->kind == SGEP_KIND_CCA) {
        h->n_tx = (int)((cfg->dx + h->ft - 1) / h->ft);
        h->n_ty = (int)((cfg->dy + h->ft - 1) / h->ft);
    } else {
        h->n_tx = (int)((cfg->dx + h->ft - 1) / h->ft);
        h->n_ty = 0;
    }
    h->n_tiles = h->n_tx + h->n_ty;
    h->fwd_blocks_max = (cfg->b_max + 15) / 16;
    h->ldg = (int)((h->fwd_blocks_max + 1) / 2 * 2);
    h->lds = (h->n_tiles + 1) / 2 * 2;
    h->W = (int64_t)h->kp * (h->kp + 1) / 2 + h->kp;
    auto r4 = [](int64_t x) { return (x + 3) / 4 * 4; };
    if (cfg->kind == SGEP_KIND_CCA) {
        h->dxp = r4(cfg->dx);
        h->ldv = h->dxp + r4(cfg->dy);
    } else {
        h->dxp = 0;
        h->ldv = r4(h->d);
    }
    h->ldp = r4(cfg->b_max);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return SGEP_EDEVICE;
    }

    const int64_t kp = h->kp, d = h->d;
    const size_t st_bytes = (size_t)h->ldv * kp * h->esz;
    bool ok = true;
    auto alloc = [&](void **p, size_t n) {
        if (ok && hipMalloc(p, n < 256 ? 256 : n) != hipSuccess) {
            *p = nullptr;
            ok = false;
        }
    };
    alloc(&h->V, st_bytes);
    alloc(&h->G, st_bytes);
    if (cfg->optimizer == SGEP_ADAM) {
        alloc(&h->Am, st_bytes);
        alloc(&h->As, st_bytes);
    }
    alloc(&h->P, (size_t)h->ldp * kp * h->esz);
    alloc(&h->Q, (size_t)h->ldp * kp * h->esz);
    alloc((void **)&h->gram_part, (size_t)h->W * h->ldg * sizeof(double));
    alloc((void **)&h->stat_part, (size_t)h->W * h->lds * sizeof(double));
    alloc((void **)&h->stat_tot, (size_t)h->W * sizeof(double));
    alloc((void **)&h->readout, (size_t)d * cfg->k * sizeof(double));
    alloc((void **)&h->coef, sizeof(Coef));
    if (!ok) {
        free_all(h);
        delete h;
        return SGEP_ENOMEM;
    }
    // zero state, then upload the raw starting points (padding columns zero)
    bool hok = hipMemsetAsync(h->coef, 0, sizeof(Coef), h->stream) == hipSuccess &&
               hipMemsetAsync(h->stat_part, 0, (size_t)h->W * h->lds * sizeof(double),
                              h->stream) == hipSuccess &&
               hipMemsetAsync(h->gram_part, 0, (size_t)h->W * h->ldg * sizeof(double),
                              h->stream) == hipSuccess;
    if (h->Am)
        hok = hok && hipMemsetAsync(h->Am, 0, st_bytes, h->stream) == hipSuccess &&
              hipMemsetAsync(h->As, 0, st_bytes, h->stream) == hipSuccess;
    // quad-interleaved with padded views: (feature f, player i) at
    // (sf / 4) 4 KP + 4 i + sf % 4, sf = storage position of f
    std::vector<unsigned char> host(st_bytes, 0);
    const int64_t dxv = cfg->kind == SGEP_KIND_CCA ? cfg->dx : d;
    for (int i = 0; i < cfg->k; ++i)
        for (int64_t f = 0; f < d; ++f) {
            const double v = V0[(size_t)i * d + f];
            const int64_t sf = f < dxv ? f : h->dxp + (f - dxv);
            const int64_t at = (sf >> 2) * 4 * kp + 4 * i + (sf & 3);
            if (h->esz == sizeof(double))
                ((double *)host.data())[at] = v;
            else
                ((float *)host.data())[at] = (float)v;
        }
    hok = hok && hipMemcpyAsync(h->V, host.data(), st_bytes, hipMemcpyHostToDevice, h->stream) ==
                     hipSuccess;
    if (!hok) {
        free_all(h);
        delete h;
        return SGEP_EDEVICE;
    }
    rc = SGEP_DISPATCH(h, launch_init, h);
    if (rc == SGEP_OK)
        rc = latch_status(h); // also waits for the upload of the host buffer
    if (rc != SGEP_OK) {
        free_all(h);
        delete h;
        return rc == SGEP_ENONFINITE ? SGEP_EINVAL : rc; // zero starting column
    }
    *out = h;
    return SGEP_OK;
}

static sgep_status step_impl(sgep_handle *h, const void *X, int64_t ldx, const void *Y,
                             int64_t ldy, const int32_t *labels, int64_t b, void *const *events)
{
    if (!h)
        return SGEP_EINVAL;
    if (h->poisoned)
        return SGEP_EPOISONED;
    if (h->wide)
        return step_wide(h, X, ldx, Y, ldy, labels, b, events);
    if (!X || !Y || labels)
        return SGEP_EINVAL;
    if (b < 1 || b > h->cfg.b_max)
        return SGEP_ESHAPE;
    if (ldx < h->cfg.dx || ldy < h->cfg.dy)
        return SGEP_ESHAPE;
    const int64_t vec = 16 / (int64_t)h->esz;
    const bool vec_ok = ldx % vec == 0 && ldy % vec == 0 && ((uintptr_t)X & 15u) == 0 &&
                        ((uintptr_t)Y & 15u) == 0 && ((uintptr_t)X % h->esz) == 0 &&
                        ((uintptr_t)Y % h->esz) == 0;
    if (((uintptr_t)X % h->esz) != 0 || ((uintptr_t)Y % h->esz) != 0)
        return SGEP_ESHAPE; // not even element-aligned
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.X = X;
    a.Y = Y;
    a.ldx = ldx;
    a.ldy = ldy;
    a.b = b;
    a.dx = h->cfg.dx;
    a.dy = h->cfg.dy;
    a.dxp = h->dxp;
    a.ldv = h->ldv;
    a.ldp = h->ldp;
    a.k = h->cfg.k;
    a.n_tx = h->n_tx;
    a.n_ty = h->n_ty;
    a.vec_ok = vec_ok ? 1 : 0;
    a.n_fwd = (int32_t)((b + 15) / 16);
    a.ldg = h->ldg;
    a.lds = h->lds;
    a.V = h->V;
    a.G = h->G;
    a.Am = h->Am;
    a.As = h->As;
    a.P = h->P;
    a.Q = h->Q;
    a.gram_part = h->gram_part;
    a.stat_part = h->stat_part;
    a.stat_tot = h->stat_tot;
    a.coef = h->coef;
    a.schedule = h->cfg.schedule;
    a.eta0 = h->cfg.eta0;
    a.eta_T = h->cfg.eta_T;
    a.t0 = h->cfg.t0;
    a.t_c = h->cfg.t_c;
    a.T = h->cfg.T;
    a.gamma = h->cfg.gamma;
    a.rho = h->cfg.rho;
    a.eps_reg = h->cfg.eps_reg;
    a.adam_b1 = h->cfg.adam_b1;
    a.adam_b2 = h->cfg.adam_b2;
    a.adam_eps = h->cfg.adam_eps;
    return SGEP_DISPATCH(h, launch_step, h, a, events);
}

sgep_status sgep_step(sgep_handle *h, const void *X, int64_t ldx, const void *Y, int64_t ldy,
                      int64_t b)
{
    if (h && h->cfg.kind == SGEP_KIND_LDA)
        return SGEP_EINVAL; // labelled data: sgep_step_lda
    return step_impl(h, X, ldx, Y, ldy, nullptr, b, nullptr);
}

sgep_status sgep_step_lda(sgep_handle *h, const void *X, int64_t ldx, const int32_t *labels,
                          int64_t b)
{
    if (!h || h->cfg.kind != SGEP_KIND_LDA)
        return SGEP_EINVAL;
    return step_impl(h, X, ldx, nullptr, 0, labels, b, nullptr);
}

sgep_status sgep_kernels_per_step(const sgep_handle *h, int32_t *n)
{
    if (!h || !n)
        return SGEP_EINVAL;
    *n = h->wide ? 3 : 2;
    return SGEP_OK;
}

sgep_status sgep_step_profiled(sgep_handle *h, const void *X, int64_t ldx, const void *Y,
                               int64_t ldy, const int32_t *labels, int64_t b,
                               void *const *events, int32_t n_events)
{
    if (!h || !events)
        return SGEP_EINVAL;
    const int32_t need = h->wide ? 6 : 4;
    if (n_events != need)
        return SGEP_EINVAL;
    for (int i = 0; i < need; ++i)
        if (!events[i])
            return SGEP_EINVAL;
    if ((h->cfg.kind == SGEP_KIND_LDA) != (labels != nullptr))
        return SGEP_EINVAL;
    return step_impl(h, X, ldx, Y, ldy, labels, b, events);
}

sgep_status sgep_sync(sgep_handle *h)
{
    if (!h)
        return SGEP_EINVAL;
    if (h->poisoned)
        return SGEP_EPOISONED;
    return latch_status(h);
}

sgep_status sgep_eigvals(sgep_handle *h, double *out)
{
    if (!h || !out)
        return SGEP_EINVAL;
    if (h->poisoned)
        return SGEP_EPOISONED;
    sgep_status rc = latch_status(h);
    if (rc != SGEP_OK)
        return rc;
    Coef c;
    HIPCHK(hipMemcpyAsync(&c, h->coef, sizeof(Coef), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->cfg.k; ++i)
        out[i] = c.ema_a[i] / c.ema_b[i];
    return SGEP_OK;
}

static sgep_status readout(sgep_handle *h, const void *S, int mode, double *out)
{
    if (!h || !out)
        return SGEP_EINVAL;
    if (h->poisoned)
        return SGEP_EPOISONED;
    sgep_status rc = latch_status(h);
    if (rc != SGEP_OK)
        return rc;
    if (h->wide)
        rc = WIDE_DISPATCH(h, wide_readout_t, h, h->wa, S, mode);
    else
        rc = SGEP_DISPATCH(h, launch_readout, h, S, mode);
    if (rc != SGEP_OK)
        return rc;
    HIPCHK(hipMemcpyAsync(out, h->readout, (size_t)h->d * h->cfg.k * sizeof(double),
                          hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return SGEP_OK;
}

sgep_status sgep_vectors(sgep_handle *h, int32_t b_normalized, double *out)
{
    if (!h)
        return SGEP_EINVAL;
    return readout(h, h->V, b_normalized ? 2 : 1, out);
}

sgep_status sgep_auxiliary(sgep_handle *h, double *out)
{
    if (!h)
        return SGEP_EINVAL;
    return readout(h, h->G, 0, out);
}

sgep_status sgep_step_count(sgep_handle *h, int64_t *t)
{
    if (!h || !t)
        return SGEP_EINVAL;
    if (h->poisoned)
        return SGEP_EPOISONED;
    double tt = 0.0;
    HIPCHK(hipMemcpyAsync(&tt, &h->coef->t, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    *t = (int64_t)tt;
    return SGEP_OK;
}

sgep_status sgep_state_size(const sgep_handle *h, size_t *bytes)
{
    if (!h || !bytes)
        return SGEP_EINVAL;
    if (h->wide) {
        const size_t st = (size_t)h->wa.dtot * h->kp * sizeof(float);
        const size_t op = (size_t)h->kp * h->wa.dtot * sizeof(uint16_t);
        *bytes = sizeof(StateHeader) + sizeof(Coef) + st * (h->Am ? 4 : 2) + 2 * op +
                 (size_t)h->wa.Ws * h->wa.lds * sizeof(double);
        return SGEP_OK;
    }
    const size_t st = (size_t)h->ldv * h->kp * h->esz;
    *bytes = sizeof(StateHeader) + sizeof(Coef) + st * (h->Am ? 4 : 2) +
             (size_t)h->W * h->lds * sizeof(double);
    return SGEP_OK;
}

sgep_status sgep_get_state(sgep_handle *h, void *host_buf, size_t bytes)
{
    if (!h || !host_buf)
        return SGEP_EINVAL;
    size_t need = 0;
    sgep_state_size(h, &need);
    if (bytes < need)
        return SGEP_ESHAPE;
    if (h->poisoned)
        return SGEP_EPOISONED;
    sgep_status rc = latch_status(h);
    if (rc != SGEP_OK)
        return rc;
    StateHeader hd = {kStateMagic, kStateVersion, config_hash(h->cfg), h->d, h->kp,
                      (int64_t)h->esz, h->Am ? 1 : 0};
    unsigned char *p = (unsigned char *)host_buf;
    memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    HIPCHK(hipMemcpyAsync(p, h->coef, sizeof(Coef), hipMemcpyDeviceToHost, h->stream));
    p += sizeof(Coef);
    StateLayout L = state_layout(h);
    for (int i = 0; i < L.n; ++i) {
        HIPCHK(hipMemcpyAsync(p, L.ptr[i], L.bytes[i], hipMemcpyDeviceToHost, h->stream));
        p += L.bytes[i];
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return SGEP_OK;
}

sgep_status sgep_set_state(sgep_handle *h, const void *host_buf, size_t bytes)
{
    if (!h || !host_buf)
        return SGEP_EINVAL;
    size_t need = 0;
    sgep_state_size(h, &need);
    if (bytes < need)
        return SGEP_ESHAPE;
    StateHeader hd;
    memcpy(&hd, host_buf, sizeof(hd));
    if (hd.magic != kStateMagic || hd.version != kStateVersion ||
        hd.cfg_hash != config_hash(h->cfg) || hd.d != h->d || hd.kp != h->kp ||
        hd.elem != (int64_t)h->esz || hd.adam != (h->Am ? 1 : 0))
        return SGEP_EINVAL;
    const unsigned char *p = (const unsigned char *)host_buf + sizeof(hd);
    // drain any queued work before overwriting the state it uses
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpyAsync(h->coef, p, sizeof(Coef), hipMemcpyHostToDevice, h->stream));
    p += sizeof(Coef);
    StateLayout L = state_layout(h);
    for (int i = 0; i < L.n; ++i) {
        HIPCHK(hipMemcpyAsync(L.ptr[i], p, L.bytes[i], hipMemcpyHostToDevice, h->stream));
        p += L.bytes[i];
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    int st_word = 0;
    memcpy(&st_word, (const unsigned char *)host_buf + sizeof(hd) + offsetof(Coef, status),
           sizeof(int));
    h->poisoned = st_word != 0;
    return h->poisoned ? SGEP_ENONFINITE : SGEP_OK;
}

sgep_status sgep_destroy(sgep_handle *h)
{
    if (!h)
        return SGEP_EINVAL;
    (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
    return SGEP_OK;
}

} // extern "C"
