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

#include <new>
#include <vector>

#include "../../include/sgep.h"
#include "sgep_kernels.hpp"

using sgep::Coef;
using sgep::StepArgs;

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
    void *ptrs[] = {h->V, h->G, h->Am, h->As, h->P, h->Q, h->gram_part, h->stat_part,
                    h->stat_tot, h->readout, h->coef};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
}

sgep_status check_cfg(const sgep_config *c)
{
    if (!c)
        return SGEP_EINVAL;
    if (c->kind == SGEP_KIND_LDA)
        return SGEP_EUNSUPPORTED;
    if (c->kind != SGEP_KIND_CCA && c->kind != SGEP_KIND_GENERAL)
        return SGEP_EINVAL;
    if (c->dtype == SGEP_BF16 || c->dtype == SGEP_FP8_E4M3)
        return SGEP_EUNSUPPORTED;
    if (c->dtype != SGEP_F64 && c->dtype != SGEP_F32)
        return SGEP_EINVAL;
    if (c->k < 1 || c->k > 64 || (c->dtype == SGEP_F64 && c->k > 32))
        return c->k < 1 ? SGEP_EINVAL : SGEP_EUNSUPPORTED;
    if (c->optimizer != SGEP_SGD && c->optimizer != SGEP_ADAM)
        return SGEP_EINVAL;
    if (c->schedule < SGEP_SCHED_CONST || c->schedule > SGEP_SCHED_WARMUP_HARMONIC)
        return SGEP_EINVAL;
    if (c->dx < 1 || c->dy < 1 || c->b_max < 1)
        return SGEP_ESHAPE;
    if (c->kind == SGEP_KIND_GENERAL && c->dx != c->dy)
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

} // namespace

extern "C" {

int32_t sgep_version(void) { return 100; }

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
    if (!out)
        return SGEP_EINVAL;
    *out = nullptr;
    sgep_status rc = check_cfg(cfg);
    if (rc != SGEP_OK)
        return rc;
    if (!V0)
        return SGEP_EINVAL;
    sgep_handle *h = new (std::nothrow) sgep_handle_s();
    if (!h)
        return SGEP_ENOMEM;
    h->cfg = *cfg;
    h->stream = (hipStream_t)hip_stream;
    h->d = cfg->kind == SGEP_KIND_CCA ? cfg->dx + cfg->dy : cfg->dx;
    h->kp = cfg->k <= 16 ? 16 : (cfg->k <= 32 ? 32 : 64);
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
                             int64_t ldy, int64_t b, void *const *events)
{
    if (!h)
        return SGEP_EINVAL;
    if (h->poisoned)
        return SGEP_EPOISONED;
    if (!X || !Y)
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
    return step_impl(h, X, ldx, Y, ldy, b, nullptr);
}

sgep_status sgep_step_profiled(sgep_handle *h, const void *X, int64_t ldx, const void *Y,
                               int64_t ldy, int64_t b, void *const *events)
{
    if (!events || !events[0] || !events[1] || !events[2] || !events[3])
        return SGEP_EINVAL;
    return step_impl(h, X, ldx, Y, ldy, b, events);
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
    const size_t st = (size_t)h->ldv * h->kp * h->esz;
    HIPCHK(hipMemcpyAsync(p, h->coef, sizeof(Coef), hipMemcpyDeviceToHost, h->stream));
    p += sizeof(Coef);
    void *arrs[] = {h->V, h->G, h->Am, h->As};
    for (void *a : arrs) {
        if (!a)
            continue;
        HIPCHK(hipMemcpyAsync(p, a, st, hipMemcpyDeviceToHost, h->stream));
        p += st;
    }
    HIPCHK(hipMemcpyAsync(p, h->stat_part, (size_t)h->W * h->lds * sizeof(double),
                          hipMemcpyDeviceToHost, h->stream));
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
    const size_t st = (size_t)h->ldv * h->kp * h->esz;
    // drain any queued work before overwriting the state it uses
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpyAsync(h->coef, p, sizeof(Coef), hipMemcpyHostToDevice, h->stream));
    p += sizeof(Coef);
    void *arrs[] = {h->V, h->G, h->Am, h->As};
    for (void *a : arrs) {
        if (!a)
            continue;
        HIPCHK(hipMemcpyAsync(a, p, st, hipMemcpyHostToDevice, h->stream));
        p += st;
    }
    HIPCHK(hipMemcpyAsync(h->stat_part, p, (size_t)h->W * h->lds * sizeof(double),
                          hipMemcpyHostToDevice, h->stream));
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
