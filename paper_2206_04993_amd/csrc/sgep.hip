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

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/sgep.h"
#include "sgep_batch.hpp"
#include "sgep_kernels.hpp"
#include "sgep_wide.hpp"

using sgep::Coef;
using sgep::StepArgs;
using sgep::wide::WideArgs;

namespace {

constexpr uint32_t kStateMagic = 0x53474550u; // "SGEP"
constexpr uint32_t kStateVersion = 2u;

struct StateHeader {
    uint32_t magic, version;
    uint64_t cfg_hash;
    int64_t d, kp;
    int64_t elem;
    int64_t adam;
};

// Read-out staging of sgep_vectors_noalloc: a device array of fixed size
// that every GPU the library runs on holds until the process ends, so that
// read-out allocates nothing.  Its host-side name is not a device address:
// host code uses the per-device address from hipGetSymbolAddress (kept in
// g_scratch) and passes that to kernels and copies.
constexpr size_t kScratchDoubles = (size_t)1 << 22; // 32 MiB: d * k <= 4,194,304
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// The address of this device's scratch array; call with `device` current.
// Looked up once per device (at the first sgep_init on it, else at the
// first sgep_vectors_noalloc).
double *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
            g_scratch[device] = (double *)p;
    }
    return g_scratch[device];
}

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
    void *cpre = nullptr; // coefficient block of the iteration (k_coef)
    int nsplit = 1;        // row slices of the backward products (1: one pass)
    void *mu = nullptr;    // running means of the views (centring): 2 ldv elements (large-d: dtot FP32)
    void *xsum = nullptr;  // large-d split backward with centring: minibatch column sums (dtot FP32)
    void *S1 = nullptr, *S2 = nullptr; // ICA: first backward pass products
    double *bb_part = nullptr;         // ICA: S1^T S1 tile partials
    double *gsum = nullptr; // column totals of the Gram partials (two-stage coefficients)
    bool coef2 = false;     // coefficients in two stages (k_coefa, k_coefb)
    void *bpart = nullptr; // the slices' partial products (nsplit > 1)
    void *fpart = nullptr; // per-view forward: stamped words of P (nsplit > 1)
    size_t fpart_bytes = 0;
    bool fused = false;    // row split without a finishing pass (no centring)
    void *xw = nullptr;    // fused row split: stamped words (slices' products, coefficient block)
    size_t xw_bytes = 0;
    int64_t xw_coef = 0;   // word offset of the coefficient block in xw
    unsigned long long *cflag = nullptr; // fused row split: iteration of the published block
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
    void *Vf = nullptr, *Wf = nullptr; // FP32 input: V operand and W rows
    void *prod = nullptr, *ctile = nullptr; // split backward: products, coefficient tile
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
    const int32_t ints[] = {c.kind,      c.dtype,    c.k,      c.optimizer,
                            c.schedule,  c.n_classes, c.smooth, c.center};
    const int64_t dims[] = {c.dx, c.dy, c.b_max};
    const double reals[] = {c.eta0, c.eta_T, c.t0, c.t_c, c.T, c.gamma, c.rho, c.eps_reg,
                            c.adam_b1, c.adam_b2, c.adam_eps, c.smooth ? c.nu : 0.0};
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
                    h->Ppart, h->Wh, h->Wl, h->Mcls, h->Mbar, h->prior, h->cpre, h->bpart,
                    h->mu,   h->S1, h->S2,     h->bb_part, h->gsum, h->fpart,
                    h->xw, h->cflag, h->Vf, h->Wf, h->prod, h->ctile, h->xsum};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
}

sgep_status check_cfg(const sgep_config *c)
{
    if (!c)
        return SGEP_EINVAL;
    if (c->kind != SGEP_KIND_CCA && c->kind != SGEP_KIND_GENERAL && c->kind != SGEP_KIND_LDA &&
        c->kind != SGEP_KIND_ICA)
        return SGEP_EINVAL;
    if (c->dtype < SGEP_F64 || c->dtype > SGEP_FP8_E4M3)
        return SGEP_EINVAL;
    const bool narrow = c->dtype == SGEP_BF16 || c->dtype == SGEP_FP8_E4M3;
    const bool lda = c->kind == SGEP_KIND_LDA;
    // LDA runs on the large-d path in BF16 or FP32; GENERAL and ICA on the
    // F64 / F32 path only
    const bool ica = c->kind == SGEP_KIND_ICA;
    if ((lda && c->dtype != SGEP_BF16 && c->dtype != SGEP_F32) ||
        (narrow && (c->kind == SGEP_KIND_GENERAL || ica)))
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
    } else if (ica) {
        if (c->n_classes != 0)
            return SGEP_EINVAL;
        if (c->dx < 1 || c->dy != 0 || c->b_max < 1)
            return SGEP_ESHAPE;
    } else if (c->dx < 1 || c->dy < 1 || c->b_max < 1) {
        return SGEP_ESHAPE;
    }
    if (c->kind == SGEP_KIND_GENERAL && c->dx != c->dy)
        return SGEP_ESHAPE;
    if ((narrow || lda) && (c->dx % 8 != 0 || c->dy % 8 != 0))
        return SGEP_ESHAPE;
    const int64_t d = c->kind == SGEP_KIND_CCA ? c->dx + c->dy : c->dx;
    if (c->k > d)
        return SGEP_ESHAPE;
    // partial reductions are sized for at most 2^19 rows / features
    if (c->b_max > (int64_t)1 << 19 || d > (int64_t)1 << 19)
        return SGEP_EUNSUPPORTED;
    if (!(c->eta0 >= 0.0) || !(c->gamma > 0.0 && c->gamma <= 1.0) || !(c->rho >= 0.0))
        return SGEP_EINVAL;
    if ((c->smooth != 0 && c->smooth != 1) || (c->center != 0 && c->center != 1))
        return SGEP_EINVAL;
    if (c->center && (lda || ica || (narrow && c->kind != SGEP_KIND_CCA)))
        return SGEP_EUNSUPPORTED; // centring: F64 / F32 CCA and GENERAL, BF16 / FP8 CCA
    if (c->smooth && !(c->rho > 0.0 && c->nu > c->rho && std::isfinite(c->nu)))
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
                  const StepArgs &a, int threads = sgep::kNT)
{
    if (e0)
        hipExtLaunchKernelGGL(kernel, grid, dim3(threads), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(kernel, grid, dim3(threads), 0, s, a);
}

// The backward mode of a single handle: four helper waves compute the
// coefficients during the main loop when the tile is one 16-feature block
// and the player tile small enough for eight waves' registers; otherwise
// k_coef computes them once per iteration.
template <typename T> bool spec_mode(int kp, int mb) { return mb == 1 && kp * (int)sizeof(T) <= 128; }

// Row-split backward (CCA, one 16-feature tile per workgroup): with few tiles
// and long minibatches one workgroup per tile leaves most CUs idle; two row
// slices per tile (k_bwdp, with the coefficient block on one more
// workgroup), then a finishing pass per tile.  Measured at d = 512 + 512,
// k = 16, b = 1024 (64 tiles): 2 slices ~1 us per step faster than the
// single pass with helper waves; 4 and 8 slices slower (the extra launch
// and the partials' round trip outweigh the shorter main loop).  GENERAL
// handles keep one pass, so that an instance of a batch matches its single
// handle bit for bit.  The split launches wait inside the kernel (k_fwds: the
// y workgroup of a row tile on the x workgroup's stamped P words; the fused
// k_bwdp: the last slice of a tile on the other slices and on workgroup 0's
// coefficient words), so every workgroup of a launch must be resident at
// once: the bounds below keep k_fwds within 2 * 128 + 1 workgroups (b_max <=
// 2048) and k_bwdp within 2 * 128 + 8 (at most 128 feature tiles), while
// the 256 CUs hold at least two workgroups of either kernel each.  Every
// wait is bounded besides (a give-up sets the status word).
constexpr int kSplit = 2;
bool split_mode(const sgep_config &c, int mb, int n_tiles)
{
    return c.kind == SGEP_KIND_CCA && mb == 1 && n_tiles <= 128 && c.b_max >= 512 &&
           c.b_max <= 2048;
}

template <typename T, int KP, int MB, int MODE, bool C>
void launch_bwd(sgep_handle *h, const StepArgs &a, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 gb(h->n_tiles);
    const bool cca = h->cfg.kind == SGEP_KIND_CCA;
    const bool adam = h->cfg.optimizer == SGEP_ADAM;
    const int nt = MODE == sgep::kModeSpec ? 2 * sgep::kNT : sgep::kNT;
    using namespace sgep;
    if (cca && !adam)
        launch_timed(k_bwd<T, KP, MB, kKindCCA, kOptSGD, MODE, C>, gb, h->stream, e0, e1, a, nt);
    else if (cca && adam)
        launch_timed(k_bwd<T, KP, MB, kKindCCA, kOptAdam, MODE, C>, gb, h->stream, e0, e1, a, nt);
    else if (!adam)
        launch_timed(k_bwd<T, KP, MB, kKindGeneral, kOptSGD, MODE, C>, gb, h->stream, e0, e1, a,
                     nt);
    else
        launch_timed(k_bwd<T, KP, MB, kKindGeneral, kOptAdam, MODE, C>, gb, h->stream, e0, e1, a,
                     nt);
}

int narrow_kernels(const sgep_handle *h);
// kernels of one iteration of a large-d handle: forward, middle pass and the
// backward in one kernel, or split into products and epilogue
int wide_kernels(const sgep_handle *h) { return h->wa.ft == sgep::wide::kFT ? 3 : 4; }

// one iteration; C: the views are centred by their running means
template <typename T, int KP, bool C>
sgep_status launch_step_c(sgep_handle *h, const StepArgs &a, void *const *events)
{
    const dim3 gf(a.n_fwd + 1); // + the norm-totals workgroup
    hipEvent_t ev[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    const bool split = h->nsplit > 1;
    const bool spec = !split && spec_mode<T>(KP, h->mb);
    if (events)
        for (int i = 0; i < 2 * narrow_kernels(h); ++i)
            ev[i] = (hipEvent_t)events[i];
    const bool cca = h->cfg.kind == SGEP_KIND_CCA;
    if (split) // CCA only: several workgroups per row tile
        launch_timed(sgep::k_fwds<T, KP, C>, dim3(2 * a.n_fwd + 1), h->stream, ev[0], ev[1], a);
    else if (cca)
        launch_timed(sgep::k_fwd<T, KP, sgep::kKindCCA, C>, gf, h->stream, ev[0], ev[1], a);
    else
        launch_timed(sgep::k_fwd<T, KP, sgep::kKindGeneral, C>, gf, h->stream, ev[0], ev[1], a);
    constexpr int MBW = mb_wide<T>(KP);
    constexpr bool can_spec = KP * (int)sizeof(T) <= 128; // spec_mode's player-tile bound
    if (split && h->fused) { // CCA without centring
        const dim3 gp(h->n_tiles * h->nsplit + 8);
        if (h->cfg.optimizer == SGEP_ADAM)
            launch_timed(sgep::k_bwdp<T, KP, sgep::kKindCCA, false, true, sgep::kOptAdam>, gp,
                         h->stream, ev[2], ev[3], a);
        else
            launch_timed(sgep::k_bwdp<T, KP, sgep::kKindCCA, false, true, sgep::kOptSGD>, gp,
                         h->stream, ev[2], ev[3], a);
    } else if (split) {
        const dim3 gp(h->n_tiles * h->nsplit + 8); // + the coefficient workgroup and 7 idle
        if (cca)
            launch_timed(sgep::k_bwdp<T, KP, sgep::kKindCCA, C>, gp, h->stream, ev[2], ev[3], a);
        else
            launch_timed(sgep::k_bwdp<T, KP, sgep::kKindGeneral, C>, gp, h->stream, ev[2], ev[3],
                         a);
        launch_bwd<T, KP, 1, sgep::kModeFin, C>(h, a, ev[4], ev[5]);
    } else if (spec) {
        if constexpr (can_spec)
            launch_bwd<T, KP, 1, sgep::kModeSpec, C>(h, a, ev[2], ev[3]);
    } else {
        int e = 2; // next event pair
        if (h->coef2) {
            const int W = KP * (KP + 1) / 2 + KP;
            launch_timed(sgep::k_coefa<KP>, dim3((W + sgep::kCoefCols - 1) / sgep::kCoefCols),
                         h->stream, ev[2], ev[3], a, 64);
            if (cca)
                launch_timed(sgep::k_coefb<T, KP, sgep::kKindCCA>, dim3(1), h->stream, ev[4],
                             ev[5], a);
            else
                launch_timed(sgep::k_coefb<T, KP, sgep::kKindGeneral>, dim3(1), h->stream, ev[4],
                             ev[5], a);
            e = 6;
        } else if (cca) {
            launch_timed(sgep::k_coef<T, KP, sgep::kKindCCA>, dim3(1), h->stream, ev[2], ev[3], a);
            e = 4;
        } else {
            launch_timed(sgep::k_coef<T, KP, sgep::kKindGeneral>, dim3(1), h->stream, ev[2], ev[3],
                         a);
            e = 4;
        }
        if (h->mb == 1)
            launch_bwd<T, KP, 1, sgep::kModePre, C>(h, a, ev[e], ev[e + 1]);
        else
            launch_bwd<T, KP, MBW, sgep::kModePre, C>(h, a, ev[e], ev[e + 1]);
    }
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

// ICA: forward (P, Q = diag(||x_r||^2) P, Grams), first backward pass (S1 =
// X^T P, S2 = X^T Q, S1^T S1 partials), second forward pass (R = X S1 / b and
// the coefficient block), second backward pass (X^T R, update)
template <typename T, int KP>
sgep_status launch_step_ica(sgep_handle *h, const StepArgs &a, void *const *events)
{
    using namespace sgep;
    hipEvent_t ev[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (events)
        for (int i = 0; i < 8; ++i)
            ev[i] = (hipEvent_t)events[i];
    const dim3 gf(a.n_fwd + 1), gb(h->n_tiles);
    launch_timed(k_fwd<T, KP, kKindICA>, gf, h->stream, ev[0], ev[1], a);
    launch_timed(k_bwd<T, KP, 1, kKindICA, kOptSGD, kModeIca1>, gb, h->stream, ev[2], ev[3], a);
    launch_timed(k_fwd2<T, KP>, gf, h->stream, ev[4], ev[5], a);
    if (h->cfg.optimizer == SGEP_ADAM)
        launch_timed(k_bwd<T, KP, 1, kKindICA, kOptAdam, kModeIca2>, gb, h->stream, ev[6], ev[7],
                     a);
    else
        launch_timed(k_bwd<T, KP, 1, kKindICA, kOptSGD, kModeIca2>, gb, h->stream, ev[6], ev[7],
                     a);
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

template <typename T, int KP>
sgep_status launch_step(sgep_handle *h, const StepArgs &a, void *const *events)
{
    if (h->cfg.kind == SGEP_KIND_ICA)
        return launch_step_ica<T, KP>(h, a, events);
    return h->cfg.center ? launch_step_c<T, KP, true>(h, a, events)
                         : launch_step_c<T, KP, false>(h, a, events);
}

// kernels of one iteration of a narrow handle
int narrow_kernels(const sgep_handle *h)
{
    if (h->cfg.kind == SGEP_KIND_ICA)
        return 4;
    const bool spec = h->esz == sizeof(double) ? spec_mode<double>(h->kp, h->mb)
                                               : spec_mode<float>(h->kp, h->mb);
    if ((spec && h->nsplit == 1) || h->fused)
        return 2;
    return (h->nsplit == 1 && h->coef2) ? 4 : 3;
}

template <typename T, int KP>
sgep_status launch_readout(sgep_handle *h, const void *S, int mode, double *dst)
{
    const int64_t dx = h->cfg.kind == SGEP_KIND_CCA ? h->cfg.dx : h->d;
    hipLaunchKernelGGL((sgep::k_readout<T, KP>), dim3(1), dim3(sgep::kNT), 0, h->stream,
                       (const T *)S, h->d, dx, h->dxp, h->ldv, h->cfg.k, h->stat_part, h->n_tiles,
                       h->lds, h->cfg.rho, h->coef, mode, dst);
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

// bytes of the statistics partials: groups of 16 statistics x lds columns
static size_t wide_stat_part_bytes(const WideArgs &a)
{
    return (size_t)wide_stat_blocks(a) * sgep::wide::kStatCols * a.lds * sizeof(double);
}

template <int KP, int IN, int KIND>
sgep_status wide_step_t(sgep_handle *h, const WideArgs &a, const hipEvent_t *ev)
{
    using namespace sgep::wide;
    const dim3 blk(kWT);
    const bool adam = h->cfg.optimizer == SGEP_ADAM;
    // forward workgroups, then the statistics reductions
    const dim3 gf(a.n_rb * a.nview * a.n_split + wide_stat_blocks(a));
    auto forward = [&]() {
        if constexpr (IN != kInF32) {
            if constexpr (KP == 32 || KP == 64) {
                if (a.rbf == kFwdVRows) { // V shared through LDS (k_wfwdv)
                    launch_k(k_wfwdv<KP, IN>, gf, dim3(512), h->stream, ev[0], ev[1], a);
                    return;
                }
            }
            if (a.rbf == fwd4_rows<KP>()) { // four waves (k_wfwd4)
                launch_k(k_wfwd4<KP, IN>, gf, dim3(256), h->stream, ev[0], ev[1], a);
                return;
            }
            if constexpr (KP <= 32) {
                if (a.rbf == 128) {
                    launch_k(k_wfwd<KP, IN, 128>, gf, blk, h->stream, ev[0], ev[1], a);
                    return;
                }
            }
        }
        launch_k(k_wfwd<KP, IN, 64>, gf, blk, h->stream, ev[0], ev[1], a);
    };
    forward();
    launch_k(k_wmid<KP, IN, KIND>, dim3(a.nA), dim3(kMT), h->stream, ev[2], ev[3], a);
    const dim3 bblk(kBT);
    constexpr bool can128 = IN != kInF32; // 128-feature subtiles: BF16 / FP8 only
    if (can128 && a.ft == 2 * kFT) {
        if constexpr (can128) { // products, then the epilogue per 64-feature tile
            launch_k(k_wprod<KP, IN, KIND>, dim3(a.nwg), bblk, h->stream, ev[4], ev[5], a);
            if (adam)
                launch_k(k_wepi<KP, IN, KIND, sgep::kOptAdam>, dim3(a.nstat), bblk, h->stream,
                         ev[6], ev[7], a);
            else
                launch_k(k_wepi<KP, IN, KIND, sgep::kOptSGD>, dim3(a.nstat), bblk, h->stream,
                         ev[6], ev[7], a);
        }
    } else if (adam) {
        launch_k(k_wbwd<KP, IN, KIND, sgep::kOptAdam>, dim3(a.nwg), bblk, h->stream, ev[4], ev[5], a);
    } else {
        launch_k(k_wbwd<KP, IN, KIND, sgep::kOptSGD>, dim3(a.nwg), bblk, h->stream, ev[4], ev[5], a);
    }
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

// reduce the latest statistics, then scale the state rows into dst
template <int KP, int IN, int KIND>
sgep_status wide_readout_t(sgep_handle *h, const WideArgs &a, const void *S, int mode,
                           double *dst)
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
                       h->cfg.rho, h->coef, mode, dst);
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

// dispatch on (input format, kind, KP) for the BF16 / FP8 path
#define WIDE_DISPATCH(h, FN, ...)                                                          \
    ([&]() -> sgep_status {                                                                \
        using namespace sgep::wide;                                                        \
        if ((h)->cfg.kind == SGEP_KIND_LDA && (h)->cfg.dtype == SGEP_F32) {                \
            if ((h)->kp == 16) return FN<16, kInF32, kKindLDA>(__VA_ARGS__);               \
            if ((h)->kp == 32) return FN<32, kInF32, kKindLDA>(__VA_ARGS__);               \
            if ((h)->kp == 64) return FN<64, kInF32, kKindLDA>(__VA_ARGS__);               \
        } else if ((h)->cfg.kind == SGEP_KIND_LDA) {                                       \
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
        if (st & sgep::kStatusSync)
            return SGEP_EDEVICE;
        if (st & sgep::wide::kStatusBadLabel)
            return SGEP_ELABEL;
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
    const bool f32 = c.dtype == SGEP_F32;
    const int64_t KP = h->kp, d = h->d;
    WideArgs &a = h->wa;
    memset(&a, 0, sizeof(a));
    // backward subtiles of 128 features where the views keep >= 256 of them
    // (one per workgroup): fewer W loads per byte of X; else 64
    {
        const int64_t n128 = (c.dx + 127) / 128 + (lda ? 0 : (c.dy + 127) / 128);
        a.ft = (!f32 && n128 >= 256) ? 2 * kFT : kFT;
    }
    const int64_t ft = a.ft;
    auto r64 = [ft](int64_t x) { return (x + ft - 1) / ft * ft; }; // views padded to subtiles
    h->esz = fp8 ? 1 : (f32 ? 4 : 2); // element size of the minibatch (checkpoint header)
    a.nview = lda ? 1 : 2;
    a.dv[0] = c.dx;
    a.dv[1] = lda ? 0 : c.dy;
    a.off[0] = 0;
    a.off[1] = r64(c.dx);
    a.dtot = lda ? r64(c.dx) : r64(c.dx) + r64(c.dy);
    a.k = c.k;
    a.ncls = lda ? c.n_classes : 0;
    // forward kernels: KP = 32 or 64 BF16 / FP8 minibatches of >= 1024 rows take
    // k_wfwdv (512-row workgroups sharing the V operand through LDS, rows
    // padded to 512); other BF16 / FP8 minibatches of >= 256 rows the
    // four-wave k_wfwd4 (rows padded to 256); the rest k_wfwd
    const bool fwdv = (KP == 32 || KP == 64) && !f32 && c.b_max >= 1024;
    const bool fwd4 = !fwdv && !f32 && c.b_max >= 256;
    const int64_t rowpad = fwdv ? kFwdVRows : (fwd4 ? 256 : kRowPad);
    a.ldr = (c.b_max + rowpad - 1) / rowpad * rowpad;
    // k_wfwd: aim at >= 512 workgroups of 64 rows at b_max (the same number of
    // rows in flight with 128-row blocks), each wave >= one 64-feature step;
    // 128-row blocks when they still give >= 256 workgroups.  k_wfwd4: 512
    // workgroups; k_wfwdv: 256 (one per CU: each slice's partial costs 512
    // rows x KP of memory traffic)
    const int64_t dvmax = a.dv[0] > a.dv[1] ? a.dv[0] : a.dv[1];
    const int64_t nf64 = (dvmax + 63) / 64;
    const int64_t ns_cap = (nf64 + kNW - 1) / kNW;
    a.rbf = fwdv ? kFwdVRows
                 : (fwd4 ? (KP <= 32 ? 256 : 128)
                         : ((KP <= 32 && !f32 && (a.ldr / 128) * a.nview * ns_cap >= 256) ? 128 : 64));
    const int64_t rbf = a.rbf;
    // feature ranges per forward workgroup (k_wfwdv: one, shared by its waves)
    const int64_t nwv = fwdv ? 1 : (fwd4 ? 4 : kNW);
    const int64_t nrb = a.ldr / rbf;
    const int64_t target = fwdv ? 256 : (fwd4 ? 512 : 512 * kRB / rbf); // forward workgroups
    int64_t ns = (target + nrb * a.nview - 1) / (nrb * a.nview);
    const int64_t ns_max = (nf64 + nwv - 1) / nwv;
    if (ns > ns_max)
        ns = ns_max;
    if (ns < 1)
        ns = 1;
    a.fw = 64 * ((nf64 + nwv * ns - 1) / (nwv * ns));
    a.fs = nwv * a.fw;
    a.n_split = (int32_t)((dvmax + a.fs - 1) / a.fs);
    // backward: subtiles of ft features, about 256 workgroups (64-feature
    // subtiles) or one 128-feature subtile per workgroup
    a.nsubv[0] = (int32_t)((a.dv[0] + ft - 1) / ft);
    a.nsubv[1] = (int32_t)((a.dv[1] + ft - 1) / ft);
    const int nsubt = a.nsubv[0] + a.nsubv[1];
    a.nsub = (ft == kFT && nsubt / 256 > 1) ? nsubt / 256 : 1;
    a.nwg0 = (a.nsubv[0] + a.nsub - 1) / a.nsub;
    a.nwg = a.nwg0 + (a.nsubv[1] + a.nsub - 1) / a.nsub;
    // statistics partials: one column per backward workgroup, or per epilogue
    // workgroup (64-feature tile) of the split backward
    a.nstat = ft == kFT ? a.nwg : (int32_t)(nsubt * (ft / kFT));
    a.lds = (a.nstat + 1) / 2 * 2;
    // statistics: v_i^T G_j (lower triangle), ||v_i||^2, then LDA the class
    // means times v_i, CCA each view's running mean times v_i (centring)
    a.Ws = (int32_t)(KP * (KP + 1) / 2 + KP + (lda ? a.ncls * KP : 2 * KP));
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
    const size_t wbytes = (size_t)MW * a.ldr * sizeof(uint16_t); // FP32 input: twice this
    const size_t spb = wide_stat_part_bytes(a);
    alloc(&h->V, st);
    alloc(&h->G, st);
    if (c.optimizer == SGEP_ADAM) {
        alloc(&h->Am, st);
        alloc(&h->As, st);
    }
    if (f32) {
        alloc(&h->Vf, 2 * op);
    } else {
        alloc(&h->Vh, op);
        alloc(&h->Vl, op);
    }
    if (fp8)
        alloc(&h->colscale, (size_t)a.dtot * sizeof(float));
    alloc(&h->Ppart, (size_t)a.n_split * a.nview * a.ldr * KP * sizeof(float));
    if (f32) {
        alloc(&h->Wf, 2 * wbytes);
    } else {
        alloc(&h->Wh, wbytes);
        alloc(&h->Wl, wbytes);
    }
    if (ft != kFT) {
        const int64_t mwa = lda ? KP : 2 * KP; // rows of W in the products
        alloc(&h->prod, (size_t)a.dtot * mwa * sizeof(float));
        alloc(&h->ctile, (size_t)(KP * KP + 4 * KP + 2 * kMaxCls * KP) * sizeof(float));
        if (c.center)
            alloc(&h->xsum, (size_t)a.dtot * sizeof(float));
    }
    if (c.center)
        alloc(&h->mu, (size_t)a.dtot * sizeof(float));
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
    a.Vf = (float *)h->Vf;
    a.colscale = (const float *)h->colscale;
    a.Ppart = (float *)h->Ppart;
    a.Wh = (uint16_t *)h->Wh;
    a.Wl = (uint16_t *)h->Wl;
    a.Wf = (float *)h->Wf;
    a.prod = (float *)h->prod;
    a.ctile = (float *)h->ctile;
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
    a.smooth = c.smooth;
    a.lrho = c.smooth ? log(c.rho) : 0.0;
    a.lspan = c.smooth ? log(c.nu) - log(c.rho) : 0.0;
    a.eps_reg = c.eps_reg;
    a.adam_b1 = c.adam_b1;
    a.adam_b2 = c.adam_b2;
    a.adam_eps = c.adam_eps;
    a.center = c.center;
    a.mu = (float *)h->mu;
    a.xsum = (float *)h->xsum;

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
               hipMemcpyAsync(h->V, hv.data(), st, hipMemcpyHostToDevice, h->stream) == hipSuccess;
    // operand copies and W rows (rows past the minibatch must read as zero)
    if (f32)
        hok = hok && hipMemsetAsync(h->Vf, 0, 2 * op, h->stream) == hipSuccess &&
              hipMemsetAsync(h->Wf, 0, 2 * wbytes, h->stream) == hipSuccess;
    else
        hok = hok && hipMemsetAsync(h->Vh, 0, op, h->stream) == hipSuccess &&
              hipMemsetAsync(h->Vl, 0, op, h->stream) == hipSuccess &&
              hipMemsetAsync(h->Wh, 0, wbytes, h->stream) == hipSuccess &&
              hipMemsetAsync(h->Wl, 0, wbytes, h->stream) == hipSuccess;
    if (h->Am)
        hok = hok && hipMemsetAsync(h->Am, 0, st, h->stream) == hipSuccess &&
              hipMemsetAsync(h->As, 0, st, h->stream) == hipSuccess;
    if (h->mu) // the running means start at zero
        hok = hok && hipMemsetAsync(h->mu, 0, (size_t)a.dtot * sizeof(float), h->stream) == hipSuccess;
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
    a.n_rb = (int32_t)((b + a.rbf - 1) / a.rbf);
    a.nA = (sgep::wide::kRB / sgep::wide::kMR) * (int32_t)((b + sgep::wide::kRB - 1) / sgep::wide::kRB);
    hipEvent_t ev[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (events)
        for (int i = 0; i < 2 * wide_kernels(h); ++i)
            ev[i] = (hipEvent_t)events[i];
    return WIDE_DISPATCH(h, wide_step_t, h, a, ev);
}

// device arrays of a checkpoint after the header and the coefficient block
struct StateLayout {
    int n = 0;
    void *ptr[10];
    size_t bytes[10];
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
        L.add(h->Vf, 2 * op); // FP32 input: in place of Vh, Vl
        L.add(h->stat_part, wide_stat_part_bytes(h->wa));
        L.add(h->mu, (size_t)h->wa.dtot * sizeof(float)); // centring: running means
    } else {
        const size_t st = (size_t)h->ldv * h->kp * h->esz;
        L.add(h->V, st);
        L.add(h->G, st);
        L.add(h->Am, st);
        L.add(h->As, st);
        L.add(h->stat_part, (size_t)h->W * h->lds * sizeof(double));
        L.add(h->mu, (size_t)2 * h->ldv * h->esz);
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
    case SGEP_EUNSUPPORTED: return "not supported by the library";
    case SGEP_EPOISONED: return "handle poisoned by an earlier fault";
    case SGEP_ELABEL: return "LDA label outside [0, n_classes) in a step";
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
    {
        int dev = 0; // the current device: the no-allocation read-out's staging
        if (hipGetDevice(&dev) == hipSuccess)
            (void)scratch_of(dev);
    }
    if (cfg->dtype == SGEP_BF16 || cfg->dtype == SGEP_FP8_E4M3 || cfg->kind == SGEP_KIND_LDA) {
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
    h->mb = (!wide || cfg->kind == SGEP_KIND_ICA)
                ? 1
                : (cfg->dtype == SGEP_F64 ? mb_wide<double>(h->kp) : mb_wide<float>(h->kp));
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
    const bool ica = cfg->kind == SGEP_KIND_ICA;
    const int64_t tri = (int64_t)kp * (kp + 1) / 2;
    // ICA Gram rows: P^T diag(n) P and P^T P (lower triangles) and sum_r n_r
    const int64_t wg = ica ? 2 * tri + 1 : h->W;
    alloc((void **)&h->gram_part, (size_t)wg * h->ldg * sizeof(double));
    alloc((void **)&h->stat_part, (size_t)h->W * h->lds * sizeof(double));
    alloc((void **)&h->stat_tot, (size_t)h->W * sizeof(double));
    alloc((void **)&h->readout, (size_t)d * cfg->k * sizeof(double));
    alloc((void **)&h->coef, sizeof(Coef));
    alloc(&h->cpre, (size_t)(kp * kp + 3 * kp + 4) * h->esz);
    if (split_mode(*cfg, h->mb, h->n_tiles)) {
        h->nsplit = kSplit;
        alloc(&h->bpart, (size_t)h->n_tiles * kSplit * (2 * h->ft * kp + 2 * h->ft) * h->esz);
        // the per-view forward's stamped words of P (two per FP64 value)
        h->fpart_bytes = (size_t)h->fwd_blocks_max * 16 * kp * (h->esz / 4) * 8;
        alloc(&h->fpart, h->fpart_bytes);
        // iteration stamp of the coefficient block (also the forward's stamp base)
        alloc((void **)&h->cflag, sizeof(unsigned long long));
        // without centring the last slice of each tile runs the epilogue
        h->fused = !cfg->center;
        if (h->fused) {
            const int64_t nw = h->esz / 4; // words per value
            h->xw_coef = (int64_t)h->n_tiles * kSplit * 2 * h->ft * kp * nw;
            h->xw_bytes = (size_t)(h->xw_coef + (kp * kp + 3 * kp + 4) * nw) * 8;
            alloc(&h->xw, h->xw_bytes);
        }
    }
    if (cfg->center)
        alloc(&h->mu, (size_t)2 * h->ldv * h->esz);
    alloc((void **)&h->gsum, (size_t)h->W * sizeof(double));
    // many Gram partials: sum their columns over many workgroups first
    h->coef2 = !ica && h->fwd_blocks_max * h->W >= 32768;
    if (ica) {
        alloc(&h->S1, st_bytes);
        alloc(&h->S2, st_bytes);
        alloc((void **)&h->bb_part, (size_t)tri * h->lds * sizeof(double));
    }
    if (!ok) {
        free_all(h);
        delete h;
        return SGEP_ENOMEM;
    }
    // zero state, then upload the raw starting points (padding columns zero)
    bool hok = hipMemsetAsync(h->coef, 0, sizeof(Coef), h->stream) == hipSuccess &&
               hipMemsetAsync(h->stat_part, 0, (size_t)h->W * h->lds * sizeof(double),
                              h->stream) == hipSuccess &&
               hipMemsetAsync(h->gram_part, 0, (size_t)wg * h->ldg * sizeof(double),
                              h->stream) == hipSuccess;
    if (h->Am)
        hok = hok && hipMemsetAsync(h->Am, 0, st_bytes, h->stream) == hipSuccess &&
              hipMemsetAsync(h->As, 0, st_bytes, h->stream) == hipSuccess;
    if (h->mu)
        hok = hok && hipMemsetAsync(h->mu, 0, (size_t)2 * h->ldv * h->esz, h->stream) == hipSuccess;
    if (h->fpart) // stamps are at least 1: zero words never match
        hok = hok && hipMemsetAsync(h->fpart, 0, h->fpart_bytes, h->stream) == hipSuccess &&
              hipMemsetAsync(h->cflag, 0, sizeof(unsigned long long), h->stream) == hipSuccess;
    if (h->xw)
        hok = hok && hipMemsetAsync(h->xw, 0, h->xw_bytes, h->stream) == hipSuccess;
    if (h->S1) // features past d are never written and must read as zero
        hok = hok && hipMemsetAsync(h->S1, 0, st_bytes, h->stream) == hipSuccess &&
              hipMemsetAsync(h->S2, 0, st_bytes, h->stream) == hipSuccess;
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

// Arguments of one iteration of the narrow path that do not depend on the
// minibatch itself (X, Y, b and n_fwd are left zero).
static StepArgs make_args(const sgep_handle *h, int64_t ldx, int64_t ldy, bool vec_ok)
{
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.ldx = ldx;
    a.ldy = ldy;
    a.dx = h->cfg.dx;
    a.dy = h->cfg.dy;
    a.dxp = h->dxp;
    a.ldv = h->ldv;
    a.ldp = h->ldp;
    a.k = h->cfg.k;
    a.n_tx = h->n_tx;
    a.n_ty = h->n_ty;
    a.vec_ok = vec_ok ? 1 : 0;
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
    a.cpre = h->cpre;
    a.bpart = h->bpart;
    a.fpart = h->fpart;
    a.xw = h->xw;
    a.xw_coef = h->xw_coef;
    a.cflag = h->cflag;
    a.mu = h->mu;
    a.S1 = h->S1;
    a.S2 = h->S2;
    a.bb_part = h->bb_part;
    a.gsum = h->gsum;
    a.nsplit = h->nsplit;
    a.schedule = h->cfg.schedule;
    a.eta0 = h->cfg.eta0;
    a.eta_T = h->cfg.eta_T;
    a.t0 = h->cfg.t0;
    a.t_c = h->cfg.t_c;
    a.T = h->cfg.T;
    a.gamma = h->cfg.gamma;
    a.rho = h->cfg.rho;
    a.smooth = h->cfg.smooth;
    a.lrho = h->cfg.smooth ? log(h->cfg.rho) : 0.0;
    a.lspan = h->cfg.smooth ? log(h->cfg.nu) - log(h->cfg.rho) : 0.0;
    a.eps_reg = h->cfg.eps_reg;
    a.adam_b1 = h->cfg.adam_b1;
    a.adam_b2 = h->cfg.adam_b2;
    a.adam_eps = h->cfg.adam_eps;
    return a;
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
    const bool ica = h->cfg.kind == SGEP_KIND_ICA;
    if (!X || labels || (ica ? Y != nullptr : !Y))
        return SGEP_EINVAL;
    if (ica) { // one stream: the second view's slots point at it
        Y = X;
        ldy = ldx;
    }
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
    StepArgs a = make_args(h, ldx, ldy, vec_ok);
    a.X = X;
    a.Y = Y;
    a.b = b;
    a.n_fwd = (int32_t)((b + 15) / 16);
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
    *n = h->wide ? wide_kernels(h) : narrow_kernels(h);
    return SGEP_OK;
}

const char *sgep_step_kernel_name(const sgep_handle *h, int32_t i)
{
    if (!h || i < 0)
        return nullptr;
    static const char *wide[] = {"k_wfwd", "k_wmid", "k_wbwd"};
    static const char *wide4[] = {"k_wfwd", "k_wmid", "k_wprod", "k_wepi"};
    static const char *spec[] = {"k_fwd", "k_bwd"};
    static const char *pre[] = {"k_fwd", "k_coef", "k_bwd"};
    static const char *split[] = {"k_fwds", "k_bwdp", "k_bwd"};
    static const char *fused[] = {"k_fwds", "k_bwdp"};
    static const char *ica[] = {"k_fwd", "k_bwd1", "k_fwd2", "k_bwd"};
    static const char *pre2[] = {"k_fwd", "k_coefa", "k_coefb", "k_bwd"};
    if (h->wide) {
        if (h->wa.ft != sgep::wide::kFT)
            return i < 4 ? wide4[i] : nullptr;
        return i < 3 ? wide[i] : nullptr;
    }
    const int n = narrow_kernels(h);
    if (i >= n)
        return nullptr;
    if (h->cfg.kind == SGEP_KIND_ICA)
        return ica[i];
    if (n == 4)
        return pre2[i];
    if (h->fused)
        return fused[i];
    return n == 2 ? spec[i] : (h->nsplit > 1 ? split[i] : pre[i]);
}

sgep_status sgep_step_profiled(sgep_handle *h, const void *X, int64_t ldx, const void *Y,
                               int64_t ldy, const int32_t *labels, int64_t b,
                               void *const *events, int32_t n_events)
{
    if (!h || !events)
        return SGEP_EINVAL;
    const int32_t need = 2 * (h->wide ? wide_kernels(h) : narrow_kernels(h));
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

// The state rows S scaled per player (mode 0: as stored, 1: unit, 2:
// B-normalised), staged as FP64 d x k column-major in dst (device), signs
// canonicalised when canon is set, then copied to the host array out.
static sgep_status readout(sgep_handle *h, const void *S, int mode, bool canon, double *dst,
                           double *out)
{
    if (!h || !out)
        return SGEP_EINVAL;
    if (h->poisoned)
        return SGEP_EPOISONED;
    sgep_status rc = latch_status(h);
    if (rc != SGEP_OK)
        return rc;
    if (h->wide)
        rc = WIDE_DISPATCH(h, wide_readout_t, h, h->wa, S, mode, dst);
    else
        rc = SGEP_DISPATCH(h, launch_readout, h, S, mode, dst);
    if (rc != SGEP_OK)
        return rc;
    if (canon) {
        hipLaunchKernelGGL(sgep::k_canon, dim3(h->cfg.k), dim3(sgep::kNT), 0, h->stream, dst,
                           h->d);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(out, dst, (size_t)h->d * h->cfg.k * sizeof(double),
                          hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return SGEP_OK;
}

sgep_status sgep_vectors(sgep_handle *h, int32_t flags, double *out)
{
    if (!h || (flags & ~(SGEP_VEC_BNORM | SGEP_VEC_CANONICAL)) != 0)
        return SGEP_EINVAL;
    return readout(h, h->V, (flags & SGEP_VEC_BNORM) ? 2 : 1, (flags & SGEP_VEC_CANONICAL) != 0,
                   h->readout, out);
}

sgep_status sgep_vectors_noalloc(sgep_handle *h, int32_t flags, double *out)
{
    if (!h || !out || (flags & ~(SGEP_VEC_BNORM | SGEP_VEC_CANONICAL)) != 0)
        return SGEP_EINVAL;
    if ((uint64_t)h->d * (uint64_t)h->cfg.k > (uint64_t)kScratchDoubles)
        return SGEP_EUNSUPPORTED; // larger than the fixed staging array
    double *dst = g_scratch[h->device];
    if (!dst) { // not set up at init: look it up now, with the handle's device current
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        if (cur != h->device)
            HIPCHK(hipSetDevice(h->device));
        dst = scratch_of(h->device);
        if (cur != h->device)
            HIPCHK(hipSetDevice(cur));
        if (!dst)
            return SGEP_EDEVICE;
    }
    return readout(h, h->V, (flags & SGEP_VEC_BNORM) ? 2 : 1, (flags & SGEP_VEC_CANONICAL) != 0,
                   dst, out);
}

sgep_status sgep_auxiliary(sgep_handle *h, double *out)
{
    if (!h)
        return SGEP_EINVAL;
    return readout(h, h->G, 0, false, h->readout, out);
}

sgep_status sgep_means(sgep_handle *h, double *out)
{
    if (!h || !out || !h->mu)
        return SGEP_EINVAL;
    if (h->poisoned)
        return SGEP_EPOISONED;
    if (h->wide) { // FP32 at the state rows of the views
        std::vector<float> mb((size_t)h->wa.dtot);
        HIPCHK(hipMemcpyAsync(mb.data(), h->mu, mb.size() * sizeof(float), hipMemcpyDeviceToHost,
                              h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int64_t f = 0; f < h->cfg.dx; ++f)
            out[f] = (double)mb[(size_t)(h->wa.off[0] + f)];
        for (int64_t f = 0; f < h->cfg.dy; ++f)
            out[h->cfg.dx + f] = (double)mb[(size_t)(h->wa.off[1] + f)];
        return SGEP_OK;
    }
    const int64_t n = 2 * h->ldv;
    std::vector<unsigned char> buf((size_t)n * h->esz);
    HIPCHK(hipMemcpyAsync(buf.data(), h->mu, buf.size(), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    auto at = [&](int64_t i) {
        return h->esz == sizeof(double) ? ((const double *)buf.data())[i]
                                        : (double)((const float *)buf.data())[i];
    };
    // storage: CCA view x at 0, view y at dxp; GENERAL view x at 0, view y at ldv
    const int64_t dx = h->cfg.dx, dy = h->cfg.kind == SGEP_KIND_CCA ? h->cfg.dy : h->cfg.dx;
    const int64_t oy = h->cfg.kind == SGEP_KIND_CCA ? h->dxp : h->ldv;
    for (int64_t f = 0; f < dx; ++f)
        out[f] = at(f);
    for (int64_t f = 0; f < dy; ++f)
        out[dx + f] = at(oy + f);
    return SGEP_OK;
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
                 wide_stat_part_bytes(h->wa) + (h->mu ? (size_t)h->wa.dtot * sizeof(float) : 0);
        return SGEP_OK;
    }
    const size_t st = (size_t)h->ldv * h->kp * h->esz;
    *bytes = sizeof(StateHeader) + sizeof(Coef) + st * (h->Am ? 4 : 2) +
             (size_t)h->W * h->lds * sizeof(double) + (h->mu ? 2 * h->ldv * h->esz : 0);
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
    if (h->cflag) { // stamps left by later iterations must not match the next ones
        HIPCHK(hipMemsetAsync(h->cflag, 0, sizeof(unsigned long long), h->stream));
        HIPCHK(hipMemsetAsync(h->fpart, 0, h->fpart_bytes, h->stream));
    }
    if (h->xw)
        HIPCHK(hipMemsetAsync(h->xw, 0, h->xw_bytes, h->stream));
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

// ---------------------------------------------------------------------------
// Batched instances (sgep_batch.hpp): n narrow handles of kind GENERAL that
// share one stream, advanced together by a fixed sequence of launches.
// ---------------------------------------------------------------------------
namespace {

constexpr int kBuckets = 3; // d <= 256, d <= 1024, larger
constexpr int kMaxLag = 64;  // largest look-ahead of the persistent plan (instances)

int bucket_of(int64_t d) { return d <= 256 ? 0 : (d <= 1024 ? 1 : 2); }

struct BatchLaunchRec {
    int mb;         // 0: forward launch; otherwise the backward feature-tile height
    size_t map_off; // first entry of its map in the device map array
    int per_xcd;    // map entries per XCD
};

} // namespace

struct sgep_batch_s {
    sgep_config cfg;
    int n = 0;
    hipStream_t stream = nullptr;
    std::vector<sgep_handle *> inst;
    std::vector<int64_t> d, ld;
    std::vector<int> mb_min; // smallest tile height each instance's partials allow
    int mb_wide = 4;         // the larger candidate tile height for (dtype, KP)
    int groups = 1;
    int mb_bucket[kBuckets] = {1, 1, 1};
    std::vector<BatchLaunchRec> launches;
    StepArgs *d_args = nullptr;
    uint32_t *d_map = nullptr;
    // persistent plan (groups < 0): one launch per iteration over per-XCC
    // work queues with a look-ahead of `lag` instances
    int lag = 0;
    int n_xcc = 0;                       // XCCs of the device (0: unknown)
    int pers_grid = 0;                   // workgroups of the persistent launch
    unsigned long long *d_items = nullptr;
    int32_t *d_meta = nullptr;
    uint32_t *d_sync = nullptr;
    sgep::batch::Queues queues;
};

namespace {

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Build and upload the argument table and the launch maps for a plan:
// `groups` contiguous instance ranges of about equal total width, and the
// backward feature-tile height mb_bucket[bucket(d)] per instance.  Within a
// group every instance goes to one XCD, largest first, each to the XCD with
// the least total width so far.  Synchronous (init and tuning only).
// The persistent plan needs the XCC count (one queue per XCC), a player
// block of at most 128 bytes per feature (FP32 k <= 32, FP64 k <= 16) and
// 16-feature backward tiles for every instance.
bool persistent_ok(const sgep_batch *bt, const int *mb_bucket)
{
    const sgep_handle *h0 = bt->inst[0];
    if (bt->n_xcc < 1 || bt->n_xcc > sgep::batch::kMaxQueues || h0->kp * h0->esz > 128)
        return false;
    for (int c = 0; c < kBuckets; ++c)
        if (mb_bucket[c] != 1)
            return false;
    for (int i = 0; i < bt->n; ++i)
        if (bt->mb_min[i] != 1)
            return false;
    return true;
}

// The persistent plan: every instance to one XCC queue (largest first, each
// to the XCC with the least total width so far); per queue the items
//     F(i1) .. F(i_lag)  F(i_lag+1) C(i1) B(i1)  F(i_lag+2) C(i2) B(i2) ..
// (sgep_batch.hpp, k_bpers).  Synchronous (init and tuning only).
sgep_status apply_persistent(sgep_batch *bt, int lag)
{
    using namespace sgep::batch;
    const int n = bt->n;
    const int nq = bt->n_xcc;
    if (nq < 1 || nq > kMaxQueues || lag < 1)
        return SGEP_EUNSUPPORTED;
    std::vector<int> ids(n);
    for (int i = 0; i < n; ++i)
        ids[i] = i;
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return bt->d[a] > bt->d[b]; });
    std::vector<std::vector<int>> lists(nq);
    std::vector<int64_t> load(nq, 0);
    for (int i : ids) {
        int x = 0;
        for (int c = 1; c < nq; ++c)
            if (load[c] < load[x])
                x = c;
        load[x] += bt->d[i];
        lists[x].push_back(i);
    }
    const int64_t nf_max = ceil_div(bt->cfg.b_max, 16);
    auto item = [](int kind, int inst, int64_t tile) {
        return ((unsigned long long)kind << 48) | ((unsigned long long)inst << 32) |
               (unsigned long long)tile;
    };
    std::vector<unsigned long long> items;
    std::vector<int32_t> meta(2 * nq); // offsets, then lengths
    Queues Q;
    memset(&Q, 0, sizeof(Q));
    for (int x = 0; x < nq; ++x) {
        meta[x] = (int32_t)items.size();
        const int m = (int)lists[x].size();
        for (int j = 0; j < m + lag; ++j) {
            if (j < m) { // forward: the norm-totals workgroup first, then the row tiles
                const int i = lists[x][j];
                items.push_back(item(kItemFwd, i, nf_max));
                for (int64_t r = 0; r < nf_max; ++r)
                    items.push_back(item(kItemFwd, i, r));
            }
            if (j - lag >= 0 && j - lag < m) {
                const int i = lists[x][j - lag];
                const sgep_handle *h = bt->inst[i];
                items.push_back(item(kItemCoef, i, 0));
                for (int t = 0; t < h->n_tiles; ++t)
                    items.push_back(item(kItemBwd, i, t));
            }
        }
        meta[nq + x] = (int32_t)items.size() - meta[x];
    }
    Q.nq = nq;
    Q.nf_max = (int32_t)nf_max;
    Q.n = n;
    HIPCHK(hipStreamSynchronize(bt->stream));
    if (bt->d_items)
        HIPCHK(hipFree(bt->d_items));
    bt->d_items = nullptr;
    HIPCHK(hipMalloc((void **)&bt->d_items, items.size() * sizeof(unsigned long long)));
    HIPCHK(hipMemcpy(bt->d_items, items.data(), items.size() * sizeof(unsigned long long),
                     hipMemcpyHostToDevice));
    if (!bt->d_meta)
        HIPCHK(hipMalloc((void **)&bt->d_meta, 2 * kMaxQueues * sizeof(int32_t)));
    HIPCHK(hipMemcpy(bt->d_meta, meta.data(), meta.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice));
    const size_t nsync = (size_t)kSyncInst + 2 * (size_t)n;
    if (!bt->d_sync)
        HIPCHK(hipMalloc((void **)&bt->d_sync, nsync * sizeof(uint32_t)));
    HIPCHK(hipMemset(bt->d_sync, 0, nsync * sizeof(uint32_t)));
    HIPCHK(hipDeviceSynchronize());
    Q.items = bt->d_items;
    Q.meta = bt->d_meta;
    Q.sync = bt->d_sync;
    bt->queues = Q;
    bt->launches.assign(1, BatchLaunchRec{-2, 0, 0});
    bt->lag = lag;
    bt->groups = -lag;
    return SGEP_OK;
}

sgep_status apply_plan(sgep_batch *bt, int groups, const int *mb_bucket)
{
    const int n = bt->n;
    if (groups > n)
        groups = n;
    if (groups == 0)
        groups = 1;
    if (groups < 0 && !persistent_ok(bt, mb_bucket))
        return SGEP_EUNSUPPORTED;
    std::vector<StepArgs> args(n);
    for (int i = 0; i < n; ++i) {
        sgep_handle *h = bt->inst[i];
        int mb = mb_bucket[bucket_of(bt->d[i])];
        if (mb < bt->mb_min[i])
            mb = bt->mb_min[i];
        h->mb = mb;
        h->ft = 16 * mb;
        h->n_tx = (int)ceil_div(bt->d[i], h->ft);
        h->n_ty = 0;
        h->n_tiles = h->n_tx;
        const int64_t vec = 16 / (int64_t)h->esz;
        args[i] = make_args(h, bt->ld[i], bt->ld[i], bt->ld[i] % vec == 0);
    }
    if (groups < 0) {
        HIPCHK(hipStreamSynchronize(bt->stream)); // the old table may still be in use
        HIPCHK(hipMemcpy(bt->d_args, args.data(), n * sizeof(StepArgs), hipMemcpyHostToDevice));
        const sgep_status rc = apply_persistent(bt, -groups);
        if (rc == SGEP_OK)
            for (int c = 0; c < kBuckets; ++c)
                bt->mb_bucket[c] = mb_bucket[c];
        return rc;
    }
    // contiguous groups of about equal total width
    int64_t total = 0;
    for (int i = 0; i < n; ++i)
        total += bt->d[i];
    std::vector<int> gstart(1, 0);
    int64_t acc = 0;
    for (int i = 0; i < n && (int)gstart.size() < groups; ++i) {
        acc += bt->d[i];
        if (acc * groups >= total * (int64_t)gstart.size() && i + 1 < n)
            gstart.push_back(i + 1);
    }
    gstart.push_back(n);
    std::vector<uint32_t> map;
    std::vector<BatchLaunchRec> recs;
    for (size_t g = 0; g + 1 < gstart.size(); ++g) {
        std::vector<int> ids;
        for (int i = gstart[g]; i < gstart[g + 1]; ++i)
            ids.push_back(i);
        std::stable_sort(ids.begin(), ids.end(),
                         [&](int a, int b) { return bt->d[a] > bt->d[b]; });
        std::vector<int> xcd_of(n, 0);
        std::vector<std::vector<int>> lists(8);
        int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int i : ids) {
            int x = 0;
            for (int c = 1; c < 8; ++c)
                if (load[c] < load[x])
                    x = c;
            load[x] += bt->d[i];
            lists[x].push_back(i);
        }
        // forward: one entry per instance
        size_t per = 0;
        for (auto &l : lists)
            per = l.size() > per ? l.size() : per;
        BatchLaunchRec fr = {0, map.size(), (int)per};
        for (int x = 0; x < 8; ++x)
            for (size_t j = 0; j < per; ++j)
                map.push_back(j < lists[x].size() ? (uint32_t)lists[x][j] : sgep::batch::kNoTile);
        recs.push_back(fr);
        // coefficients: one workgroup per instance, same map as the forward
        recs.push_back(BatchLaunchRec{-1, fr.map_off, fr.per_xcd});
        // backward: one launch per tile height in use, entries (instance, tile)
        const int heights[2] = {1, bt->mb_wide};
        for (int hh = 0; hh < 2; ++hh) {
            const int mb = heights[hh];
            if (hh == 1 && mb == heights[0])
                break;
            std::vector<std::vector<uint32_t>> tl(8);
            size_t tper = 0;
            for (int x = 0; x < 8; ++x) {
                for (int i : lists[x])
                    if (bt->inst[i]->mb == mb)
                        for (int t = 0; t < bt->inst[i]->n_tiles; ++t)
                            tl[x].push_back(((uint32_t)i << 16) | (uint32_t)t);
                tper = tl[x].size() > tper ? tl[x].size() : tper;
            }
            if (tper == 0)
                continue;
            BatchLaunchRec br = {mb, map.size(), (int)tper};
            for (int x = 0; x < 8; ++x)
                for (size_t j = 0; j < tper; ++j)
                    map.push_back(j < tl[x].size() ? tl[x][j] : sgep::batch::kNoTile);
            recs.push_back(br);
        }
    }
    // upload (drain the stream first: the old tables may still be in use)
    HIPCHK(hipStreamSynchronize(bt->stream));
    if (bt->d_map)
        HIPCHK(hipFree(bt->d_map));
    bt->d_map = nullptr;
    HIPCHK(hipMalloc((void **)&bt->d_map, map.size() * sizeof(uint32_t)));
    HIPCHK(hipMemcpy(bt->d_map, map.data(), map.size() * sizeof(uint32_t),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bt->d_args, args.data(), n * sizeof(StepArgs), hipMemcpyHostToDevice));
    bt->launches = recs;
    bt->groups = (int)gstart.size() - 1;
    bt->lag = 0;
    for (int c = 0; c < kBuckets; ++c)
        bt->mb_bucket[c] = mb_bucket[c];
    return SGEP_OK;
}

template <typename T, int KP, bool CEN>
sgep_status batch_launch_c(sgep_batch *bt, const sgep::batch::Launch &base, void *const *events)
{
    using namespace sgep::batch;
    const bool adam = bt->cfg.optimizer == SGEP_ADAM;
    const int64_t nf = ceil_div(base.b, 16);
    int ie = 0;
    for (const BatchLaunchRec &r : bt->launches) {
        Launch L = base;
        L.map = bt->d_map + r.map_off;
        L.per_xcd = r.per_xcd;
        hipEvent_t e0 = events ? (hipEvent_t)events[ie] : nullptr;
        hipEvent_t e1 = events ? (hipEvent_t)events[ie + 1] : nullptr;
        ie += 2;
        const dim3 blk(sgep::kNT);
        constexpr int MBW = mb_wide<T>(KP);
        constexpr int GEN = sgep::kKindGeneral;
        if (r.mb == -2) { // persistent: every item of the iteration in one launch
          if constexpr (KP * sizeof(T) <= 128) {
            auto kern = adam ? k_bpers<T, KP, sgep::kOptAdam, CEN> : k_bpers<T, KP, sgep::kOptSGD, CEN>;
            if (bt->pers_grid == 0) {
                // as many workgroups as the CUs hold at once (the queues are
                // drained by whichever run; more would only wait to start)
                int occ = 0, cus = 0, dev = 0;
                HIPCHK(hipGetDevice(&dev));
                HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
                HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, sgep::kNT, 0));
                bt->pers_grid = (occ < 1 ? 1 : occ) * (cus < 1 ? 1 : cus);
            }
            launch_k(kern, dim3((unsigned)bt->pers_grid), blk, bt->stream, e0, e1, L, bt->queues,
                     L.args, L.X, L.Y);
          } else {
            return SGEP_EUNSUPPORTED; // not planned for larger player blocks
          }
        } else if (r.mb == 0) {
            launch_k(k_bfwd<T, KP, GEN, CEN>, dim3((unsigned)(8 * r.per_xcd * (nf + 1))), blk,
                     bt->stream, e0, e1, L, L.args, L.X, L.Y);
        } else if (r.mb < 0) {
            launch_k(k_bcoef<T, KP, GEN>, dim3((unsigned)(8 * r.per_xcd)), blk, bt->stream, e0, e1,
                     L, L.args, L.X, L.Y);
        } else {
            const dim3 grid((unsigned)(8 * r.per_xcd));
            if (r.mb == 1 && !adam)
                launch_k(k_bbwd<T, KP, 1, GEN, sgep::kOptSGD, CEN>, grid, blk, bt->stream, e0, e1, L,
                         L.args, L.X, L.Y);
            else if (r.mb == 1)
                launch_k(k_bbwd<T, KP, 1, GEN, sgep::kOptAdam, CEN>, grid, blk, bt->stream, e0, e1, L,
                         L.args, L.X, L.Y);
            else if (!adam)
                launch_k(k_bbwd<T, KP, MBW, GEN, sgep::kOptSGD, CEN>, grid, blk, bt->stream, e0, e1, L,
                         L.args, L.X, L.Y);
            else
                launch_k(k_bbwd<T, KP, MBW, GEN, sgep::kOptAdam, CEN>, grid, blk, bt->stream, e0, e1, L,
                         L.args, L.X, L.Y);
        }
    }
    HIPCHK(hipGetLastError());
    return SGEP_OK;
}

// the batch's centring flag as a compile-time choice of the kernels
template <typename T, int KP>
sgep_status batch_launch_t(sgep_batch *bt, const sgep::batch::Launch &base, void *const *events)
{
    return bt->cfg.center ? batch_launch_c<T, KP, true>(bt, base, events)
                          : batch_launch_c<T, KP, false>(bt, base, events);
}

sgep_status batch_step_impl(sgep_batch *bt, const void *const *X, const void *const *Y, int64_t b,
                            void *const *events)
{
    if (!bt || !X || !Y)
        return SGEP_EINVAL;
    if (b < 1 || b > bt->cfg.b_max)
        return SGEP_ESHAPE;
    for (sgep_handle *h : bt->inst)
        if (h->poisoned)
            return SGEP_EPOISONED;
    sgep::batch::Launch L;
    memset(&L, 0, sizeof(L));
    L.args = bt->d_args;
    L.X = X;
    L.Y = Y;
    L.b = b;
    sgep_handle *h0 = bt->inst[0];
    return SGEP_DISPATCH(h0, batch_launch_t, bt, L, events);
}

void batch_free(sgep_batch *bt)
{
    for (sgep_handle *h : bt->inst)
        if (h) {
            free_all(h);
            delete h;
        }
    if (bt->d_args)
        (void)hipFree(bt->d_args);
    if (bt->d_map)
        (void)hipFree(bt->d_map);
    if (bt->d_items)
        (void)hipFree(bt->d_items);
    if (bt->d_sync)
        (void)hipFree(bt->d_sync);
    if (bt->d_meta)
        (void)hipFree(bt->d_meta);
    delete bt;
}

// device state of every instance that an iteration changes (the players, the
// auxiliary variable, the Adam moments, the norm / parent partials and the
// coefficient block), for the tuner's trial iterations
struct BatchSnapshot {
    void *buf = nullptr;
    std::vector<std::pair<void *, size_t>> parts;
    size_t total = 0;
};

sgep_status batch_snapshot(sgep_batch *bt, BatchSnapshot &s)
{
    for (sgep_handle *h : bt->inst) {
        StateLayout L = state_layout(h);
        for (int i = 0; i < L.n; ++i)
            s.parts.push_back({L.ptr[i], L.bytes[i]});
        s.parts.push_back({h->coef, sizeof(Coef)});
    }
    for (auto &p : s.parts)
        s.total += (p.second + 255) / 256 * 256;
    HIPCHK(hipMalloc(&s.buf, s.total));
    size_t off = 0;
    for (auto &p : s.parts) {
        HIPCHK(hipMemcpyAsync((char *)s.buf + off, p.first, p.second, hipMemcpyDeviceToDevice,
                              bt->stream));
        off += (p.second + 255) / 256 * 256;
    }
    return SGEP_OK;
}

sgep_status batch_restore(sgep_batch *bt, const BatchSnapshot &s)
{
    size_t off = 0;
    for (auto &p : s.parts) {
        HIPCHK(hipMemcpyAsync(p.first, (char *)s.buf + off, p.second, hipMemcpyDeviceToDevice,
                              bt->stream));
        off += (p.second + 255) / 256 * 256;
    }
    return SGEP_OK;
}

// every instance still at its initial state (no iteration run yet)
sgep_status batch_at_start(sgep_batch *bt, bool *yes)
{
    *yes = true;
    for (sgep_handle *h : bt->inst) {
        double t = 0.0;
        HIPCHK(hipMemcpyAsync(&t, &h->coef->t, sizeof(double), hipMemcpyDeviceToHost,
                              bt->stream));
        HIPCHK(hipStreamSynchronize(bt->stream));
        if (t != 0.0)
            *yes = false;
    }
    return SGEP_OK;
}

} // namespace

extern "C" {

sgep_status sgep_batch_init(sgep_batch **out, int32_t n, const int64_t *d, const int64_t *ld,
                            const sgep_config *common, const double *const *V0, void *hip_stream)
{
    if (!out)
        return SGEP_EINVAL;
    *out = nullptr;
    if (!d || !ld || !common || !V0 || n < 1)
        return SGEP_EINVAL;
    if (n > 65535)
        return SGEP_EUNSUPPORTED;
    if (common->kind != SGEP_KIND_GENERAL)
        return SGEP_EUNSUPPORTED;
    if (common->dtype != SGEP_F32 && common->dtype != SGEP_F64)
        return SGEP_EUNSUPPORTED;
    for (int i = 0; i < n; ++i) {
        if (!V0[i])
            return SGEP_EINVAL;
        if (d[i] < 1 || ld[i] < d[i])
            return SGEP_ESHAPE;
    }
    sgep_batch *bt = new (std::nothrow) sgep_batch_s();
    if (!bt)
        return SGEP_ENOMEM;
    bt->cfg = *common;
    bt->n = n;
    bt->stream = (hipStream_t)hip_stream;
    bt->d.assign(d, d + n);
    bt->ld.assign(ld, ld + n);
    bt->inst.assign(n, nullptr);
    bt->mb_min.assign(n, 1);
    for (int i = 0; i < n; ++i) {
        sgep_config c = *common;
        c.dx = c.dy = d[i];
        sgep_status rc = sgep_init(&bt->inst[i], &c, V0[i], hip_stream);
        if (rc != SGEP_OK) {
            bt->inst[i] = nullptr;
            batch_free(bt);
            return rc;
        }
        bt->mb_min[i] = bt->inst[i]->mb; // partials sized for this height or larger
    }
    const sgep_handle *h0 = bt->inst[0];
    bt->mb_wide = h0->esz == sizeof(double) ? (h0->kp * 8 <= 128 ? 4 : 2)
                                            : (h0->kp * 4 <= 128 ? 4 : 2);
    if (hipMalloc((void **)&bt->d_args, (size_t)n * sizeof(StepArgs)) != hipSuccess) {
        bt->d_args = nullptr;
        batch_free(bt);
        return SGEP_ENOMEM;
    }
    {
        int dev = 0, nx = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) == hipSuccess)
            bt->n_xcc = nx;
    }
    const int mb1[kBuckets] = {1, 1, 1};
    sgep_status rc = apply_plan(bt, 1, mb1);
    if (rc != SGEP_OK) {
        batch_free(bt);
        return rc;
    }
    *out = bt;
    return SGEP_OK;
}

sgep_status sgep_batch_instance(sgep_batch *bt, int32_t i, sgep_handle **h)
{
    if (!bt || !h || i < 0 || i >= bt->n)
        return SGEP_EINVAL;
    *h = bt->inst[i];
    return SGEP_OK;
}

sgep_status sgep_batch_step(sgep_batch *bt, const void *const *X, const void *const *Y, int64_t b)
{
    return batch_step_impl(bt, X, Y, b, nullptr);
}

sgep_status sgep_batch_launches(const sgep_batch *bt, int32_t *n, int32_t *kinds, int32_t cap)
{
    if (!bt || !n)
        return SGEP_EINVAL;
    *n = (int32_t)bt->launches.size();
    if (kinds) {
        if (cap < *n)
            return SGEP_ESHAPE;
        for (int32_t i = 0; i < *n; ++i)
            kinds[i] = bt->launches[i].mb;
    }
    return SGEP_OK;
}

sgep_status sgep_batch_step_profiled(sgep_batch *bt, const void *const *X, const void *const *Y,
                                     int64_t b, void *const *events, int32_t n_events)
{
    if (!bt || !events || n_events != 2 * (int32_t)bt->launches.size())
        return SGEP_EINVAL;
    for (int32_t i = 0; i < n_events; ++i)
        if (!events[i])
            return SGEP_EINVAL;
    return batch_step_impl(bt, X, Y, b, events);
}

sgep_status sgep_batch_plan(const sgep_batch *bt, int32_t *groups, int32_t *mb_bucket)
{
    if (!bt || !groups || !mb_bucket)
        return SGEP_EINVAL;
    *groups = bt->groups;
    for (int c = 0; c < kBuckets; ++c)
        mb_bucket[c] = bt->mb_bucket[c];
    return SGEP_OK;
}

sgep_status sgep_batch_set_plan(sgep_batch *bt, int32_t groups, const int32_t *mb_bucket)
{
    if (!bt || !mb_bucket || groups == 0 || groups < -kMaxLag)
        return SGEP_EINVAL;
    int mb[kBuckets];
    for (int c = 0; c < kBuckets; ++c) {
        if (mb_bucket[c] != 1 && mb_bucket[c] != bt->mb_wide)
            return SGEP_EINVAL;
        mb[c] = mb_bucket[c];
    }
    bool start = false;
    sgep_status rc = batch_at_start(bt, &start);
    if (rc != SGEP_OK)
        return rc;
    if (!start)
        return SGEP_EINVAL; // the partials of a running state fix the tile heights
    return apply_plan(bt, groups, mb);
}

sgep_status sgep_batch_tune(sgep_batch *bt, const void *const *X, const void *const *Y, int64_t b,
                            int32_t reps, double *best_us)
{
    if (!bt || !X || !Y || reps < 1)
        return SGEP_EINVAL;
    if (b < 1 || b > bt->cfg.b_max)
        return SGEP_ESHAPE;
    for (sgep_handle *h : bt->inst)
        if (h->poisoned)
            return SGEP_EPOISONED;
    bool start = false;
    sgep_status rc = batch_at_start(bt, &start);
    if (rc != SGEP_OK)
        return rc;
    if (!start)
        return SGEP_EINVAL;
    bool used[kBuckets] = {false, false, false};
    for (int i = 0; i < bt->n; ++i)
        used[bucket_of(bt->d[i])] = true;
    BatchSnapshot snap;
    rc = batch_snapshot(bt, snap);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == SGEP_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = SGEP_EDEVICE;
    double best = 1e300;
    int best_g = 1, best_mb[kBuckets] = {1, 1, 1};
    // grouped launches (1, 2, 4, 8 groups) and the persistent launch with a
    // look-ahead of 1, 2 or 4 instances (when the XCC count is known)
    const int gcand[7] = {1, 2, 4, 8, -1, -2, -4};
    for (int gi = 0; gi < 7 && rc == SGEP_OK; ++gi) {
        if (gcand[gi] > bt->n || (gcand[gi] < 0 && -gcand[gi] > bt->n))
            continue;
        if (gcand[gi] < 0) {
            const int mb1[kBuckets] = {1, 1, 1};
            if (!persistent_ok(bt, mb1))
                continue;
        }
        for (int mask = 0; mask < (1 << kBuckets) && rc == SGEP_OK; ++mask) {
            int mb[kBuckets];
            bool dup = false;
            for (int c = 0; c < kBuckets; ++c) {
                const bool wide = (mask >> c) & 1;
                if (wide && (!used[c] || bt->mb_wide == 1))
                    dup = true; // same plan as with this bit clear
                mb[c] = wide ? bt->mb_wide : 1;
            }
            if (dup || (gcand[gi] < 0 && mask != 0))
                continue; // the persistent form has 16-feature tiles only
            rc = apply_plan(bt, gcand[gi], mb);
            if (rc == SGEP_OK)
                rc = batch_restore(bt, snap);
            if (rc == SGEP_OK)
                rc = batch_step_impl(bt, X, Y, b, nullptr); // warm-up
            if (rc != SGEP_OK)
                break;
            if (hipEventRecord(e0, bt->stream) != hipSuccess) {
                rc = SGEP_EDEVICE;
                break;
            }
            for (int r = 0; r < reps && rc == SGEP_OK; ++r)
                rc = batch_step_impl(bt, X, Y, b, nullptr);
            float ms = 0.f;
            if (rc != SGEP_OK || hipEventRecord(e1, bt->stream) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = rc != SGEP_OK ? rc : SGEP_EDEVICE;
                break;
            }
            const double us = 1e3 * ms / reps;
            if (us < best) {
                best = us;
                best_g = gcand[gi];
                for (int c = 0; c < kBuckets; ++c)
                    best_mb[c] = mb[c];
            }
        }
    }
    if (rc == SGEP_OK)
        rc = apply_plan(bt, best_g, best_mb);
    if (rc == SGEP_OK && snap.buf)
        rc = batch_restore(bt, snap);
    if (hipStreamSynchronize(bt->stream) != hipSuccess && rc == SGEP_OK)
        rc = SGEP_EDEVICE;
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (snap.buf)
        (void)hipFree(snap.buf);
    // trial iterations may have latched a fault in a status word: the
    // restored coefficient blocks clear it
    for (sgep_handle *h : bt->inst)
        h->poisoned = false;
    if (rc == SGEP_OK && best_us)
        *best_us = best;
    return rc;
}

sgep_status sgep_batch_sync(sgep_batch *bt)
{
    if (!bt)
        return SGEP_EINVAL;
    sgep_status first = SGEP_OK;
    for (sgep_handle *h : bt->inst) {
        const sgep_status rc = sgep_sync(h);
        if (rc != SGEP_OK && first == SGEP_OK)
            first = rc;
    }
    return first;
}

sgep_status sgep_batch_destroy(sgep_batch *bt)
{
    if (!bt)
        return SGEP_EINVAL;
    (void)hipStreamSynchronize(bt->stream);
    batch_free(bt);
    return SGEP_OK;
}

} // extern "C"
