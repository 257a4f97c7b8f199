// sgep_kernels.hpp -- CDNA4 (gfx950) kernels of the stochastic gamma-EigenGame
// step (Alg. 2 of Gemp, Chen, McWilliams, ICLR 2023, with M = 1).
//
// One iteration is two launches in the basic form (below); the row-split form
// of the CCA handles (k_fwds, k_bwdp) is described at those kernels: there a
// workgroup may wait on stamped words published by workgroups of lower index
// in the same launch (bounded polls; a give-up sets the status word).  The
// basic form has no cross-workgroup wait inside a launch:
//   k_fwd  P = X V and Q = Y V for a 16-row tile (tall-skinny products on
//          MFMA, features split over the four waves), stored unnormalised,
//          plus the tile's partial k x k Gram terms (column-major partials).
//          One extra workgroup reduces the previous iteration's norm /
//          parent-term partials to totals and advances the step counter.
//   k_bwd  for a tile of features: A_t V and B_t V (X^T [Q|P] on MFMA over
//          all minibatch rows), then every workgroup reduces -- in the same
//          fixed order, so all obtain identical bits -- the Gram partials,
//          forms the k x k coefficients, and runs the fused epilogue:
//          update direction, retraction step (SGD or Adam), auxiliary update,
//          and this tile's partials of ||v_i||^2 and v_i^T [Bv]_j.
//
// Matrix form of the update direction.  With unit players v_i, auxiliary
// G_j = [Bv]_j, minibatch Gram M_A = V^T A_t V, m_B,i = v_i^T B_t v_i,
// s_j = max(v_j^T G_j, rho), C_ij = v_i^T G_j, T_ij = (M_A)_ij / s_j (j < i)
// and c_i = sum_{j<i} T_ij C_ij, the rewards-minus-penalties direction of
// Alg. 2 for all players at once is
//     grad = (A_t V - G T^T) diag(m_B) - B_t V diag(m_A - c),
// because v_i^T A_t y_j = (M_A)_ij / sqrt(s_j), [By]_j = G_j / sqrt(s_j) and
// <v_i, [By]_j> = C_ij / sqrt(s_j).  Sharing A_t V and B_t V across players
// turns the per-player O(b d k^2) of the paper's loop into O(b d k + d k^2).
//
// Normalisation is lazy: the stored V is the iterate before it is projected
// back to the sphere, and 1/||V_i|| (from the norm partials) scales every use.
// Storage is quad-interleaved: element (f, i) of V, G and the Adam moments
// (feature f, player i; KP = 16, 32 or 64 players, those beyond k zero) sits
// at qidx(f, i) = (f / 4) 4 KP + 4 i + f % 4, each view padded to a multiple
// of 4 features; the projections P = X V and Q = Y V use the same layout with
// the minibatch row in place of f.  A lane fetches the MFMA B operand of four
// consecutive k-indices (features or rows) of one player in one 16-byte load,
// and the 64 lanes of a wave read one contiguous 1 KB block.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace sgep {

// Global-memory pointer type.  Pointers that reach a kernel through memory
// (the batched argument table) are otherwise generic, and generic (flat)
// accesses also count against the LDS / scalar wait counter.
#define SGEP_G __attribute__((address_space(1)))

constexpr int kNT = 256;     // threads per workgroup: four wave64
constexpr int kKPMax = 64;   // largest padded player count

constexpr int kKindCCA = 0;
constexpr int kKindGeneral = 1;
constexpr int kKindICA = 3; // kurtosis form of ICA: one view, A and B from its moments
constexpr int kOptSGD = 0;
constexpr int kOptAdam = 1;

constexpr int kStatusNonFinite = 1;
constexpr int kStatusSync = 4; // a workgroup gave up waiting for the coefficient block (2: wide path, bad label)
// s_waitcnt operand: vector memory counter 0 (stores included), the
// export and LDS / scalar counters at their maxima (not waited for)
constexpr int kWaitVm0 = 0x0F70;
constexpr int kSpinMax = 1 << 20; // polls a thread may spend on all its bounded waits of a launch (each with a short sleep)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// 16x16x4 MFMA for one element type.  Operand layout (wave64), identical for
// FP32 and FP64:
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
// The result layout differs (measured on gfx950):
//   FP32 D (16 x 16): lane l, register r holds D[4 (l / 16) + r][l % 16]
//   FP64 D (16 x 16): lane l, register r holds D[(l / 16) + 4 r][l % 16]
// drow(l / 16, r) gives the row of D held in register r.
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef f32x4 acc;
    static __device__ __forceinline__ acc fma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int kk, int r) { return 4 * kk + r; }
};
template <> struct Mfma<double> {
    typedef f64x4 acc;
    static __device__ __forceinline__ acc fma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int kk, int r) { return kk + 4 * r; }
};

// Public per-handle block (device memory, FP64): step counter, the
// coefficients of the latest iteration, running means and the status word.
struct Coef {
    double t;                // completed iterations (incremented by k_fwd)
    double eta, gamma;       // step sizes of the latest iteration
    double mA[kKPMax];       // v_i^T A_t v_i (latest iteration)
    double mB[kKPMax];       // v_i^T B_t v_i
    double c[kKPMax];        // sum_{j<i} T_ij C_ij
    double s[kKPMax];        // estimate of v_j^T B v_j used by the latest iteration
    double ema_a[kKPMax];    // running mean of mA (rate gamma)
    double ema_b[kKPMax];    // running mean of mB
    double z[2][kKPMax];     // Alg. 3 variables: iteration t reads z[t & 1] and
                             // writes z[(t + 1) & 1] (other workgroups may still
                             // read z[t & 1] while the writer stores)
    int status;              // kStatus* bits
    int clip_count;          // parents clipped at rho, cumulative
};

struct StepArgs {
    const void *X, *Y;
    int64_t ldx, ldy, b;
    int64_t dx, dy;          // CCA: view widths; GENERAL: dx = dy = d
    int64_t dxp;             // storage offset of view y in a player row (CCA), 0 otherwise
    int64_t ldv;             // padded feature count of V, G and the Adam moments
    int64_t ldp;             // padded row count of P and Q (multiple of 4)
    int32_t k, n_tx, n_ty;   // feature tiles over view x and view y (GENERAL: n_ty = 0)
    int32_t vec_ok;          // rows of X and Y 16-byte aligned: vector loads allowed
    int32_t n_fwd;           // forward workgroups (16-row tiles) of this iteration
    int32_t ldg, lds;        // rows allocated for the Gram / stats partials
    void *V, *G, *Am, *As;   // ldv x KP, quad-interleaved
    void *P, *Q;             // ldp x KP, quad-interleaved raw projections X V, Y V
    double *gram_part;       // [ldg][W]: row blk = forward workgroup blk
    void *fpart;             // per-view forward: [n_fwd][16 KP] stamped words of P (Stamped<T>)
    unsigned long long *cflag; // row split: iteration of the latest coefficient block
    void *xw;                // fused row split: stamped words of the slices' products, then of
    int64_t xw_coef;         //   the coefficient block from word xw_coef on
    double *stat_part;       // [lds][W]: row tile = backward workgroup tile
    double *stat_tot;        // [W]: reduced stat_part of the state entering this iteration
    Coef *coef;
    void *cpre;              // coefficient block of the iteration (kModePre, kModeFin)
    void *bpart;             // [tile][split][2 FT KP + 2 FT] partial products and
                             // centred column sums (kModePart)
    void *mu;                // running means of the views (centring): view x (CCA:
                             // both views) at storage positions, GENERAL view y at +ldv
    void *S1, *S2;           // ICA: X^T P and X^T diag(||x_r||^2) P of the iteration,
                             // quad-interleaved like V (raw sums over the rows)
    double *bb_part;         // ICA: [tiles][KP(KP+1)/2] partials of S1^T S1
    double *gsum;            // column totals of the Gram partials (two-stage k_coef)
    int32_t nsplit;          // row slices of the backward products (kModePart)
    int32_t schedule;
    int32_t smooth;          // Alg. 3 estimate of v_j^T B v_j instead of the clip
    double eta0, eta_T, t0, t_c, T, gamma, rho, eps_reg, adam_b1, adam_b2, adam_eps;
    double lrho, lspan;      // Alg. 3: log rho, log nu - log rho
};

__device__ __forceinline__ int tri_idx(int i, int j) { return i * (i + 1) / 2 + j; } // j <= i

// Workgroup index -> tile index such that consecutive tiles run on the same
// XCD (workgroups are dealt to the 8 XCDs round-robin): neighbouring feature
// tiles share the 128-byte lines of a minibatch row, so they should share an
// L2.  Identity when the count is not a multiple of 8.
__device__ __forceinline__ int xcd_tile(int b, int nblk)
{
    if (nblk % 8 != 0)
        return b;
    return (b % 8) * (nblk / 8) + b / 8;
}

// quad-interleaved position of (feature or row f, player i) for KP players
template <int KP>
__device__ __forceinline__ int64_t qidx(int64_t f, int i)
{
    return (f >> 2) * (4 * KP) + 4 * i + (f & 3);
}

__device__ __forceinline__ void tri_ij(int e, int &i, int &j)
{
    int ii = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while (ii * (ii + 1) / 2 > e)
        --ii;
    while ((ii + 1) * (ii + 2) / 2 <= e)
        ++ii;
    i = ii;
    j = e - ii * (ii + 1) / 2;
}

// eta_t for iteration t = 1, 2, ...: constant, eta0 / (1 + t / t0), or linear
// warmup to t_c followed by harmonic decay reaching eta_T at T.
__device__ inline double eta_at(const StepArgs &a, double t)
{
    if (a.schedule == 0)
        return a.eta0;
    if (a.schedule == 1)
        return a.eta0 / (1.0 + t / a.t0);
    if (t < a.t_c)
        return a.eta0 * t / a.t_c;
    const double D = (a.eta_T * a.T - a.eta0 * a.t_c) / (a.eta0 - a.eta_T);
    return a.eta0 * (a.t_c + D) / (t + D);
}

// Column sums out[c] = sum_{r < n} part[r * ld + c], rows in ascending
// order, for c < W: thread q of nthr takes columns q, q + nthr, ...  Rows
// are the partials of one workgroup each (W contiguous values), so the
// threads of a wave read consecutive addresses; R rows per thread are in
// flight together (more for the one-workgroup coefficient kernel, which has
// the registers).  No synchronisation inside (the caller orders the writes
// to out).  Every caller uses the same order of the sums, so all obtain the
// same bits.
template <int R = 32>
__device__ inline void colsum(const SGEP_G double *__restrict__ part, int n, int ld, int W,
                              double *__restrict__ out, int q, int nthr)
{
    for (int c = q; c < W; c += nthr) {
        double s = 0.0;
        for (int r0 = 0; r0 < n; r0 += R) {
            double v[R];
#pragma unroll
            for (int u = 0; u < R; ++u)
                v[u] = r0 + u < n ? part[(uint32_t)((r0 + u) * ld + c)] : 0.0;
#pragma unroll
            for (int u = 0; u < R; ++u)
                if (r0 + u < n)
                    s += v[u];
        }
        out[c] = s;
    }
}

template <typename T, int N> struct VecLoad;
template <> struct VecLoad<float, 1> {
    static __device__ __forceinline__ void run(const SGEP_G float *p, float *o) { o[0] = p[0]; }
};
template <> struct VecLoad<double, 1> {
    static __device__ __forceinline__ void run(const SGEP_G double *p, double *o) { o[0] = p[0]; }
};
template <> struct VecLoad<float, 4> {
    static __device__ __forceinline__ void run(const SGEP_G float *p, float *o)
    {
        f32x4 v = *reinterpret_cast<const SGEP_G f32x4 *>(p);
        o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
    }
};
template <> struct VecLoad<float, 2> {
    static __device__ __forceinline__ void run(const SGEP_G float *p, float *o)
    {
        f32x2 v = *reinterpret_cast<const SGEP_G f32x2 *>(p);
        o[0] = v[0]; o[1] = v[1];
    }
};
template <> struct VecLoad<double, 2> {
    static __device__ __forceinline__ void run(const SGEP_G double *p, double *o)
    {
        f64x2 v = *reinterpret_cast<const SGEP_G f64x2 *>(p);
        o[0] = v[0]; o[1] = v[1];
    }
};
template <> struct VecLoad<double, 4> {
    static __device__ __forceinline__ void run(const SGEP_G double *p, double *o)
    {
        f64x2 v0 = *reinterpret_cast<const SGEP_G f64x2 *>(p);
        f64x2 v1 = *reinterpret_cast<const SGEP_G f64x2 *>(p + 2);
        o[0] = v0[0]; o[1] = v0[1]; o[2] = v1[0]; o[3] = v1[1];
    }
};

// ---------------------------------------------------------------------------
// Forward products.  One wave accumulates the 16 x KP tile of one view over a
// contiguous quarter of the feature chunks (CH = 4 VEC features).  Lane l
// loads VEC consecutive features fb = c CH + VEC (l/16) .. + VEC - 1 of its
// row, and for B the same VEC features of player row (l % 16) of V^T: MFMA j
// of the chunk consumes element j of both, so its k-index l/16 stands for
// feature fb + j and the sum over features is unchanged.  Batches of U chunks
// issue all loads before any MFMA; chunks past the wave's full range are
// loaded from a valid chunk and zeroed; the ragged last chunk runs masked.
// `row` is a valid row index; rows past the minibatch are zeroed through rv.
// ---------------------------------------------------------------------------
template <typename T, int KP, bool CENTER = false, bool SQ = false, int NW = 4>
__device__ __forceinline__ void fwd_view(const SGEP_G T *__restrict__ X, int64_t ldx, int64_t nf,
                                         int64_t row, bool rv, bool vec_ok,
                                         const SGEP_G T *__restrict__ VQ,
                                         int lane, int w, typename Mfma<T>::acc (*acc)[KP / 16],
                                         const SGEP_G T *__restrict__ mu = nullptr,
                                         T *sq = nullptr)
{
    constexpr int VEC = 16 / (int)sizeof(T);
    constexpr int CH = 4 * VEC;
    constexpr int NB = KP / 16;
    constexpr int U = (CENTER ? 4 : 8) / NB * 4 / NW > 0 ? (CENTER ? 4 : 8) / NB * 4 / NW : 1;
    const int kk = lane >> 4, n = lane & 15;
    const int64_t nch = (nf + CH - 1) / CH;
    const int64_t nfull = nf / CH; // chunks whose features are all valid
    const int64_t c0 = (nch * w) / NW, c1 = (nch * (w + 1)) / NW;
    const int64_t cf = c1 < nfull ? c1 : nfull;
    const SGEP_G T *xr = X + row * ldx;
    for (int64_t c = c0; c < cf; c += U) {
        T xv[U][VEC], mv[U][VEC];
        T bv[U][NB][VEC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t cu = (c + u < cf) ? c + u : c;
            const int64_t fb = cu * CH + (int64_t)VEC * kk;
            if (vec_ok) {
                VecLoad<T, VEC>::run(xr + fb, xv[u]);
            } else {
#pragma unroll
                for (int j = 0; j < VEC; ++j)
                    xv[u][j] = xr[fb + j];
            }
            if (CENTER)
                VecLoad<T, VEC>::run(mu + fb, mv[u]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                VecLoad<T, VEC>::run(VQ + qidx<KP>(fb, nb * 16 + n), bv[u][nb]);
        }
        // keep the batch's loads ahead of its MFMAs (no interleaving by the
        // scheduler, which would serialise the memory latency)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = rv && (c + u < cf);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const T xs = ok ? (CENTER ? xv[u][j] - mv[u][j] : xv[u][j]) : T(0);
                if (SQ)
                    *sq += xs * xs; // this lane's part of ||x_row||^2
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[j & 1][nb] = Mfma<T>::fma(xs, bv[u][nb][j], acc[j & 1][nb]);
            }
        }
    }
    if (nfull < c1 && nfull >= c0) { // the ragged last chunk, features masked
        const int64_t fb = nfull * CH + (int64_t)VEC * kk;
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const int64_t fe = fb + j;
            const bool fv = fe < nf;
            const int64_t fc = fv ? fe : nf - 1;
            const T xs = (rv && fv) ? (CENTER ? xr[fc] - mu[fc] : xr[fc]) : T(0);
            if (SQ)
                *sq += xs * xs;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const T bvv = fv ? VQ[qidx<KP>(fc, nb * 16 + n)] : T(0);
                acc[0][nb] = Mfma<T>::fma(xs, bvv, acc[0][nb]);
            }
        }
    }
}

// Both views of the same width in one pass: the loads of a batch cover the
// chunks of both, so the memory latency is paid once per batch instead of
// once per view.  Same arithmetic (per view, chunk order and accumulator
// assignment) as two calls of fwd_view.  SAMEV (GENERAL: one V for both
// products) loads the V operand once; a compile-time choice, because a
// run-time one makes the compiler drain all loads in flight around it.
// LOWREG halves the chunks per batch (fewer registers, more workgroups per
// CU, for launches with many workgroups); the accumulation order is the same.
template <typename T, int KP, bool SAMEV, bool LOWREG, bool CENTER = false>
__device__ __forceinline__ void fwd_view2(const SGEP_G T *__restrict__ X, int64_t ldx,
                                          const SGEP_G T *__restrict__ Y, int64_t ldy, int64_t nf,
                                          int64_t row, bool rv, bool vec_ok,
                                          const SGEP_G T *__restrict__ VQx,
                                          const SGEP_G T *__restrict__ VQy,
                                          int lane, int w, typename Mfma<T>::acc (*accx)[KP / 16],
                                          typename Mfma<T>::acc (*accy)[KP / 16],
                                          const SGEP_G T *__restrict__ mux = nullptr,
                                          const SGEP_G T *__restrict__ muy = nullptr)
{
    constexpr int VEC = 16 / (int)sizeof(T);
    constexpr int CH = 4 * VEC;
    constexpr int NB = KP / 16;
    constexpr int U = ((LOWREG || CENTER) ? 4 : 8) / NB;
    const int kk = lane >> 4, n = lane & 15;
    const int64_t nch = (nf + CH - 1) / CH;
    const int64_t nfull = nf / CH;
    const int64_t c0 = (nch * w) >> 2, c1 = (nch * (w + 1)) >> 2;
    const int64_t cf = c1 < nfull ? c1 : nfull;
    const SGEP_G T *xr = X + row * ldx;
    const SGEP_G T *yr = Y + row * ldy;
    for (int64_t c = c0; c < cf; c += U) {
        T xv[U][VEC], yv[U][VEC], mx[U][VEC], my[U][VEC];
        T bx[U][NB][VEC], by[U][NB][VEC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t cu = (c + u < cf) ? c + u : c;
            const int64_t fb = cu * CH + (int64_t)VEC * kk;
            if (vec_ok) {
                VecLoad<T, VEC>::run(xr + fb, xv[u]);
                VecLoad<T, VEC>::run(yr + fb, yv[u]);
            } else {
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    xv[u][j] = xr[fb + j];
                    yv[u][j] = yr[fb + j];
                }
            }
            if (CENTER) {
                VecLoad<T, VEC>::run(mux + fb, mx[u]);
                VecLoad<T, VEC>::run(muy + fb, my[u]);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                VecLoad<T, VEC>::run(VQx + qidx<KP>(fb, nb * 16 + n), bx[u][nb]);
                if (!SAMEV)
                    VecLoad<T, VEC>::run(VQy + qidx<KP>(fb, nb * 16 + n), by[u][nb]);
            }
        }
        __builtin_amdgcn_sched_barrier(0); // the whole batch's loads first
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = rv && (c + u < cf);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const T xs = ok ? (CENTER ? xv[u][j] - mx[u][j] : xv[u][j]) : T(0);
                const T ys = ok ? (CENTER ? yv[u][j] - my[u][j] : yv[u][j]) : T(0);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    accx[j & 1][nb] = Mfma<T>::fma(xs, bx[u][nb][j], accx[j & 1][nb]);
                    accy[j & 1][nb] =
                        Mfma<T>::fma(ys, SAMEV ? bx[u][nb][j] : by[u][nb][j], accy[j & 1][nb]);
                }
            }
        }
    }
    if (nfull < c1 && nfull >= c0) { // the ragged last chunk, features masked
        const int64_t fb = nfull * CH + (int64_t)VEC * kk;
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const int64_t fe = fb + j;
            const bool fv = fe < nf;
            const int64_t fc = fv ? fe : nf - 1;
            const T xs = (rv && fv) ? (CENTER ? xr[fc] - mux[fc] : xr[fc]) : T(0);
            const T ys = (rv && fv) ? (CENTER ? yr[fc] - muy[fc] : yr[fc]) : T(0);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const T bxv = fv ? VQx[qidx<KP>(fc, nb * 16 + n)] : T(0);
                const T byv = fv ? VQy[qidx<KP>(fc, nb * 16 + n)] : T(0);
                accx[0][nb] = Mfma<T>::fma(xs, bxv, accx[0][nb]);
                accy[0][nb] = Mfma<T>::fma(ys, byv, accy[0][nb]);
            }
        }
    }
}

// P and Q of row tile blk (16 rows, from pt / qt) to memory, and the tile's
// row of Gram partials (raw players, FP64): lower triangle of b V^T A_t V and
// the diagonal of b V^T B_t V (without the ridge); ICA: lower triangles of
// P^T diag(n) P and P^T P, and sum_r ||x_r||^2 (nrow: the rows' ||x_r||^2)
// Entry e of a row tile's Gram partial row (CCA / GENERAL; raw players,
// FP64 products summed over the 16 rows in order): e < TRI the lower
// triangle of b V^T A_t V, else the diagonal of b V^T B_t V (no ridge)
template <typename T, int KP, int KIND>
__device__ __forceinline__ double gram_entry(const T (*pt)[KP], const T (*qt)[KP], int e)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    double s = 0.0;
    if (e < TRI) {
        int i, j;
        tri_ij(e, i, j);
        for (int r = 0; r < 16; ++r) {
            if (KIND == kKindCCA)
                s += (double)pt[r][i] * (double)qt[r][j] + (double)qt[r][i] * (double)pt[r][j];
            else
                s += (double)qt[r][i] * (double)qt[r][j];
        }
    } else {
        const int i = e - TRI;
        for (int r = 0; r < 16; ++r) {
            if (KIND == kKindCCA)
                s += (double)pt[r][i] * (double)pt[r][i] + (double)qt[r][i] * (double)qt[r][i];
            else
                s += (double)pt[r][i] * (double)pt[r][i];
        }
    }
    return s;
}

template <typename T, int KP, int KIND>
__device__ __forceinline__ void fwd_store(const StepArgs &a, int blk, const T (*pt)[KP],
                                          const T (*qt)[KP], const T *nrow, int tid)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    constexpr int GW = TRI + KP;
    constexpr bool ICA = KIND == kKindICA;
    constexpr int GWF = ICA ? 2 * TRI + 1 : GW;
    const int64_t r0 = (int64_t)blk * 16;
    SGEP_G T *PQ = (SGEP_G T *)a.P, *QQ = (SGEP_G T *)a.Q;
    // P, Q of these 16 rows: one contiguous quad-interleaved block
    for (int e = tid; e < 16 * KP; e += kNT) {
        const int rq = e / (4 * KP), c = (e / 4) % KP, r = 4 * rq + (e & 3);
        if (r0 + r < a.b) {
            PQ[r0 * KP + e] = pt[r][c];
            QQ[r0 * KP + e] = qt[r][c];
        }
    }
    for (int e = tid; e < GWF; e += kNT) {
        double s = 0.0;
        if (ICA) {
            if (e < 2 * TRI) {
                int i, j;
                tri_ij(e < TRI ? e : e - TRI, i, j);
                for (int r = 0; r < 16; ++r)
                    s += (double)pt[r][i] * (double)(e < TRI ? qt[r][j] : pt[r][j]);
            } else {
                for (int r = 0; r < 16; ++r)
                    s += (double)nrow[r];
            }
        } else {
            s = gram_entry<T, KP, KIND>(pt, qt, e);
        }
        ((SGEP_G double *)a.gram_part)[(int64_t)blk * GWF + e] = s;
    }
}

// Forward body: workgroup blk takes rows 16 blk .. 16 blk + 15; the four waves
// split the features.  Workgroup blk == n_fwd reduces the norm / parent
// partials of the current state and advances the step counter.
template <typename T, int KP, int KIND, bool LOWREG = false, bool CENTER = false>
__device__ __forceinline__ void fwd_body(const StepArgs &a, int blk)
{
    typedef typename Mfma<T>::acc Acc;
    constexpr int NB = KP / 16;
    constexpr int TRI = KP * (KP + 1) / 2;
    constexpr int GW = TRI + KP;
    constexpr bool ICA = KIND == kKindICA;
    __shared__ T red[4][16 * KP];
    __shared__ T pt[16][KP], qt[16][KP];
    __shared__ T rn[ICA ? 16 : 1][16], nrow[16]; // ICA: ||x_r||^2 partials and totals

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kk = lane >> 4, n = lane & 15;
    if (blk == a.n_fwd) {
        // norm / parent-term totals of the current state (sum over the
        // previous backward pass's tiles, fixed order); advance t
        colsum((const SGEP_G double *)a.stat_part, a.n_tx + a.n_ty, GW, GW, a.stat_tot, tid, kNT);
        if (tid == 0)
            ((SGEP_G Coef *)a.coef)->t += 1.0; // read by k_bwd only, after this kernel has finished
        return;
    }
    const int64_t r0 = (int64_t)blk * 16;
    const bool rv = r0 + n < a.b;
    const int64_t row = rv ? r0 + n : a.b - 1; // valid address; zeroed through rv
    const bool vec_ok = a.vec_ok != 0;
    const SGEP_G T *X = (const SGEP_G T *)a.X, *Y = (const SGEP_G T *)a.Y;
    const SGEP_G T *VQ = (const SGEP_G T *)a.V;

    Acc aP[2][NB], aQ[2][NB];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            aP[h][nb] = Acc{0, 0, 0, 0};
            aQ[h][nb] = Acc{0, 0, 0, 0};
        }
    // view y's players start at feature dxp (a multiple of 4) for CCA
    const SGEP_G T *VQy = KIND == kKindCCA ? VQ + a.dxp * KP : VQ;
    const int64_t nfy = KIND == kKindCCA ? a.dy : a.dx;
    // centring: running means at the views' storage positions (GENERAL: view
    // y's at +ldv)
    const SGEP_G T *mux = (const SGEP_G T *)a.mu;
    const SGEP_G T *muy = CENTER ? mux + (KIND == kKindCCA ? a.dxp : a.ldv) : nullptr;
    T sq = T(0); // ICA: this lane's part of its row's squared norm
    if constexpr (ICA) {
        fwd_view<T, KP, false, true>(X, a.ldx, a.dx, row, rv, vec_ok, VQ, lane, w, aP, nullptr,
                                     &sq);
    } else if (nfy == a.dx) {
        fwd_view2<T, KP, KIND != kKindCCA, LOWREG, CENTER>(X, a.ldx, Y, a.ldy, a.dx, row, rv,
                                                           vec_ok, VQ, VQy, lane, w, aP, aQ,
                                                           mux, muy);
    } else {
        fwd_view<T, KP, CENTER>(X, a.ldx, a.dx, row, rv, vec_ok, VQ, lane, w, aP, mux);
        fwd_view<T, KP, CENTER>(Y, a.ldy, nfy, row, rv, vec_ok, VQy, lane, w, aQ, muy);
    }

    // sum the accumulator sets and the four waves' tiles in a fixed order
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const Acc s = aP[0][nb] + aP[1][nb];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[w][Mfma<T>::drow(kk, r) * KP + nb * 16 + n] = s[r];
    }
    __syncthreads();
    for (int e = tid; e < 16 * KP; e += kNT)
        (&pt[0][0])[e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
    __syncthreads();
    if constexpr (ICA) {
        // Q = diag(||x_r||^2) P: row norms from the lanes' partials, fixed order
        rn[4 * w + kk][n] = sq;
        __syncthreads();
        if (tid < 16) {
            T s = T(0);
            for (int q = 0; q < 16; ++q)
                s += rn[q][tid];
            nrow[tid] = s;
        }
        __syncthreads();
        for (int e = tid; e < 16 * KP; e += kNT)
            (&qt[0][0])[e] = nrow[e / KP] * (&pt[0][0])[e];
        __syncthreads();
    } else {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const Acc s = aQ[0][nb] + aQ[1][nb];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                red[w][Mfma<T>::drow(kk, r) * KP + nb * 16 + n] = s[r];
        }
        __syncthreads();
        for (int e = tid; e < 16 * KP; e += kNT)
            (&qt[0][0])[e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
        __syncthreads();
    }
    fwd_store<T, KP, KIND>(a, blk, pt, qt, nrow, tid);
}

template <typename T, int KP, int KIND, bool CENTER = false>
__global__ void __launch_bounds__(kNT) k_fwd(StepArgs a)
{
    fwd_body<T, KP, KIND, false, CENTER>(a, blockIdx.x);
}

// Stamped words for exchanges inside one launch: the high 32 bits carry the
// iteration stamp, the low 32 bits one half of the value (FP32: all of it;
// FP64: word 0 the low half, word 1 the high half).  A reader polls the
// words themselves with device-coherent loads until every stamp matches, so
// no completion wait, counter or flag is needed; words are written with
// single 64-bit device-coherent stores, so a matching stamp implies its value.
template <typename T> struct Stamped;
template <> struct Stamped<float> {
    static constexpr int N = 1; // words per value
    static __device__ __forceinline__ void put(unsigned long long *w, float v, unsigned st)
    {
        __hip_atomic_store(w, ((unsigned long long)st << 32) | __float_as_uint(v),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // false if the bounded wait gave up (value then zero).  budget: the polls
    // the calling thread has left for all its waits of the launch; once it is
    // spent every further wait looks once and gives up
    static __device__ __forceinline__ bool get(const unsigned long long *w, unsigned st, float &v,
                                               int &budget)
    {
        unsigned long long x;
        for (;;) {
            x = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((unsigned)(x >> 32) == st)
                break;
            if (--budget < 0) {
                budget = 0;
                v = 0.0f;
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        v = __uint_as_float((unsigned)x);
        return true;
    }
};
template <> struct Stamped<double> {
    static constexpr int N = 2;
    static __device__ __forceinline__ void put(unsigned long long *w, double v, unsigned st)
    {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        const unsigned long long hs = (unsigned long long)st << 32;
        __hip_atomic_store(w, hs | (b & 0xffffffffull), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(w + 1, hs | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    static __device__ __forceinline__ bool get(const unsigned long long *w, unsigned st, double &v,
                                               int &budget)
    {
        unsigned long long x[2];
        for (int h = 0; h < 2; ++h) {
            for (;;) {
                x[h] = __hip_atomic_load(w + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((unsigned)(x[h] >> 32) == st)
                    break;
                if (--budget < 0) {
                    budget = 0;
                    v = 0.0;
                    return false;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        v = __longlong_as_double((long long)((x[1] << 32) | (x[0] & 0xffffffffull)));
        return true;
    }
};

// Per-view forward (CCA handles with the row-split backward): two
// workgroups per 16-row tile, 2 blk streaming view x's features of the rows
// and 2 blk + 1 view y's, so twice as many CUs stream the minibatch as with
// k_fwd (same chunk order and accumulators as k_fwd's per-view pass, hence
// the same P and Q).  The x workgroup stores P and publishes it as stamped
// words; the y workgroup stores Q, reads P from the stamped words and writes
// the tile's Gram partials as k_fwd does.  The stamp is this iteration's
// number, one past the stamp the previous backward launch left in a.cflag.
// Workgroup 2 n_fwd is k_fwd's norm-totals workgroup.
template <typename T, int KP, bool CENTER = false>
__global__ void __launch_bounds__(kNT) k_fwds(StepArgs a)
{
    typedef typename Mfma<T>::acc Acc;
    constexpr int NB = KP / 16;
    constexpr int GW = KP * (KP + 1) / 2 + KP;
    constexpr int TS = 16 * KP; // elements of one tile of P or Q
    __shared__ T red[4][TS];
    __shared__ T pt[16][KP], qt[16][KP];
    __shared__ int bad;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kk = lane >> 4, n = lane & 15;
    const int g = blockIdx.x;
    if (g == 2 * a.n_fwd) {
        colsum((const SGEP_G double *)a.stat_part, a.n_tx + a.n_ty, GW, GW, a.stat_tot, tid, kNT);
        if (tid == 0)
            ((SGEP_G Coef *)a.coef)->t += 1.0;
        return;
    }
    const unsigned stamp = (unsigned)*(const SGEP_G unsigned long long *)a.cflag + 1u;
    const int blk = g >> 1;
    const bool vy = (g & 1) != 0;
    const int64_t r0 = (int64_t)blk * 16;
    const bool rv = r0 + n < a.b;
    const int64_t row = rv ? r0 + n : a.b - 1; // valid address; zeroed through rv
    const SGEP_G T *Xv = (const SGEP_G T *)(vy ? a.Y : a.X);
    const SGEP_G T *VQ = (const SGEP_G T *)a.V + (vy ? a.dxp * KP : 0);
    const SGEP_G T *mu = CENTER ? (const SGEP_G T *)a.mu + (vy ? a.dxp : 0) : nullptr;
    Acc acc[2][NB];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            acc[h][nb] = Acc{0, 0, 0, 0};
    fwd_view<T, KP, CENTER>(Xv, vy ? a.ldy : a.ldx, vy ? a.dy : a.dx, row, rv, a.vec_ok != 0, VQ,
                            lane, w, acc, mu);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const Acc s = acc[0][nb] + acc[1][nb];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[w][Mfma<T>::drow(kk, r) * KP + nb * 16 + n] = s[r];
    }
    if (tid == 0)
        bad = 0;
    __syncthreads();
    // this view's 16 x KP product (the four waves' tiles summed in order),
    // one contiguous quad-interleaved block
    SGEP_G T *out = (SGEP_G T *)(vy ? a.Q : a.P) + r0 * KP;
    unsigned long long *pw = (unsigned long long *)a.fpart + (int64_t)blk * TS * Stamped<T>::N;
    int budget = kSpinMax; // polls left for all of this thread's waits
    for (int e = tid; e < TS; e += kNT) {
        const int rq = e / (4 * KP), c = (e / 4) % KP, r = 4 * rq + (e & 3);
        const int ti = r * KP + c;
        const T v = red[0][ti] + red[1][ti] + red[2][ti] + red[3][ti];
        if (r0 + r < a.b)
            out[e] = v;
        if (vy) {
            qt[r][c] = v;
            T p;
            if (!Stamped<T>::get(pw + e * Stamped<T>::N, stamp, p, budget))
                bad = 1;
            pt[r][c] = p;
        } else {
            Stamped<T>::put(pw + e * Stamped<T>::N, v, stamp);
        }
    }
    if (!vy)
        return;
    __syncthreads();
    if (tid == 0 && bad)
        atomicOr(&((Coef *)a.coef)->status, kStatusSync);
    for (int e = tid; e < GW; e += kNT)
        ((SGEP_G double *)a.gram_part)[(int64_t)blk * GW + e] = gram_entry<T, KP, kKindCCA>(pt, qt, e);
}


// ---------------------------------------------------------------------------
// Coefficients of one iteration, as the backward epilogue uses them: with the
// totals ss of the state entering the iteration (||V_i||^2, V_i^T G_j) and
// the minibatch Gram totals gs (lower b V^T A_t V, diagonal of b V^T B_t V,
// raw players), inv_i = 1/||V_i||, s_j = max(v_j^T G_j, rho), the penalty
// weights T_ij = (M_A)_ij / s_j (j < i), m_B,i, m_A,i - c_i with
// c_i = sum_{j<i} T_ij C_ij, the step size and the Adam bias corrections.
// Computed either by four extra waves of the backward workgroup while the
// main waves stream the minibatch (few workgroups), or once per iteration by
// k_coef (many workgroups); both run the functions below, so both give the
// same bits.
// ---------------------------------------------------------------------------
constexpr int kModePre = 0;  // backward reads the block k_coef wrote
constexpr int kModeSpec = 1; // backward computes it on four extra waves
constexpr int kModePart = 2; // one row slice of the products -> partial tiles
constexpr int kModeFin = 3;  // sum of the partial tiles, block from k_coef, epilogue
constexpr int kModeIca1 = 4; // ICA: S1 = X^T P, S2 = X^T Q to memory, S1^T S1 partials
constexpr int kModeIca2 = 5; // ICA: S3 = X^T R, A-side = S2 - tr S1 - 2 S3, epilogue
constexpr int kModeFused = 6; // one row slice; the tile's last slice sums them and runs the epilogue

template <typename T, int KP> struct CoefTile {
    T Tl[KP * KP];            // T_ij, row i
    T mB[KP], mAc[KP], inv[KP];
    T eta, c1, c2, pad;       // eta_t, 1 - b1^t, 1 - b2^t; pad: ICA tr(C_t)
};

// Alg. 3 estimate of v_j^T B v_j from its log-space variable z
__device__ __forceinline__ double smooth_s(double lrho, double lspan, double z)
{
    return exp(lrho + lspan / (1.0 + exp(-z)));
}

// inv_i and s_i (thread q < KP) of iteration t: s_i = max(v_i^T G_i, rho)
// (Alg. 2) or the smooth estimate from z_i (Alg. 3)
template <int KP>
__device__ __forceinline__ void coef_norms(const StepArgs &a, const double *ss, double *dInv,
                                           double *dS, double t, int q)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    if (q < KP) {
        const int i = q;
        double inv = 0.0, s = 1.0;
        if (i < a.k) {
            inv = 1.0 / sqrt(ss[TRI + i]);
            if (a.smooth) {
                const SGEP_G Coef *cg = (const SGEP_G Coef *)a.coef;
                s = smooth_s(a.lrho, a.lspan, cg->z[(int64_t)t & 1][i]);
            } else {
                s = ss[tri_idx(i, i)] * inv; // v_i^T G_i with the unit v_i
                if (!(s >= a.rho))
                    s = a.rho;
            }
        }
        dInv[i] = inv;
        dS[i] = s;
    }
}

// T_ij = (M_A)_ij / s_j with (M_A)_ij = b^{-1} inv_i inv_j (raw Gram)_ij, in
// the element type (Tl) and in FP64 (Td)
template <typename T, int KP>
__device__ __forceinline__ void coef_T(const StepArgs &a, const double *gs, const double *dInv,
                                       const double *dS, T *Tl, double *Td, int q, int nthr)
{
    const double ib = 1.0 / (double)a.b;
    for (int e = q; e < KP * KP; e += nthr) {
        const int i = e / KP, j = e % KP;
        double v = 0.0;
        if (i < a.k && j < i)
            v = gs[tri_idx(i, j)] * dInv[i] * dInv[j] * ib / dS[j];
        Tl[e] = (T)v;
        Td[e] = v;
    }
}

// Terms of the iteration that depend only on its number t: eta_t and the Adam
// bias corrections (thread q == 0), and the running means the writer updates
// (thread q < KP, into ema[2 KP]); read before the Gram totals are known
template <typename T, int KP>
__device__ __forceinline__ void coef_early(const StepArgs &a, double t, CoefTile<T, KP> &C,
                                           double *ema, bool writer, int q)
{
    if (q == 0) {
        C.eta = (T)eta_at(a, t);
        C.c1 = (T)(1.0 - pow(a.adam_b1, t));
        C.c2 = (T)(1.0 - pow(a.adam_b2, t));
        C.pad = T(0);
    }
    if (writer && q < KP) {
        const SGEP_G Coef *cg = (const SGEP_G Coef *)a.coef;
        ema[q] = cg->ema_a[q];
        ema[KP + q] = cg->ema_b[q];
    }
}

// m_A, m_B, c per player (thread q < KP), the uniform terms (q == 0), and --
// by the one writer of the iteration -- the running means, clip count,
// status word and the public coefficient fields
template <typename T, int KP, int KIND>
__device__ __forceinline__ void coef_rows(const StepArgs &a, const double *gs, const double *ss,
                                          const double *dInv, const double *dS, const double *Td,
                                          const double *ema, double t, CoefTile<T, KP> &C,
                                          bool writer, int q)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    const double ib = 1.0 / (double)a.b;
    SGEP_G Coef *cw = (SGEP_G Coef *)a.coef;
    if (q < KP) {
        const int i = q;
        double mA = 0.0, mB = 0.0, c = 0.0;
        if (i < a.k) {
            const double ii2 = dInv[i] * dInv[i];
            mA = gs[tri_idx(i, i)] * ii2 * ib;
            mB = gs[TRI + i] * ii2 * ib + (KIND == kKindCCA ? 0.0 : a.eps_reg);
#pragma unroll
            for (int j = 0; j < KP - 1; ++j) // j < i, in order; unrolled so the LDS reads overlap
                if (j < i)
                    c += Td[i * KP + j] * (ss[tri_idx(i, j)] * dInv[i]); // T_ij C_ij
        }
        C.mB[i] = (T)mB;
        C.mAc[i] = (T)(mA - c);
        C.inv[i] = (T)dInv[i];
        if (writer) {
            if (i < a.k) {
                cw->ema_a[i] = ema[i] + a.gamma * (mA - ema[i]);
                cw->ema_b[i] = ema[KP + i] + a.gamma * (mB - ema[KP + i]);
                const double craw = ss[tri_idx(i, i)] * dInv[i];
                if (a.smooth) {
                    // Alg. 3: z_i += gamma (c_i - s_i) s_i (log nu - log rho) sig (1 - sig)
                    const double z = cw->z[(int64_t)t & 1][i];
                    const double sg = 1.0 / (1.0 + exp(-z));
                    const double zn =
                        z + a.gamma * (craw - dS[i]) * dS[i] * a.lspan * sg * (1.0 - sg);
                    cw->z[((int64_t)t + 1) & 1][i] = zn;
                    if (!isfinite(zn))
                        atomicOr((int *)&cw->status, kStatusNonFinite);
                } else if (!(craw >= a.rho)) {
                    atomicAdd((int *)&cw->clip_count, 1);
                }
                if (!isfinite(mA) || !isfinite(mB) || !isfinite(c) || !isfinite(dInv[i]) ||
                    !(dInv[i] > 0.0) || !isfinite(craw))
                    atomicOr((int *)&cw->status, kStatusNonFinite);
            }
            cw->mA[i] = mA;
            cw->mB[i] = mB;
            cw->c[i] = c;
            cw->s[i] = dS[i];
            if (i == 0) {
                cw->eta = eta_at(a, t);
                cw->gamma = a.gamma;
            }
        }
    }
}

// k_coef: one workgroup computes the iteration's coefficient block into
// a.cpre (used with the backward mode kModePre)
template <typename T, int KP, int KIND, int R = 32, bool PRESUM = false>
__device__ __forceinline__ void coef_body(const StepArgs &a)
{
    constexpr int W = KP * (KP + 1) / 2 + KP;
    constexpr int NC = (int)(sizeof(CoefTile<T, KP>) / sizeof(T));
    __shared__ double gs[W], ss[W], dInv[KP], dS[KP], Td[KP * KP], ema[2 * KP];
    __shared__ CoefTile<T, KP> C;
    const int tid = threadIdx.x;
    const double t = ((const SGEP_G Coef *)a.coef)->t; // this iteration's number (k_fwd)
    // the t-dependent terms (three FP64 pow) on the last wave, which has no
    // column of the sums below (W <= kNT - 64 for KP <= 16; otherwise the
    // wave also sums columns and only the placement changes)
    if (tid >= kNT - 64)
        coef_early<T, KP>(a, t, C, ema, true, tid - (kNT - 64));
    for (int e = tid; e < W; e += kNT)
        ss[e] = ((const SGEP_G double *)a.stat_tot)[e];
    if constexpr (KIND == kKindICA) {
        // b V^T A_t V = P^T diag(n) P - tr(C_t) P^T P - (2 / b) S1^T S1 (S1 = X^T P),
        // b diag(V^T B_t V) = diag(P^T P) (before the ridge); tr(C_t) = sum_r n_r / b
        constexpr int TRI = KP * (KP + 1) / 2;
        __shared__ double gi[2 * TRI + 1], gb2[TRI];
        colsum((const SGEP_G double *)a.gram_part, a.n_fwd, 2 * TRI + 1, 2 * TRI + 1, gi, tid,
               kNT);
        colsum((const SGEP_G double *)a.bb_part, a.n_tx, TRI, TRI, gb2, tid, kNT);
        __syncthreads();
        const double ib = 1.0 / (double)a.b, tr = gi[2 * TRI] * ib;
        for (int e = tid; e < TRI; e += kNT)
            gs[e] = gi[e] - tr * gi[TRI + e] - 2.0 * ib * gb2[e];
        for (int i = tid; i < KP; i += kNT)
            gs[TRI + i] = gi[TRI + tri_idx(i, i)];
        if (tid == 0)
            C.pad = (T)tr; // read by the second backward pass
    } else if (PRESUM) { // the totals of k_coefa, summed in the same order
        for (int e = tid; e < W; e += kNT)
            gs[e] = ((const SGEP_G double *)a.gsum)[e];
    } else {
        colsum<R>((const SGEP_G double *)a.gram_part, a.n_fwd, W, W, gs, tid, kNT);
    }
    __syncthreads();
    coef_norms<KP>(a, ss, dInv, dS, t, tid);
    __syncthreads();
    coef_T<T, KP>(a, gs, dInv, dS, C.Tl, Td, tid, kNT);
    __syncthreads();
    coef_rows<T, KP, KIND>(a, gs, ss, dInv, dS, Td, ema, t, C, true, tid);
    __syncthreads();
    // the block for the backward epilogue (kModePre / kModeFin, a later launch)
    SGEP_G T *out = (SGEP_G T *)a.cpre;
    for (int e = tid; e < NC; e += kNT)
        out[e] = (&C.Tl[0])[e];
    if (a.xw) { // fused row split: the last slices read the block as stamped words
        unsigned long long *cw = (unsigned long long *)a.xw + a.xw_coef;
        for (int e = tid; e < NC; e += kNT)
            Stamped<T>::put(cw + e * Stamped<T>::N, (&C.Tl[0])[e], (unsigned)t);
    }
    // this iteration's number: the next per-view forward stamps with t + 1
    if (a.cflag && tid == 0)
        __hip_atomic_store(a.cflag, (unsigned long long)t, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int KP, int KIND>
__global__ void __launch_bounds__(kNT) k_coef(StepArgs a)
{
    coef_body<T, KP, KIND, 64>(a);
}

// Two-stage coefficient kernel for many Gram partials (one CU streams only
// ~30 GB/s): k_coefa sums 16 columns per workgroup over all rows (thread per
// column, rows ascending: the order of colsum, so the totals carry the same
// bits), then k_coefb (one workgroup) computes the block from the totals.
constexpr int kCoefCols = 16;
template <int KP>
__global__ void __launch_bounds__(64) k_coefa(StepArgs a)
{
    constexpr int W = KP * (KP + 1) / 2 + KP;
    const int c0 = blockIdx.x * kCoefCols;
    const int nc = W - c0 < kCoefCols ? W - c0 : kCoefCols;
    colsum<64>((const SGEP_G double *)a.gram_part + c0, a.n_fwd, W, nc, a.gsum + c0,
               threadIdx.x, kCoefCols);
}

template <typename T, int KP, int KIND>
__global__ void __launch_bounds__(kNT) k_coefb(StepArgs a)
{
    coef_body<T, KP, KIND, 32, true>(a);
}

// ICA, second forward pass: R = X (S1 / b) = X C_t V for 16-row tiles (S1 =
// X^T P from the first backward pass, read like V), stored where Q was; the
// extra workgroup n_fwd computes the iteration's coefficient block (it needs
// the S1^T S1 partials of the first backward pass).
template <typename T, int KP>
__global__ void __launch_bounds__(kNT) k_fwd2(StepArgs a)
{
    typedef typename Mfma<T>::acc Acc;
    constexpr int NB = KP / 16;
    const int blk = blockIdx.x;
    if (blk == a.n_fwd) {
        coef_body<T, KP, kKindICA>(a);
        return;
    }
    __shared__ T red[4][16 * KP];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kk = lane >> 4, n = lane & 15;
    const int64_t r0 = (int64_t)blk * 16;
    const bool rv = r0 + n < a.b;
    const int64_t row = rv ? r0 + n : a.b - 1;
    Acc aR[2][NB];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            aR[h][nb] = Acc{0, 0, 0, 0};
    fwd_view<T, KP>((const SGEP_G T *)a.X, a.ldx, a.dx, row, rv, a.vec_ok != 0,
                    (const SGEP_G T *)a.S1, lane, w, aR);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const Acc s = aR[0][nb] + aR[1][nb];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[w][Mfma<T>::drow(kk, r) * KP + nb * 16 + n] = s[r];
    }
    __syncthreads();
    const T ib = (T)(1.0 / (double)a.b);
    SGEP_G T *RQ = (SGEP_G T *)a.Q;
    for (int e = tid; e < 16 * KP; e += kNT) {
        const int rq = e / (4 * KP), c = (e / 4) % KP, r = 4 * rq + (e & 3);
        const int ti = r * KP + c;
        if (r0 + r < a.b)
            RQ[r0 * KP + e] = (red[0][ti] + red[1][ti] + red[2][ti] + red[3][ti]) * ib;
    }
}

// ---------------------------------------------------------------------------
// Backward products + fused update for a tile of FT = 16 MB features.
// Rows go in groups of 16; wave w takes groups w, w + 4, ...  Within a group
// the four MFMAs j = 0..3 cover rows 16 g + 4 (l/16) + j: lane l supplies
// A = X[that row][f0 + MB (l%16) + jm] for M-block jm (MB consecutive features
// in one load) and B = element j of the 4 consecutive rows 16 g + 4 (l/16) ..
// of P^T / Q^T for player l % 16 (one 16-byte load), so M-block jm, M-row m
// holds feature f0 + MB m + jm.  Batches of UB groups issue all loads before
// any MFMA; the ragged last group runs masked.
//
// MODE kModeSpec: the workgroup has eight waves; waves 4..7 reduce the Gram
// partials and compute the coefficients while waves 0..3 run the main loop.
// MODE kModePre: four waves; the coefficient block comes from k_coef.
// MODE kModePart: four waves over row slice `split` of nsplit (16-row groups
// in contiguous ranges); the reduced products go to the partial buffer.
// MODE kModeFin: four waves; the products are the fixed-order sum of the
// slices' partials, the coefficient block comes from k_coef.
// ---------------------------------------------------------------------------
template <typename T, int KP, int MB, int KIND, int OPT, int MODE, bool LOWREG = false,
          bool CENTER = false>
__device__ __forceinline__ void bwd_body(const StepArgs &a, int tile, int split = 0)
{
    typedef typename Mfma<T>::acc Acc;
    constexpr int NB = KP / 16;
    constexpr int FT = 16 * MB;
    constexpr int TRI = KP * (KP + 1) / 2;
    constexpr int W = TRI + KP; // width of both partial kinds
    constexpr int XPG = (KIND == kKindGeneral ? 8 : 4) * MB; // X registers per group
    // loads in flight per batch: ~128 VGPRs; ~192 for the smallest player
    // tile with eight waves (kModeSpec; one workgroup per CU, fewer round
    // trips, still within 256 VGPRs); ~64 with LOWREG (more workgroups per
    // CU).  The order of the row groups, hence the sums, is the same.
    constexpr bool BIG = MODE == 1 && KP * (int)sizeof(T) <= 64;
    constexpr int UB0 = (LOWREG ? 256 : (BIG ? 768 : 512)) / ((XPG + 8 * NB) * (int)sizeof(T));
    constexpr int UB = UB0 < 1 ? 1 : (UB0 > 16 ? 16 : UB0);
    constexpr int EPT = FT * KP / kNT; // epilogue elements per thread
    static_assert(EPT * kNT == FT * KP, "tile must be a multiple of the workgroup");
    constexpr bool SPEC = MODE == kModeSpec;
    constexpr int NTH = SPEC ? 2 * kNT : kNT; // threads of the workgroup
    constexpr int NC = (int)(sizeof(CoefTile<T, KP>) / sizeof(T));
    constexpr bool PART = MODE == kModePart, FIN = MODE == kModeFin;
    constexpr bool ICA1 = MODE == kModeIca1, ICA2 = MODE == kModeIca2;
    constexpr bool FUSED = MODE == kModeFused;
    static_assert(!(FUSED && CENTER), "the fused row split runs without centring");
    // no coefficient block read from memory at the start (FUSED: read later)
    constexpr bool NOCOEF = SPEC || PART || ICA1 || FUSED;
    constexpr bool TWOX = KIND == kKindGeneral;   // two views per feature tile
    constexpr int CPT = NOCOEF ? 1 : (NC + kNT - 1) / kNT;
    __shared__ T red[4][FT * KP];
    __shared__ T avt[FT * KP], bvt[FT * KP], gt[FT * KP];
    __shared__ CoefTile<T, KP> C;
    // centring: per (wave, lane group) column sums of the centred views, then
    // their fixed-order totals (A side, B side)
    __shared__ T csum[2][CENTER ? 16 : 1][CENTER ? FT : 1];
    __shared__ T ctot[2][CENTER ? FT : 1];
    constexpr int PSTR = 2 * FT * KP + 2 * FT; // partial block of one (tile, slice)
    __shared__ double gs[SPEC ? W : 1], ss[SPEC ? W : 1], Td[SPEC ? KP * KP : 1];
    __shared__ double dInv[KP], dS[KP], ema[2 * KP];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6); // wave index, scalar
    const bool main_w = !SPEC || w < 4;
    const int kk = lane >> 4, m = lane & 15;
    const bool vec_ok = a.vec_ok != 0;
    const SGEP_G T *X = (const SGEP_G T *)a.X, *Y = (const SGEP_G T *)a.Y;
    const SGEP_G T *PQ = (const SGEP_G T *)a.P, *QQ = (const SGEP_G T *)a.Q;

    const SGEP_G T *Xa;      // view multiplying the A-side operand
    const SGEP_G T *Xb;      // view multiplying the B-side operand
    int64_t lda, ldb, nf, fbase, f0;
    const SGEP_G T *opA, *opB;
    if (KIND == kKindCCA) {
        if (tile < a.n_tx) { // x features: A_t V = X^T Q / b, B_t V = X^T P / b
            Xa = X; lda = a.ldx; nf = a.dx; fbase = 0; f0 = (int64_t)tile * FT;
            opA = QQ; opB = PQ;
        } else {             // y features: A_t V = Y^T P / b, B_t V = Y^T Q / b
            Xa = Y; lda = a.ldy; nf = a.dy; fbase = a.dxp; f0 = (int64_t)(tile - a.n_tx) * FT;
            opA = PQ; opB = QQ;
        }
        Xb = Xa; ldb = lda;
    } else if (KIND == kKindICA) { // first pass: A side X^T Q = S2, B side X^T P = S1;
                                   // second pass: A side X^T R = S3 (R stored in Q)
        Xa = X; lda = a.ldx; Xb = X; ldb = a.ldx;
        nf = a.dx; fbase = 0; f0 = (int64_t)tile * FT;
        opA = QQ; opB = PQ;
    } else {                 // GENERAL: A_t V = Y^T Q / b, B_t V = X^T P / b + eps V
        Xa = Y; lda = a.ldy; Xb = X; ldb = a.ldx;
        nf = a.dx; fbase = 0; f0 = (int64_t)tile * FT;
        opA = QQ; opB = PQ;
    }

    // epilogue operands of this thread's elements: element e of the tile's
    // contiguous quad-interleaved block, i.e. feature f0 + 4 (e / 4KP) + e % 4
    // of player (e / 4) % KP
    SGEP_G T *VQ = (SGEP_G T *)a.V, *GQ = (SGEP_G T *)a.G;
    SGEP_G T *Am = (SGEP_G T *)a.Am, *As = (SGEP_G T *)a.As;
    const int64_t tbase = (fbase + f0) * KP; // first element of this tile's block
    // centring: running means of the A-side view (Xa) and the B-side view (Xb)
    SGEP_G T *muA = (SGEP_G T *)a.mu + (KIND == kKindCCA ? fbase : a.ldv);
    SGEP_G T *muB = (SGEP_G T *)a.mu + fbase;
    T ma[MB], mbm[MB], sa[MB], sb[MB]; // lane's means; its sums of the centred values
    T pv[EPT], pg[EPT], pm[EPT], ps[EPT];
    T cpr[CPT]; // kModePre: this thread's elements of the coefficient block
    typedef typename Mfma<T>::acc Acc2;
    Acc2 aA[2][MB][NB], aB[2][MB][NB];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < MB; ++j)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                aA[h][j][nb] = Acc2{0, 0, 0, 0};
                aB[h][j][nb] = Acc2{0, 0, 0, 0};
            }
    double t_it = 0.0; // helper waves: this iteration's number (set by k_fwd)
    if (main_w) {
    if (!NOCOEF) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int e = tid + q * kNT;
            cpr[q] = e < NC ? ((const SGEP_G T *)a.cpre)[e] : T(0);
        }
    }
#pragma unroll
    for (int q = 0; q < ((PART || ICA1) ? 0 : EPT); ++q) {
        const int e = tid + q * kNT;
        const int fl = 4 * (e / (4 * KP)) + (e & 3);
        const bool ok = f0 + fl < nf;
        const int64_t si = tbase + e;
        pg[q] = ok ? GQ[si] : T(0);
        pv[q] = ok ? VQ[si] : T(0);
        if (OPT == kOptAdam) {
            pm[q] = ok ? Am[si] : T(0);
            ps[q] = ok ? As[si] : T(0);
        }
    }

    // ---- main loop: raw X^T Q and X^T P over all rows ----
    const int64_t fs = f0 + (int64_t)MB * m;
    bool fok[MB];
    int64_t fcl[MB];
#pragma unroll
    for (int jm = 0; jm < MB; ++jm) {
        fok[jm] = fs + jm < nf;
        fcl[jm] = fok[jm] ? fs + jm : nf - 1;
    }
    const bool vrun = vec_ok && fs + MB <= nf;
    // centring: running means of this lane's features
#pragma unroll
    for (int jm = 0; jm < MB; ++jm) {
        ma[jm] = mbm[jm] = sa[jm] = sb[jm] = T(0);
        if (CENTER && !FIN) {
            ma[jm] = muA[fcl[jm]];
            mbm[jm] = !TWOX ? ma[jm] : muB[fcl[jm]];
        }
    }
    const SGEP_G T *pa[NB], *pb[NB]; // player (nb*16 + m): rows r..r+3 at p[r * KP]
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        pa[nb] = opA + 4 * (nb * 16 + m);
        pb[nb] = opB + 4 * (nb * 16 + m);
    }
    const int64_t ngf = a.b / 16; // full 16-row groups
    // this workgroup's groups [gb, ge) (all, or slice `split`) and whether it
    // owns the ragged last group; kModeFin runs no main loop
    int64_t gb = 0, ge = FIN ? 0 : ngf;
    bool ragged = !FIN && ngf * 16 < a.b;
    if (PART || FUSED) {
        const int64_t gps = (ngf + a.nsplit - 1) / a.nsplit;
        gb = split * gps < ngf ? split * gps : ngf;
        ge = gb + gps < ngf ? gb + gps : ngf;
        ragged = ragged && split == a.nsplit - 1;
    }
    for (int64_t g0 = gb + w; g0 < ge; g0 += 4 * UB) {
        T xa[UB][4][MB], xb[UB][4][MB], ba[UB][NB][4], bb[UB][NB][4];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int64_t g = (g0 + 4 * u < ge) ? g0 + 4 * u : g0;
            const int64_t r4 = 16 * g + 4 * kk;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = r4 + j;
                if (vrun) {
                    VecLoad<T, MB>::run(Xa + row * lda + fs, xa[u][j]);
                    if (TWOX)
                        VecLoad<T, MB>::run(Xb + row * ldb + fs, xb[u][j]);
                } else {
#pragma unroll
                    for (int jm = 0; jm < MB; ++jm) {
                        xa[u][j][jm] = Xa[row * lda + fcl[jm]];
                        if (TWOX)
                            xb[u][j][jm] = Xb[row * ldb + fcl[jm]];
                    }
                }
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                VecLoad<T, 4>::run(pa[nb] + r4 * KP, ba[u][nb]);
                if (!ICA2) // the second ICA pass has the A side only
                    VecLoad<T, 4>::run(pb[nb] + r4 * KP, bb[u][nb]);
            }
        }
        __builtin_amdgcn_sched_barrier(0); // all of the batch's loads first
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const bool gv = g0 + 4 * u < ge;
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int jm = 0; jm < MB; ++jm) {
                    const bool ok = gv && fok[jm];
                    const T va = ok ? (CENTER ? xa[u][j][jm] - ma[jm] : xa[u][j][jm]) : T(0);
                    const T vb = !TWOX
                                     ? va
                                     : (ok ? (CENTER ? xb[u][j][jm] - mbm[jm] : xb[u][j][jm])
                                           : T(0));
                    if (CENTER) {
                        sa[jm] += va;
                        if (TWOX)
                            sb[jm] += vb;
                    }
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        aA[j & 1][jm][nb] = Mfma<T>::fma(va, ba[u][nb][j], aA[j & 1][jm][nb]);
                        if (!ICA2)
                            aB[j & 1][jm][nb] =
                                Mfma<T>::fma(vb, bb[u][nb][j], aB[j & 1][jm][nb]);
                    }
                }
        }
    }
    if (ragged && w == (int)((ngf - gb) & 3)) { // the ragged last group, masked
        const int64_t r4 = 16 * ngf + 4 * kk;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t r = r4 + j;
            const bool rv = r < a.b;
            const int64_t row = rv ? r : a.b - 1;
#pragma unroll
            for (int jm = 0; jm < MB; ++jm) {
                const bool ok = rv && fok[jm];
                const T va = ok ? (CENTER ? Xa[row * lda + fcl[jm]] - ma[jm]
                                          : Xa[row * lda + fcl[jm]])
                                : T(0);
                const T vb = !TWOX
                                 ? va
                                 : (ok ? (CENTER ? Xb[row * ldb + fcl[jm]] - mbm[jm]
                                                 : Xb[row * ldb + fcl[jm]])
                                       : T(0));
                if (CENTER) {
                    sa[jm] += va;
                    if (TWOX)
                        sb[jm] += vb;
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const T qa = rv ? opA[qidx<KP>(row, nb * 16 + m)] : T(0);
                    aA[0][jm][nb] = Mfma<T>::fma(va, qa, aA[0][jm][nb]);
                    if (!ICA2) {
                        const T qb = rv ? opB[qidx<KP>(row, nb * 16 + m)] : T(0);
                        aB[0][jm][nb] = Mfma<T>::fma(vb, qb, aB[0][jm][nb]);
                    }
                }
            }
        }
    }
    } else {
        // helper waves (kModeSpec): t-dependent terms, state totals and
        // Gram totals
        const int q = tid - kNT;
        t_it = ((const SGEP_G Coef *)a.coef)->t;
        coef_early<T, KP>(a, t_it, C, ema, tile == 0, q);
        for (int e = q; e < W; e += kNT)
            ss[e] = ((const SGEP_G double *)a.stat_tot)[e];
        colsum((const SGEP_G double *)a.gram_part, a.n_fwd, W, W, gs, q, kNT);
    }

    // cross-wave reduction (fixed order) into natural feature order [fl][i],
    // interleaved with the helper waves' coefficient phases (the barriers are
    // common to all waves)
    __syncthreads();
    if (main_w && !FIN) {
#pragma unroll
        for (int jm = 0; jm < MB; ++jm)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const Acc s = aA[0][jm][nb] + aA[1][jm][nb];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    red[w][(MB * Mfma<T>::drow(kk, r) + jm) * KP + nb * 16 + m] = s[r];
            }
        if constexpr (CENTER) {
#pragma unroll
            for (int jm = 0; jm < MB; ++jm) {
                csum[0][4 * w + kk][MB * m + jm] = sa[jm];
                csum[1][4 * w + kk][MB * m + jm] = sb[jm];
            }
        }
    }
    if (main_w) {
        if (!NOCOEF) {
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const int e = tid + q * kNT;
                if (e < NC)
                    (&C.Tl[0])[e] = cpr[q];
            }
        }
    } else {
        coef_norms<KP>(a, ss, dInv, dS, t_it, tid - kNT);
    }
    __syncthreads();
    if (main_w && !FIN) {
        for (int e = tid; e < FT * KP; e += kNT)
            avt[e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
        if constexpr (CENTER) {
            if (tid < FT) {
                T t0 = T(0), t1 = T(0);
                for (int q = 0; q < 16; ++q) {
                    t0 += csum[0][q][tid];
                    t1 += csum[1][q][tid];
                }
                ctot[0][tid] = t0;
                ctot[1][tid] = t1;
            }
        }
    } else if (FIN) {
        // products (and centred column sums) = fixed-order sums of the row
        // slices' partials
        const SGEP_G T *bp = (const SGEP_G T *)a.bpart + (int64_t)tile * a.nsplit * PSTR;
        for (int e = tid; e < FT * KP; e += kNT) {
            T pa = bp[e], pb2 = bp[FT * KP + e];
            for (int sp = 1; sp < a.nsplit; ++sp) {
                pa += bp[(int64_t)sp * PSTR + e];
                pb2 += bp[(int64_t)sp * PSTR + FT * KP + e];
            }
            avt[e] = pa;
            bvt[e] = pb2;
        }
        if constexpr (CENTER) {
            if (tid < FT) {
                T t0 = bp[2 * FT * KP + tid], t1 = bp[2 * FT * KP + FT + tid];
                for (int sp = 1; sp < a.nsplit; ++sp) {
                    t0 += bp[(int64_t)sp * PSTR + 2 * FT * KP + tid];
                    t1 += bp[(int64_t)sp * PSTR + 2 * FT * KP + FT + tid];
                }
                ctot[0][tid] = t0;
                ctot[1][tid] = t1;
            }
        }
    } else {
        coef_T<T, KP>(a, gs, dInv, dS, C.Tl, Td, tid - kNT, kNT);
    }
    __syncthreads();
    if (main_w && !FIN && !ICA2) {
#pragma unroll
        for (int jm = 0; jm < MB; ++jm)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const Acc s = aB[0][jm][nb] + aB[1][jm][nb];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    red[w][(MB * Mfma<T>::drow(kk, r) + jm) * KP + nb * 16 + m] = s[r];
            }
    }
    if (main_w && !PART && !ICA1) {
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * kNT;
            gt[(4 * (e / (4 * KP)) + (e & 3)) * KP + (e / 4) % KP] = pg[q];
        }
    } else if (!main_w) {
        // this iteration's number t was set by k_fwd
        coef_rows<T, KP, KIND>(a, gs, ss, dInv, dS, Td, ema, t_it, C, tile == 0, tid - kNT);
    }
    __syncthreads();
    if (main_w && !FIN && !ICA2) {
        for (int e = tid; e < FT * KP; e += kNT)
            bvt[e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
    }
    if (ICA2) {
        // B side S1 and A side S2 - tr(C_t) S1 - 2 S3 (each b times the
        // products of the raw players), S1 and S2 from the first pass
        const SGEP_G T *S1 = (const SGEP_G T *)a.S1, *S2 = (const SGEP_G T *)a.S2;
        const T tr = C.pad;
        for (int e = tid; e < FT * KP; e += kNT) {
            const int fl = e / KP, i = e % KP;
            T s1 = T(0), s2 = T(0);
            if (f0 + fl < nf) {
                const int64_t qi = tbase + (int64_t)(fl / 4) * 4 * KP + 4 * i + (fl & 3);
                s1 = S1[qi];
                s2 = S2[qi];
            }
            bvt[e] = s1;
            avt[e] = s2 - tr * s1 - T(2) * avt[e];
        }
    }
    if (ICA1) {
        // S1 = X^T P and S2 = X^T Q of this tile to memory (quad-interleaved),
        // and the tile's partial of S1^T S1 (lower triangle, FP64)
        __syncthreads();
        SGEP_G T *S1 = (SGEP_G T *)a.S1, *S2 = (SGEP_G T *)a.S2;
        for (int e = tid; e < FT * KP; e += kNT) {
            const int fl = 4 * (e / (4 * KP)) + (e & 3), i = (e / 4) % KP;
            if (f0 + fl < nf) {
                S1[tbase + e] = bvt[fl * KP + i];
                S2[tbase + e] = avt[fl * KP + i];
            }
        }
        for (int e = tid; e < TRI; e += kNT) {
            int i, j;
            tri_ij(e, i, j);
            double sum = 0.0;
            for (int fl = 0; fl < FT; ++fl)
                sum += (double)bvt[fl * KP + i] * (double)bvt[fl * KP + j];
            ((SGEP_G double *)a.bb_part)[(int64_t)tile * TRI + e] = sum;
        }
        return;
    }
    if constexpr (FUSED) {
        // slices other than the last publish their products as stamped
        // words and finish; the last slice reads them and the coefficient
        // block (stamped words of workgroup 0) and runs the epilogue
        constexpr int NW = Stamped<T>::N;
        __shared__ int bad;
        const unsigned st = (unsigned)((const SGEP_G Coef *)a.coef)->t; // set by the forward
        unsigned long long *tw =
            (unsigned long long *)a.xw + (int64_t)tile * a.nsplit * (2 * FT * KP) * NW;
        if (tid == 0)
            bad = 0;
        __syncthreads();
        if (split != a.nsplit - 1) {
            unsigned long long *mw = tw + (int64_t)split * (2 * FT * KP) * NW;
            for (int e = tid; e < FT * KP; e += kNT) {
                Stamped<T>::put(mw + e * NW, avt[e], st);
                Stamped<T>::put(mw + (FT * KP + e) * NW, bvt[e], st);
            }
            return;
        }
        const unsigned long long *cw = (const unsigned long long *)a.xw + a.xw_coef;
        int budget = kSpinMax; // polls left for all of this thread's waits
        for (int e = tid; e < NC; e += kNT) {
            T v;
            if (!Stamped<T>::get(cw + e * NW, st, v, budget))
                bad = 1;
            (&C.Tl[0])[e] = v;
        }
        // the slices' products summed in slice order (this slice's from LDS)
        for (int e = tid; e < FT * KP; e += kNT) {
            T pa = T(0), pb2 = T(0);
            for (int sp = 0; sp < a.nsplit; ++sp) {
                T xa = avt[e], xb = bvt[e];
                if (sp != split) {
                    const unsigned long long *ow = tw + (int64_t)sp * (2 * FT * KP) * NW;
                    if (!Stamped<T>::get(ow + e * NW, st, xa, budget) ||
                        !Stamped<T>::get(ow + (FT * KP + e) * NW, st, xb, budget))
                        bad = 1;
                }
                pa = sp == 0 ? xa : pa + xa;
                pb2 = sp == 0 ? xb : pb2 + xb;
            }
            avt[e] = pa; // element e is read and written by this thread only
            bvt[e] = pb2;
        }
        __syncthreads();
        if (tid == 0 && bad)
            atomicOr(&((Coef *)a.coef)->status, kStatusSync);
    }
    if (PART) {
        // this slice's products for the finishing pass
        __syncthreads();
        SGEP_G T *bp = (SGEP_G T *)a.bpart + ((int64_t)tile * a.nsplit + split) * PSTR;
        for (int e = tid; e < FT * KP; e += kNT) {
            bp[e] = avt[e];
            bp[FT * KP + e] = bvt[e];
        }
        if constexpr (CENTER) {
            if (tid < FT) {
                bp[2 * FT * KP + tid] = ctot[0][tid];
                bp[2 * FT * KP + FT + tid] = ctot[1][tid];
            }
        }
        return;
    }

    // ---- fused epilogue (main waves) ----
    __syncthreads();
    const T gam = (T)a.gamma, ibT = (T)(1.0 / (double)a.b);
    const T eps = (T)a.eps_reg;
    const T b1 = (T)a.adam_b1, b2 = (T)a.adam_b2, aeps = (T)a.adam_eps;
    const T eta = C.eta, c1 = C.c1, c2 = C.c2;
    T vnq[EPT], gnq[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        if (!main_w)
            break;
        const int e = tid + q * kNT;
        const int i = (e / 4) % KP, fl = 4 * (e / (4 * KP)) + (e & 3);
        const int64_t f = f0 + fl;
        T vn = 0, gn = 0;
        if (f < nf && i < a.k) {
            const int64_t si = tbase + e;
            const int ti = fl * KP + i;
            const T vh = pv[q] * C.inv[i];
            const T av = avt[ti] * C.inv[i] * ibT;
            T bv = bvt[ti] * C.inv[i] * ibT;
            if (KIND != kKindCCA)
                bv += eps * vh;
            T pen = 0;
            for (int j = 0; j < i; ++j)
                pen += C.Tl[i * KP + j] * gt[fl * KP + j];
            const T grad = (av - pen) * C.mB[i] - bv * C.mAc[i];
            if (OPT == kOptSGD) {
                vn = vh + eta * grad;
            } else {
                const T mm = b1 * pm[q] + (T(1) - b1) * grad;
                const T sq = b2 * ps[q] + (T(1) - b2) * grad * grad;
                Am[si] = mm;
                As[si] = sq;
                vn = vh + eta * (mm / c1) / (sqrt(sq / c2) + aeps);
            }
            const T g0 = pg[q];
            gn = g0 + gam * (bv - g0);
            VQ[si] = vn;
            GQ[si] = gn;
        }
        vnq[q] = vn;
        gnq[q] = gn;
    }
    __syncthreads(); // every read of avt / bvt is done
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        if (!main_w)
            break;
        const int e = tid + q * kNT;
        const int ti = (4 * (e / (4 * KP)) + (e & 3)) * KP + (e / 4) % KP;
        avt[ti] = vnq[q];
        bvt[ti] = gnq[q];
    }
    __syncthreads();
    // this tile's partials of v_i^T G_j (j <= i) and ||v_i||^2 of the new state
    SGEP_G double *sout = (SGEP_G double *)a.stat_part;
    for (int e = tid; e < W; e += NTH) {
        double s = 0.0;
        if (e < TRI) {
            int i, j;
            tri_ij(e, i, j);
            for (int fl = 0; fl < FT; ++fl)
                s += (double)avt[fl * KP + i] * (double)bvt[fl * KP + j];
        } else {
            const int i = e - TRI;
            for (int fl = 0; fl < FT; ++fl)
                s += (double)avt[fl * KP + i] * (double)avt[fl * KP + i];
        }
        sout[(int64_t)tile * W + e] = s;
    }
    // centring: the running means of this tile's features move toward the
    // minibatch means, mu += gamma (xbar - mu) = mu + (gamma / b) sum_r (x_r - mu)
    if constexpr (CENTER) {
        if (tid < FT && f0 + tid < nf) {
            const T g = (T)(a.gamma / (double)a.b);
            muA[f0 + tid] = muA[f0 + tid] + g * ctot[0][tid];
            if (KIND != kKindCCA)
                muB[f0 + tid] = muB[f0 + tid] + g * ctot[1][tid];
        }
    }
}

template <typename T, int KP, int MB, int KIND, int OPT, int MODE, bool CENTER = false>
__global__ void __launch_bounds__(MODE == kModeSpec ? 2 * kNT : kNT) k_bwd(StepArgs a)
{
    bwd_body<T, KP, MB, KIND, OPT, MODE, false, CENTER>(a, xcd_tile(blockIdx.x, gridDim.x));
}

// Row-split backward, first pass: workgroup 0 computes the iteration's
// coefficient block (coef_body; first, as the longest) and workgroups 1..7
// only align the rest to the XCDs; workgroups 8.. compute one row slice of
// one 16-feature tile each.  Partial j = xcd_tile(b - 8) is tile j / nsplit,
// slice j % nsplit, so each XCD takes a contiguous run of tiles with all
// their slices: neighbouring tiles share the 128-byte lines of a minibatch
// row, which are then fetched into one L2 only.  The second pass is k_bwd
// with kModeFin, or (FUSE) none: the last slice of each tile to finish
// sums the slices' products and runs the epilogue itself once workgroup 0
// has published the coefficient block (kModeFused).
template <typename T, int KP, int KIND, bool CENTER = false, bool FUSE = false, int OPT = kOptSGD>
__global__ void __launch_bounds__(kNT) k_bwdp(StepArgs a)
{
    if (blockIdx.x < 8) {
        if (blockIdx.x == 0)
            coef_body<T, KP, KIND, 64>(a); // its column sums are on the critical path
        return;
    }
    const int j = xcd_tile(blockIdx.x - 8, (a.n_tx + a.n_ty) * a.nsplit);
    bwd_body<T, KP, 1, KIND, OPT, FUSE ? kModeFused : kModePart, false, CENTER>(a, j / a.nsplit,
                                                                              j % a.nsplit);
}

// ---------------------------------------------------------------------------
// Initialisation (one workgroup; not on the hot path): normalise the supplied
// players (player-major rows of length ldv, padding zero) to the unit sphere,
// set [Bv]_i = v_i (Alg. 2), and write the norm / parent-term sums of this
// state as row 0 of the stats partials (the other rows are zero).
// ---------------------------------------------------------------------------
template <typename T, int KP>
__global__ void __launch_bounds__(kNT) k_init(T *VQ, T *GQ, int64_t ldv, int k, double *stat0,
                                              int lds, Coef *cw)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    __shared__ double part[kNT];
    __shared__ double nrm[KP];
    const int tid = threadIdx.x;
    for (int i = 0; i < KP; ++i) {
        double s = 0.0;
        for (int64_t f = tid; f < ldv; f += kNT) {
            const double v = (double)VQ[qidx<KP>(f, i)];
            s += v * v;
        }
        part[tid] = s;
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int q = 0; q < kNT; ++q)
                tot += part[q];
            nrm[i] = tot;
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < KP * ldv; e += kNT) {
        const int i = (int)((e / 4) % KP);
        const T v = (i < k) ? (T)((double)VQ[e] / sqrt(nrm[i])) : T(0);
        VQ[e] = v;
        GQ[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < TRI + KP; e += kNT) {
        int i, j;
        if (e < TRI)
            tri_ij(e, i, j);
        else
            i = j = e - TRI;
        double s = 0.0;
        for (int64_t f = 0; f < ldv; ++f)
            s += (double)VQ[qidx<KP>(f, i)] * (double)GQ[qidx<KP>(f, j)]; // G = V
        stat0[e] = s;
        if (e >= TRI && i < k && !(s > 0.0))
            atomicOr(&cw->status, kStatusNonFinite);
    }
}

// Read-out (one workgroup): reduce the latest norm / parent partials, then
// out[i*d + f] = scale_i * S[qidx(storage(f), i)] (column-major FP64) with
// scale_i = 1/||V_i|| for the players (mode 1), additionally 1/sqrt(s_i)
// (mode 2: B-normalised), or 1 (mode 0: the auxiliary variable).  storage(f)
// maps feature f of the concatenated views to its padded position.
template <typename T, int KP>
__global__ void __launch_bounds__(kNT) k_readout(const T *S, int64_t d, int64_t dx, int64_t dxp,
                                                 int64_t ldv, int k, const double *stat_part,
                                                 int n_tiles, int lds, double rho, Coef *cw, int mode,
                                                 double *out)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    constexpr int W = TRI + KP;
    __shared__ double ss[W];
    __shared__ double scale[KP];
    colsum((const SGEP_G double *)stat_part, n_tiles, W, W, ss, threadIdx.x, kNT);
    __syncthreads();
    if (threadIdx.x < KP) {
        const int i = threadIdx.x;
        double sc = 1.0;
        if (i < k) {
            const double inv = 1.0 / sqrt(ss[TRI + i]);
            if (!isfinite(inv) || !(ss[TRI + i] > 0.0))
                atomicOr(&cw->status, kStatusNonFinite);
            if (mode >= 1)
                sc = inv;
            if (mode == 2) {
                double s = ss[tri_idx(i, i)] * inv;
                if (!(s >= rho))
                    s = rho;
                sc /= sqrt(s);
            }
        }
        scale[i] = sc;
    }
    __syncthreads();
    const int64_t n = d * (int64_t)k;
    for (int64_t e = threadIdx.x; e < n; e += kNT) {
        const int i = (int)(e / d);
        const int64_t f = e % d;
        const int64_t sf = f < dx ? f : dxp + (f - dx);
        out[e] = scale[i] * (double)S[qidx<KP>(sf, i)];
    }
}

// Sign convention of a read-out: column blockIdx.x of out (d x k,
// column-major FP64) is negated when its largest-magnitude component (the
// lowest index among equal magnitudes) is negative, so that component is
// positive.  One workgroup per column: strided per-thread maxima, then a
// fixed-order reduction in LDS.
__global__ void __launch_bounds__(kNT) k_canon(double *out, int64_t d)
{
    __shared__ double bm[kNT];
    __shared__ int64_t bi[kNT];
    double *col = out + (int64_t)blockIdx.x * d;
    double m = -1.0;
    int64_t mi = 0;
    for (int64_t f = threadIdx.x; f < d; f += kNT) {
        const double a = fabs(col[f]);
        if (a > m) { // strictly larger: the lowest index of this thread's ties
            m = a;
            mi = f;
        }
    }
    bm[threadIdx.x] = m;
    bi[threadIdx.x] = mi;
    __syncthreads();
    for (int h = kNT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const double m2 = bm[threadIdx.x + h];
            const int64_t i2 = bi[threadIdx.x + h];
            if (m2 > bm[threadIdx.x] || (m2 == bm[threadIdx.x] && i2 < bi[threadIdx.x])) {
                bm[threadIdx.x] = m2;
                bi[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (col[bi[0]] < 0.0)
        for (int64_t f = threadIdx.x; f < d; f += kNT)
            col[f] = -col[f];
}

} // namespace sgep
