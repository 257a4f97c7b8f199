// sgep_kernels.hpp -- CDNA4 (gfx950) kernels of the stochastic gamma-EigenGame
// step (Alg. 2 of Gemp, Chen, McWilliams, ICLR 2023, with M = 1).
//
// One iteration is two launches and no cross-workgroup synchronisation inside
// either of them (the kernel boundary is the only barrier):
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
// Storage: V, G and the Adam moments are d x KP row-major (KP = 16, 32 or 64,
// padding columns held at zero), so one MFMA B-operand row and one
// accumulator column are contiguous.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace sgep {

constexpr int kNT = 256;     // threads per workgroup: four wave64
constexpr int kKPMax = 64;   // largest padded player count
constexpr int kScr = 1024;   // LDS scratch (doubles) of the partial reductions

constexpr int kKindCCA = 0;
constexpr int kKindGeneral = 1;
constexpr int kOptSGD = 0;
constexpr int kOptAdam = 1;

constexpr int kStatusNonFinite = 1;

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
    double s[kKPMax];        // max(v_j^T G_j, rho) used by the latest iteration
    double ema_a[kKPMax];    // running mean of mA (rate gamma)
    double ema_b[kKPMax];    // running mean of mB
    int status;              // kStatus* bits
    int clip_count;          // parents clipped at rho, cumulative
};

struct StepArgs {
    const void *X, *Y;
    int64_t ldx, ldy, b;
    int64_t dx, dy;          // CCA: view widths; GENERAL: dx = dy = d
    int32_t k, n_tx, n_ty;   // feature tiles over view x and view y (GENERAL: n_ty = 0)
    int32_t vec_ok;          // rows of X and Y 16-byte aligned: vector loads allowed
    int32_t n_fwd;           // forward workgroups of this iteration
    int32_t ldg, lds;        // leading dimensions of the Gram / stats partials
    void *V, *G, *Am, *As;   // d x KP state
    void *P, *Q;             // b x KP raw projections X V, Y V
    double *gram_part;       // [W][ldg]: column blk = forward workgroup blk
    double *stat_part;       // [W][lds]: column tile = backward workgroup tile
    double *stat_tot;        // [W]: reduced stat_part of the state entering this iteration
    Coef *coef;
    int32_t schedule;
    double eta0, eta_T, t0, t_c, T, gamma, rho, eps_reg, adam_b1, adam_b2, adam_eps;
};

__device__ __forceinline__ int tri_idx(int i, int j) { return i * (i + 1) / 2 + j; } // j <= i

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

// out[c] = sum_{r < n} part[c * ld + r] for c < W, by all threads of the
// workgroup in a fixed order (rows in chunks of 32, chunks in order).
// ld is even and part 16-byte aligned.  scr: kScr doubles of LDS.
__device__ inline void colsum(const double *__restrict__ part, int n, int ld, int W,
                              double *__restrict__ out, double *__restrict__ scr)
{
    constexpr int CH = 32;
    const int nch = (n + CH - 1) / CH;
    int per_pass = kScr / nch;
    if (per_pass < 1)
        per_pass = 1;
    for (int c0 = 0; c0 < W; c0 += per_pass) {
        const int cols = (W - c0 < per_pass) ? W - c0 : per_pass;
        for (int p = threadIdx.x; p < cols * nch; p += kNT) {
            const int cl = p / nch, q = p - cl * nch;
            const double *src = part + (int64_t)(c0 + cl) * ld + q * CH;
            const int m = (n - q * CH < CH) ? n - q * CH : CH;
            double s = 0.0;
            if (m == CH) {
                f64x2 v[CH / 2];
#pragma unroll
                for (int u = 0; u < CH / 2; ++u)
                    v[u] = *reinterpret_cast<const f64x2 *>(src + 2 * u);
#pragma unroll
                for (int u = 0; u < CH / 2; ++u) {
                    s += v[u][0];
                    s += v[u][1];
                }
            } else {
                for (int r = 0; r < m; ++r)
                    s += src[r];
            }
            scr[p] = s;
        }
        __syncthreads();
        for (int cl = threadIdx.x; cl < cols; cl += kNT) {
            double s = 0.0;
            for (int q = 0; q < nch; ++q)
                s += scr[cl * nch + q];
            out[c0 + cl] = s;
        }
        __syncthreads();
    }
}

template <typename T, int N> struct VecLoad;
template <> struct VecLoad<float, 1> {
    static __device__ __forceinline__ void run(const float *p, float *o) { o[0] = p[0]; }
};
template <> struct VecLoad<double, 1> {
    static __device__ __forceinline__ void run(const double *p, double *o) { o[0] = p[0]; }
};
template <> struct VecLoad<float, 4> {
    static __device__ __forceinline__ void run(const float *p, float *o)
    {
        f32x4 v = *reinterpret_cast<const f32x4 *>(p);
        o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
    }
};
template <> struct VecLoad<float, 2> {
    static __device__ __forceinline__ void run(const float *p, float *o)
    {
        f32x2 v = *reinterpret_cast<const f32x2 *>(p);
        o[0] = v[0]; o[1] = v[1];
    }
};
template <> struct VecLoad<double, 2> {
    static __device__ __forceinline__ void run(const double *p, double *o)
    {
        f64x2 v = *reinterpret_cast<const f64x2 *>(p);
        o[0] = v[0]; o[1] = v[1];
    }
};
template <> struct VecLoad<double, 4> {
    static __device__ __forceinline__ void run(const double *p, double *o)
    {
        f64x2 v0 = *reinterpret_cast<const f64x2 *>(p);
        f64x2 v1 = *reinterpret_cast<const f64x2 *>(p + 2);
        o[0] = v0[0]; o[1] = v0[1]; o[2] = v1[0]; o[3] = v1[1];
    }
};

// N consecutive elements of row `row` starting at feature fs, masked beyond
// nf and for invalid rows.  The vector path needs vec_ok (16-byte aligned rows)
// and fs % N == 0.
template <typename T, int N>
__device__ __forceinline__ void load_run(const T *__restrict__ X, int64_t ld, int64_t row, bool rv,
                                         int64_t fs, int64_t nf, bool vec_ok, T *o)
{
    if (rv && vec_ok && fs + N <= nf) {
        VecLoad<T, N>::run(X + row * ld + fs, o);
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j)
            o[j] = (rv && fs + j < nf) ? X[row * ld + fs + j] : T(0);
    }
}

// ---------------------------------------------------------------------------
// Forward products.  One wave accumulates the 16 x KP tile of one view over a
// contiguous quarter of the features.  Each lane loads VEC consecutive
// features of its row; MFMA j of a group consumes element j, i.e. the MFMA
// k-index l/16 stands for feature c*4*VEC + VEC*(l/16) + j, and the B operand
// (row of V) is taken at the same feature, so the sum is unchanged.  U groups
// are loaded before their MFMAs are issued.
// ---------------------------------------------------------------------------
template <typename T, int KP>
__device__ __forceinline__ void fwd_view(const T *__restrict__ X, int64_t ldx, int64_t nf, int64_t row,
                                         bool rv, bool vec_ok, const T *__restrict__ V, int lane,
                                         int w, typename Mfma<T>::acc *acc)
{
    constexpr int VEC = 16 / (int)sizeof(T);
    constexpr int CH = 4 * VEC;
    constexpr int NB = KP / 16;
    constexpr int U = 8 / NB > 1 ? 8 / NB : 2;
    const int kk = lane >> 4, n = lane & 15;
    const int64_t nch = (nf + CH - 1) / CH;
    const int64_t c0 = (nch * w) >> 2, c1 = (nch * (w + 1)) >> 2;
    for (int64_t cb = c0; cb < c1; cb += U) {
        T xv[U][VEC];
        T bv[U][VEC][NB];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t c = cb + u;
            const bool cv = c < c1;
            const int64_t fb = c * CH + (int64_t)VEC * kk;
            load_run<T, VEC>(X, ldx, row, rv && cv, fb, nf, vec_ok, xv[u]);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const int64_t fe = fb + j;
                const bool fv = cv && fe < nf;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    bv[u][j][nb] = fv ? V[fe * KP + nb * 16 + n] : T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < VEC; ++j)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[nb] = Mfma<T>::fma(xv[u][j], bv[u][j][nb], acc[nb]);
    }
}

template <typename T, int KP, int KIND>
__global__ void __launch_bounds__(kNT) k_fwd(StepArgs a)
{
    typedef typename Mfma<T>::acc Acc;
    constexpr int NB = KP / 16;
    constexpr int TRI = KP * (KP + 1) / 2;
    constexpr int GW = TRI + KP;
    __shared__ T red[4][16][KP];
    __shared__ T pt[16][KP], qt[16][KP];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kk = lane >> 4, n = lane & 15;
    if ((int)blockIdx.x == a.n_fwd) {
        // norm / parent-term totals of the current state (sum over the
        // previous backward pass's tiles, fixed order); advance t
        __shared__ double scr[kScr];
        __shared__ double tot[GW];
        colsum(a.stat_part, a.n_tx + a.n_ty, a.lds, GW, tot, scr);
        for (int e = tid; e < GW; e += kNT)
            a.stat_tot[e] = tot[e];
        if (tid == 0)
            a.coef->t += 1.0; // read by k_bwd only, after this kernel has finished
        return;
    }
    const int64_t r0 = (int64_t)blockIdx.x * 16;
    const int64_t row = r0 + n;
    const bool rv = row < a.b;
    const bool vec_ok = a.vec_ok != 0;
    const T *X = (const T *)a.X, *Y = (const T *)a.Y, *V = (const T *)a.V;
    T *P = (T *)a.P, *Q = (T *)a.Q;

    Acc accP[NB], accQ[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        accP[nb] = Acc{0, 0, 0, 0};
        accQ[nb] = Acc{0, 0, 0, 0};
    }
    fwd_view<T, KP>(X, a.ldx, a.dx, row, rv, vec_ok, V, lane, w, accP);
    if (KIND == kKindCCA)
        fwd_view<T, KP>(Y, a.ldy, a.dy, row, rv, vec_ok, V + a.dx * KP, lane, w, accQ);
    else
        fwd_view<T, KP>(Y, a.ldy, a.dx, row, rv, vec_ok, V, lane, w, accQ);

    // sum the four waves' partial tiles in a fixed order
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[w][Mfma<T>::drow(kk, r)][nb * 16 + n] = accP[nb][r];
    __syncthreads();
    for (int e = tid; e < 16 * KP; e += kNT) {
        const int r = e / KP, c = e % KP;
        const T s = red[0][r][c] + red[1][r][c] + red[2][r][c] + red[3][r][c];
        pt[r][c] = s;
        if (r0 + r < a.b)
            P[(r0 + r) * KP + c] = s;
    }
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[w][Mfma<T>::drow(kk, r)][nb * 16 + n] = accQ[nb][r];
    __syncthreads();
    for (int e = tid; e < 16 * KP; e += kNT) {
        const int r = e / KP, c = e % KP;
        const T s = red[0][r][c] + red[1][r][c] + red[2][r][c] + red[3][r][c];
        qt[r][c] = s;
        if (r0 + r < a.b)
            Q[(r0 + r) * KP + c] = s;
    }
    __syncthreads();

    // partial Grams over these 16 rows (raw players, FP64): lower triangle of
    // b V^T A_t V and the diagonal of b V^T B_t V (without the ridge)
    for (int e = tid; e < GW; e += kNT) {
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
        a.gram_part[(int64_t)e * a.ldg + blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// Backward products + fused update for a tile of FT = 16*MB features.
// A operand = X^T: lane l loads MB consecutive features f0 + MB*(l%16) + j of
// row r + l/16; element j feeds M-block j, so M-block j, M-row m holds feature
// f0 + MB*m + j.  B operands: rows of Q and P (KP wide).  The four waves take
// interleaved 4-row groups; U groups are loaded before their MFMAs.
// ---------------------------------------------------------------------------
template <typename T, int KP, int MB, int KIND, int OPT>
__global__ void __launch_bounds__(kNT) k_bwd(StepArgs a)
{
    typedef typename Mfma<T>::acc Acc;
    constexpr int NB = KP / 16;
    constexpr int FT = 16 * MB;
    constexpr int TRI = KP * (KP + 1) / 2;
    constexpr int W = TRI + KP; // width of both partial kinds
    constexpr int U = 16 / (MB * NB) > 2 ? 16 / (MB * NB) : 2;
    constexpr int EPT = FT * KP / kNT; // epilogue elements per thread
    static_assert(EPT * kNT == FT * KP, "tile must be a multiple of the workgroup");
    __shared__ T red[4][FT * KP];
    __shared__ T avt[FT * KP], bvt[FT * KP], gt[FT * KP];
    __shared__ T Tl[KP * KP];
    __shared__ T cMB[KP], cMAc[KP], cInv[KP];
    __shared__ double gs[W], ss[W], scr[kScr];
    __shared__ double dInv[KP], dS[KP];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kk = lane >> 4, m = lane & 15;
    const int tile = blockIdx.x;
    const bool vec_ok = a.vec_ok != 0;
    const T *X = (const T *)a.X, *Y = (const T *)a.Y;
    const T *P = (const T *)a.P, *Q = (const T *)a.Q;

    const T *Xa;      // view multiplying the A-side operand
    const T *Xb;      // view multiplying the B-side operand
    int64_t lda, ldb, nf, fbase, f0;
    const T *opA, *opB;
    if (KIND == kKindCCA) {
        if (tile < a.n_tx) { // x features: A_t V = X^T Q / b, B_t V = X^T P / b
            Xa = X; lda = a.ldx; nf = a.dx; fbase = 0; f0 = (int64_t)tile * FT;
            opA = Q; opB = P;
        } else {             // y features: A_t V = Y^T P / b, B_t V = Y^T Q / b
            Xa = Y; lda = a.ldy; nf = a.dy; fbase = a.dx; f0 = (int64_t)(tile - a.n_tx) * FT;
            opA = P; opB = Q;
        }
        Xb = Xa; ldb = lda;
    } else {                 // GENERAL: A_t V = Y^T Q / b, B_t V = X^T P / b + eps V
        Xa = Y; lda = a.ldy; Xb = X; ldb = a.ldx;
        nf = a.dx; fbase = 0; f0 = (int64_t)tile * FT;
        opA = Q; opB = P;
    }

    // ---- main loop: raw X^T Q and X^T P over all rows ----
    Acc accA[MB][NB], accB[MB][NB];
#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            accA[j][nb] = Acc{0, 0, 0, 0};
            accB[j][nb] = Acc{0, 0, 0, 0};
        }
    const int64_t fs = f0 + (int64_t)MB * m;
    for (int64_t rb = 4 * w; rb < a.b; rb += 16 * U) {
        T xa[U][MB], xb[U][MB], ba[U][NB], bb[U][NB];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = rb + 16 * u + kk;
            const bool rv = row < a.b;
            load_run<T, MB>(Xa, lda, row, rv, fs, nf, vec_ok, xa[u]);
            if (KIND != kKindCCA)
                load_run<T, MB>(Xb, ldb, row, rv, fs, nf, vec_ok, xb[u]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                ba[u][nb] = rv ? opA[row * KP + nb * 16 + m] : T(0);
                bb[u][nb] = rv ? opB[row * KP + nb * 16 + m] : T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < MB; ++j)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    accA[j][nb] = Mfma<T>::fma(xa[u][j], ba[u][nb], accA[j][nb]);
                    accB[j][nb] = Mfma<T>::fma(KIND == kKindCCA ? xa[u][j] : xb[u][j], bb[u][nb],
                                               accB[j][nb]);
                }
    }

    // cross-wave reduction (fixed order) into natural feature order
#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                red[w][(MB * Mfma<T>::drow(kk, r) + j) * KP + nb * 16 + m] = accA[j][nb][r];
    __syncthreads();
    for (int e = tid; e < FT * KP; e += kNT)
        avt[e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                red[w][(MB * Mfma<T>::drow(kk, r) + j) * KP + nb * 16 + m] = accB[j][nb][r];
    __syncthreads();
    for (int e = tid; e < FT * KP; e += kNT)
        bvt[e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];

    // ---- prefetch the epilogue operands of this thread's elements ----
    T *V = (T *)a.V, *G = (T *)a.G, *Am = (T *)a.Am, *As = (T *)a.As;
    T pv[EPT], pm[EPT], ps[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * kNT;
        const int fl = e / KP, i = e % KP;
        const int64_t f = f0 + fl;
        const bool ok = f < nf;
        const int64_t gi = (fbase + (ok ? f : 0)) * KP + i;
        gt[e] = ok ? G[gi] : T(0);
        pv[q] = ok ? V[gi] : T(0);
        if (OPT == kOptAdam) {
            pm[q] = ok ? Am[gi] : T(0);
            ps[q] = ok ? As[gi] : T(0);
        }
    }

    // ---- k x k coefficients (identical in every workgroup) ----
    Coef *cw = a.coef;
    const double t = cw->t; // this iteration's number, set by k_fwd
    for (int e = tid; e < W; e += kNT)
        ss[e] = a.stat_tot[e];
    colsum(a.gram_part, a.n_fwd, a.ldg, W, gs, scr);
    const double ib = 1.0 / (double)a.b;
    if (tid < KP) {
        const int i = tid;
        double inv = 0.0, s = 1.0;
        if (i < a.k) {
            inv = 1.0 / sqrt(ss[TRI + i]);
            s = ss[tri_idx(i, i)] * inv; // v_i^T G_i with the unit v_i
            if (!(s >= a.rho))
                s = a.rho;
        }
        dInv[i] = inv;
        dS[i] = s;
    }
    __syncthreads();
    // T_ij = (M_A)_ij / s_j with (M_A)_ij = b^{-1} inv_i inv_j (raw Gram)_ij
    for (int e = tid; e < KP * KP; e += kNT) {
        const int i = e / KP, j = e % KP;
        double v = 0.0;
        if (i < a.k && j < i)
            v = gs[tri_idx(i, j)] * dInv[i] * dInv[j] * ib / dS[j];
        Tl[e] = (T)v;
    }
    if (tid < KP) {
        const int i = tid;
        double mA = 0.0, mB = 0.0, c = 0.0;
        if (i < a.k) {
            const double ii2 = dInv[i] * dInv[i];
            mA = gs[tri_idx(i, i)] * ii2 * ib;
            mB = gs[TRI + i] * ii2 * ib + (KIND == kKindCCA ? 0.0 : a.eps_reg);
            for (int j = 0; j < i; ++j) {
                const double Tij = gs[tri_idx(i, j)] * dInv[i] * dInv[j] * ib / dS[j];
                c += Tij * (ss[tri_idx(i, j)] * dInv[i]); // T_ij C_ij
            }
        }
        cMB[i] = (T)mB;
        cMAc[i] = (T)(mA - c);
        cInv[i] = (T)dInv[i];
        if (blockIdx.x == 0) {
            if (i < a.k) {
                cw->ema_a[i] += a.gamma * (mA - cw->ema_a[i]);
                cw->ema_b[i] += a.gamma * (mB - cw->ema_b[i]);
                const double craw = ss[tri_idx(i, i)] * dInv[i];
                if (!(craw >= a.rho))
                    atomicAdd(&cw->clip_count, 1);
                if (!isfinite(mA) || !isfinite(mB) || !isfinite(c) || !isfinite(dInv[i]) ||
                    !(dInv[i] > 0.0) || !isfinite(craw))
                    atomicOr(&cw->status, kStatusNonFinite);
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
    // ---- fused epilogue ----
    __syncthreads();
    const T eta = (T)eta_at(a, t), gam = (T)a.gamma, ibT = (T)ib;
    const T eps = (T)a.eps_reg;
    const T b1 = (T)a.adam_b1, b2 = (T)a.adam_b2, aeps = (T)a.adam_eps;
    const T c1 = (T)(1.0 - pow(a.adam_b1, t)), c2 = (T)(1.0 - pow(a.adam_b2, t));
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * kNT;
        const int fl = e / KP, i = e % KP;
        const int64_t f = f0 + fl;
        T vn = 0, gn = 0;
        if (f < nf && i < a.k) {
            const int64_t gi = (fbase + f) * KP + i;
            const T vh = pv[q] * cInv[i];
            const T av = avt[e] * cInv[i] * ibT;
            T bv = bvt[e] * cInv[i] * ibT;
            if (KIND != kKindCCA)
                bv += eps * vh;
            T pen = 0;
            for (int j = 0; j < i; ++j)
                pen += Tl[i * KP + j] * gt[fl * KP + j];
            const T grad = (av - pen) * cMB[i] - bv * cMAc[i];
            if (OPT == kOptSGD) {
                vn = vh + eta * grad;
            } else {
                const T mm = b1 * pm[q] + (T(1) - b1) * grad;
                const T sq = b2 * ps[q] + (T(1) - b2) * grad * grad;
                Am[gi] = mm;
                As[gi] = sq;
                vn = vh + eta * (mm / c1) / (sqrt(sq / c2) + aeps);
            }
            const T g0 = gt[e];
            gn = g0 + gam * (bv - g0);
            V[gi] = vn;
            G[gi] = gn;
        }
        avt[e] = vn; // own slot: reused for the partials below
        bvt[e] = gn;
    }
    __syncthreads();
    // this tile's partials of v_i^T G_j (j <= i) and ||v_i||^2 of the new state
    double *sout = a.stat_part;
    for (int e = tid; e < W; e += kNT) {
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
        sout[(int64_t)e * a.lds + tile] = s;
    }
}

// ---------------------------------------------------------------------------
// Initialisation (one workgroup; not on the hot path): normalise the supplied
// players to the unit sphere, set [Bv]_i = v_i (Alg. 2), and write the norm /
// parent-term sums of this state as column 0 of stats buffer 0 (the other
// columns are zero).
// ---------------------------------------------------------------------------
template <typename T, int KP>
__global__ void __launch_bounds__(kNT) k_init(T *V, T *G, int64_t d, int k, double *stat0, int lds,
                                              Coef *cw)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    __shared__ double part[kNT];
    __shared__ double nrm[KP];
    const int tid = threadIdx.x;
    for (int i = 0; i < KP; ++i) {
        double s = 0.0;
        for (int64_t f = tid; f < d; f += kNT)
            s += (double)V[f * KP + i] * (double)V[f * KP + i];
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
    for (int64_t e = tid; e < d * KP; e += kNT) {
        const int i = (int)(e % KP);
        const T v = (i < k) ? (T)((double)V[e] / sqrt(nrm[i])) : T(0);
        V[e] = v;
        G[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < TRI + KP; e += kNT) {
        int i, j;
        if (e < TRI)
            tri_ij(e, i, j);
        else
            i = j = e - TRI;
        double s = 0.0;
        for (int64_t f = 0; f < d; ++f)
            s += (double)V[f * KP + i] * (double)G[f * KP + j]; // G = V
        stat0[(int64_t)e * lds] = s;
        if (e >= TRI && i < k && !(s > 0.0))
            atomicOr(&cw->status, kStatusNonFinite);
    }
}

// Read-out (one workgroup): reduce the latest norm / parent partials, then
// out[i*d + f] = scale_i * S[f*KP + i] (column-major FP64) with scale_i =
// 1/||V_i|| for the players (mode 1), additionally 1/sqrt(s_i) (mode 2:
// B-normalised), or 1 (mode 0: the auxiliary variable).
template <typename T, int KP>
__global__ void __launch_bounds__(kNT) k_readout(const T *S, int64_t d, int k, const double *stat_part,
                                                 int n_tiles, int lds, double rho, Coef *cw, int mode,
                                                 double *out)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    constexpr int W = TRI + KP;
    __shared__ double ss[W], scr[kScr];
    __shared__ double scale[KP];
    colsum(stat_part, n_tiles, lds, W, ss, scr);
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
        out[e] = scale[i] * (double)S[f * KP + i];
    }
}

} // namespace sgep
