// sgep_kernels.hpp -- CDNA4 (gfx950) kernels of the stochastic gamma-EigenGame
// step (Alg. 2 of Gemp, Chen, McWilliams, ICLR 2023, with M = 1).
//
// One iteration is two launches:
//   k_fwd  P = X V, Q = Y V (tall-skinny products on MFMA), then per-workgroup
//          partial k x k Grams; the last workgroup to finish reduces them in a
//          fixed order and forms every k x k coefficient of the update
//          (the Rayleigh terms of the rewards and the triangular penalty
//          weights), the step sizes and the running means.
//   k_bwd  A_t V and B_t V for a tile of features (X^T [Q|P] on MFMA, X tiles
//          streamed straight from HBM, rows split over waves and optionally
//          over workgroups), then a fused epilogue: the update direction in
//          matrix form, the retraction step (SGD or Adam), the auxiliary
//          update, and per-tile partials of ||v_i||^2 and v_i^T [Bv]_j; the
//          last tile reduces those (fixed order) into the normalisation and
//          the parent terms the next iteration needs.
//
// Matrix form of the update direction used here.  With the unit players v_i,
// the auxiliary G_j = [Bv]_j, the minibatch Gram M_A = V^T A_t V and
// m_B,i = v_i^T B_t v_i, s_j = max(v_j^T G_j, rho), C_ij = v_i^T G_j,
// T_ij = (M_A)_ij / s_j for j < i and c_i = sum_{j<i} T_ij C_ij, the
// rewards-minus-penalties direction of Alg. 2 for all players at once is
//     grad = (A_t V - G T^T) diag(m_B) - B_t V diag(m_A - c),
// because v_i^T A_t y_j = (M_A)_ij / sqrt(s_j), [By]_j = G_j / sqrt(s_j) and
// <v_i, [By]_j> = C_ij / sqrt(s_j).  The paper's per-player loop costs
// O(b d k^2); sharing A_t V and B_t V across players makes it O(b d k + d k^2).
//
// Storage: V, G and the Adam moments are d x KP row-major (KP = k rounded up
// to a multiple of 16, padding columns held at zero) so that one MFMA B
// operand row and one accumulator column are contiguous.  The stored V is the
// iterate before normalisation; inv_nrm (in the coefficient block) rescales it.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace sgep {

constexpr int kNT = 256;     // threads per workgroup: four wave64
constexpr int kKPMax = 64;   // largest padded player count

constexpr int kKindCCA = 0;
constexpr int kKindGeneral = 1;
constexpr int kOptSGD = 0;
constexpr int kOptAdam = 1;

// status bits latched on the device
constexpr int kStatusNonFinite = 1;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// 16x16x4 MFMA for one element type.  Operand layout (wave64):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[4 (l / 16) + r][l % 16], r = 0..3
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef f32x4 acc;
    static __device__ __forceinline__ acc fma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    typedef f64x4 acc;
    static __device__ __forceinline__ acc fma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// Coefficient block shared by the two kernels (device memory, FP64).
// Matrices use row stride KP of the handle.
struct Coef {
    double mA[kKPMax];      // v_i^T A_t v_i (this iteration)
    double mB[kKPMax];      // v_i^T B_t v_i
    double c[kKPMax];       // sum_{j<i} T_ij C_ij
    double T[kKPMax * kKPMax];  // (M_A)_ij / s_j, j < i
    double C[kKPMax * kKPMax];  // v_i^T G_j, j <= i (for the next iteration)
    double s[kKPMax];       // max(C_jj, rho)
    double inv_nrm[kKPMax]; // 1 / ||stored V_i||
    double ema_a[kKPMax];   // running mean of mA (rate gamma)
    double ema_b[kKPMax];   // running mean of mB
    double t;               // completed iterations
    double eta, gamma;      // step sizes of the current iteration
    double adam_c1, adam_c2; // 1 - b1^t, 1 - b2^t
    int status;             // kStatus* bits
    int clip_count;         // parents clipped at rho, cumulative
    int pad[2];
};

struct StepArgs {
    const void *X, *Y;
    int64_t ldx, ldy, b;
    int64_t dx, dy;          // CCA: view widths; GENERAL: dx = dy = d
    int32_t k, n_tx, n_ty;   // feature tiles over view x and view y (GENERAL: n_ty = 0)
    int32_t splits;          // workgroups per feature tile along the rows
    int64_t rows_per_split;
    void *V, *G, *Am, *As;   // d x KP state
    void *P, *Q;             // b x KP projections (normalised players)
    void *ws;                // split partials: tiles x splits x 2 x FT x KP
    double *gram_part;       // fwd workgroups x (KP(KP+1)/2 + KP)
    double *stat_part;       // tiles x (KP(KP+1)/2 + KP)
    Coef *coef;
    unsigned *cnt;           // [0] fwd arrivals, [1] tile arrivals, [2 + tile] split arrivals
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

// Arrival counter for "last workgroup finishes the reduction".  Every thread
// releases its global writes at agent scope before the barrier; the last
// arrival acquires before reading the other workgroups' partials.
__device__ __forceinline__ bool arrive_last(unsigned *counter, unsigned total, int *flag)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = atomicAdd(counter, 1u);
        *flag = (prev == total - 1u) ? 1 : 0;
    }
    __syncthreads();
    const bool last = *flag != 0;
    if (last)
        __threadfence();
    return last;
}

template <typename T, int N> struct VecLoad;
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

// N consecutive elements of row `row` starting at feature fs (masked beyond
// nf and for invalid rows).  The vector path needs fs % N == 0 and a leading
// dimension that keeps rows 16-byte aligned (checked by the host).
template <typename T, int N>
__device__ __forceinline__ void load_run(const T *__restrict__ X, int64_t ld, int64_t row, bool rv,
                                         int64_t fs, int64_t nf, T *o)
{
    if (rv && fs + N <= nf) {
        VecLoad<T, N>::run(X + row * ld + fs, o);
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j)
            o[j] = (rv && fs + j < nf) ? X[row * ld + fs + j] : T(0);
    }
}

// ---------------------------------------------------------------------------
// Forward products: partial P-tile (16 rows x KP) of one view for this wave.
// The view's features are split in four contiguous ranges, one per wave.
// Each lane loads VEC consecutive features of its row; MFMA j of a group
// consumes element j, i.e. the k-index l/16 of the MFMA maps to feature
// fb = chunk*4*VEC + VEC*(l/16) + j.  The same feature indexes the B operand
// (row of V), so the sum over k is unchanged.
// ---------------------------------------------------------------------------
template <typename T, int KP>
__device__ __forceinline__ void fwd_view(const T *__restrict__ X, int64_t ldx, int64_t nf, int64_t row,
                                         bool rv, const T *__restrict__ V, int lane, int w,
                                         typename Mfma<T>::acc *acc)
{
    constexpr int VEC = 16 / (int)sizeof(T);
    constexpr int CH = 4 * VEC;
    constexpr int NB = KP / 16;
    const int kk = lane >> 4, n = lane & 15;
    const int64_t nch = (nf + CH - 1) / CH;
    const int64_t c0 = (nch * w) >> 2, c1 = (nch * (w + 1)) >> 2;
    for (int64_t c = c0; c < c1; ++c) {
        const int64_t fb = c * CH + (int64_t)VEC * kk;
        T xv[VEC];
        load_run<T, VEC>(X, ldx, row, rv, fb, nf, xv);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const int64_t fe = fb + j;
            const bool fv = fe < nf;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const T bv = fv ? V[fe * KP + nb * 16 + n] : T(0);
                acc[nb] = Mfma<T>::fma(xv[j], bv, acc[nb]);
            }
        }
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
    __shared__ int s_flag;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kk = lane >> 4, n = lane & 15;
    const int64_t r0 = (int64_t)blockIdx.x * 16;
    const int64_t row = r0 + n;
    const bool rv = row < a.b;
    const T *X = (const T *)a.X, *Y = (const T *)a.Y, *V = (const T *)a.V;
    T *P = (T *)a.P, *Q = (T *)a.Q;
    const Coef *cf = a.coef;

    Acc accP[NB], accQ[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        accP[nb] = Acc{0, 0, 0, 0};
        accQ[nb] = Acc{0, 0, 0, 0};
    }
    fwd_view<T, KP>(X, a.ldx, a.dx, row, rv, V, lane, w, accP);
    if (KIND == kKindCCA)
        fwd_view<T, KP>(Y, a.ldy, a.dy, row, rv, V + a.dx * KP, lane, w, accQ);
    else
        fwd_view<T, KP>(Y, a.ldy, a.dx, row, rv, V, lane, w, accQ);

    // sum the four waves' partial tiles (fixed order), normalise the columns
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[w][4 * kk + r][nb * 16 + n] = accP[nb][r];
    __syncthreads();
    for (int e = tid; e < 16 * KP; e += kNT) {
        const int r = e / KP, c = e % KP;
        T s = red[0][r][c] + red[1][r][c] + red[2][r][c] + red[3][r][c];
        s *= (T)cf->inv_nrm[c];
        pt[r][c] = s;
        if (r0 + r < a.b)
            P[(r0 + r) * KP + c] = s;
    }
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[w][4 * kk + r][nb * 16 + n] = accQ[nb][r];
    __syncthreads();
    for (int e = tid; e < 16 * KP; e += kNT) {
        const int r = e / KP, c = e % KP;
        T s = red[0][r][c] + red[1][r][c] + red[2][r][c] + red[3][r][c];
        s *= (T)cf->inv_nrm[c];
        qt[r][c] = s;
        if (r0 + r < a.b)
            Q[(r0 + r) * KP + c] = s;
    }
    __syncthreads();

    // partial Grams over these 16 rows: lower triangle of V^T A_t V (times b)
    // and the diagonal of V^T B_t V (times b), accumulated in FP64
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
        a.gram_part[(int64_t)blockIdx.x * GW + e] = s;
    }

    if (!arrive_last(&a.cnt[0], gridDim.x, &s_flag))
        return;

    // ---- last workgroup: reduce the Grams and form the coefficients ----
    __shared__ double gs[GW];
    __shared__ double Ts[KP][KP];
    for (int e = tid; e < GW; e += kNT) {
        double s = 0.0;
        for (unsigned blk = 0; blk < gridDim.x; ++blk)
            s += a.gram_part[(int64_t)blk * GW + e];
        gs[e] = s;
    }
    __syncthreads();
    Coef *cw = a.coef;
    const double ib = 1.0 / (double)a.b;
    const double t = cw->t + 1.0;
    for (int e = tid; e < KP * KP; e += kNT) {
        const int i = e / KP, j = e % KP;
        double v = 0.0;
        if (i < a.k && j < i)
            v = gs[tri_idx(i, j)] * ib / cw->s[j];
        Ts[i][j] = v;
        cw->T[e] = v;
    }
    __syncthreads();
    if (tid < KP) {
        const int i = tid;
        double mA = 0.0, mB = 0.0, c = 0.0;
        if (i < a.k) {
            mA = gs[tri_idx(i, i)] * ib;
            mB = gs[TRI + i] * ib + (KIND == kKindCCA ? 0.0 : a.eps_reg);
            for (int j = 0; j < i; ++j)
                c += Ts[i][j] * cw->C[i * KP + j];
            cw->ema_a[i] += a.gamma * (mA - cw->ema_a[i]);
            cw->ema_b[i] += a.gamma * (mB - cw->ema_b[i]);
            if (!isfinite(mA) || !isfinite(mB) || !isfinite(c))
                atomicOr(&cw->status, kStatusNonFinite);
        }
        cw->mA[i] = mA;
        cw->mB[i] = mB;
        cw->c[i] = c;
    }
    __syncthreads();
    if (tid == 0) {
        cw->t = t;
        cw->eta = eta_at(a, t);
        cw->gamma = a.gamma;
        cw->adam_c1 = 1.0 - pow(a.adam_b1, t);
        cw->adam_c2 = 1.0 - pow(a.adam_b2, t);
        atomicExch(&a.cnt[0], 0u);
    }
}

// ---------------------------------------------------------------------------
// Backward products + fused update for a tile of FT = 16*MB features.
// A operand = X^T: lane l loads MB consecutive features f0 + MB*(l%16) + j of
// row r + l/16; element j feeds M-block j, so M-block j, M-row m holds feature
// f0 + MB*m + j.  B operands: rows of Q and P (KP wide).
// ---------------------------------------------------------------------------
template <typename T, int KP, int MB, int KIND, int OPT>
__global__ void __launch_bounds__(kNT) k_bwd(StepArgs a)
{
    typedef typename Mfma<T>::acc Acc;
    constexpr int NB = KP / 16;
    constexpr int FT = 16 * MB;
    constexpr int TRI = KP * (KP + 1) / 2;
    constexpr int SW = TRI + KP;
    __shared__ T red[4][FT * KP];
    __shared__ T avt[FT * KP], bvt[FT * KP], gt[FT * KP], vt[FT * KP];
    __shared__ T Tl[KP * KP];
    __shared__ T cMB[KP], cMAc[KP], cInv[KP];
    __shared__ int s_flag;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kk = lane >> 4, m = lane & 15;
    const int tile = blockIdx.x, split = blockIdx.y;
    const T *X = (const T *)a.X, *Y = (const T *)a.Y;
    const T *P = (const T *)a.P, *Q = (const T *)a.Q;

    // geometry of this tile
    const T *Xa;      // view whose transpose multiplies the A-side operand
    const T *Xb;      // view whose transpose multiplies the B-side operand
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

    Acc accA[MB][NB], accB[MB][NB];
#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            accA[j][nb] = Acc{0, 0, 0, 0};
            accB[j][nb] = Acc{0, 0, 0, 0};
        }
    const int64_t rb = (int64_t)split * a.rows_per_split;
    const int64_t re = (rb + a.rows_per_split < a.b) ? rb + a.rows_per_split : a.b;
    const int64_t fs = f0 + (int64_t)MB * m;
    for (int64_t r = rb + 4 * w; r < re; r += 16) {
        const int64_t row = r + kk;
        const bool rv = row < re;
        T xa[MB], xb[MB];
        load_run<T, MB>(Xa, lda, row, rv, fs, nf, xa);
        if (KIND == kKindCCA) {
#pragma unroll
            for (int j = 0; j < MB; ++j)
                xb[j] = xa[j];
        } else {
            load_run<T, MB>(Xb, ldb, row, rv, fs, nf, xb);
        }
        T ba[NB], bb[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            ba[nb] = rv ? opA[row * KP + nb * 16 + m] : T(0);
            bb[nb] = rv ? opB[row * KP + nb * 16 + m] : T(0);
        }
#pragma unroll
        for (int j = 0; j < MB; ++j)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                accA[j][nb] = Mfma<T>::fma(xa[j], ba[nb], accA[j][nb]);
                accB[j][nb] = Mfma<T>::fma(xb[j], bb[nb], accB[j][nb]);
            }
    }

    // cross-wave reduction (fixed order) into natural feature order
#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                red[w][(MB * (4 * kk + r) + j) * KP + nb * 16 + m] = accA[j][nb][r];
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
                red[w][(MB * (4 * kk + r) + j) * KP + nb * 16 + m] = accB[j][nb][r];
    __syncthreads();
    for (int e = tid; e < FT * KP; e += kNT)
        bvt[e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
    __syncthreads();

    if (a.splits > 1) {
        T *ws = (T *)a.ws + ((int64_t)tile * a.splits + split) * (2 * FT * KP);
        for (int e = tid; e < FT * KP; e += kNT) {
            ws[e] = avt[e];
            ws[FT * KP + e] = bvt[e];
        }
        if (!arrive_last(&a.cnt[2 + tile], (unsigned)a.splits, &s_flag))
            return;
        const T *base = (const T *)a.ws + (int64_t)tile * a.splits * (2 * FT * KP);
        for (int e = tid; e < FT * KP; e += kNT) {
            T sa = 0, sb = 0;
            for (int s = 0; s < a.splits; ++s) {
                sa += base[(int64_t)s * 2 * FT * KP + e];
                sb += base[(int64_t)s * 2 * FT * KP + FT * KP + e];
            }
            avt[e] = sa;
            bvt[e] = sb;
        }
        if (tid == 0)
            atomicExch(&a.cnt[2 + tile], 0u);
    }

    // ---- fused epilogue ----
    const Coef *cf = a.coef;
    for (int e = tid; e < KP * KP; e += kNT)
        Tl[e] = (T)cf->T[e];
    if (tid < KP) {
        cMB[tid] = (T)cf->mB[tid];
        cMAc[tid] = (T)(cf->mA[tid] - cf->c[tid]);
        cInv[tid] = (T)cf->inv_nrm[tid];
    }
    T *V = (T *)a.V, *G = (T *)a.G, *Am = (T *)a.Am, *As = (T *)a.As;
    for (int e = tid; e < FT * KP; e += kNT) {
        const int fl = e / KP, i = e % KP;
        const int64_t f = f0 + fl;
        const bool valid = f < nf;
        const int64_t gi = (fbase + f) * KP + i;
        gt[e] = valid ? G[gi] : T(0);
        vt[e] = valid ? V[gi] : T(0);
    }
    __syncthreads();
    const T eta = (T)cf->eta, gam = (T)cf->gamma, ib = (T)(1.0 / (double)a.b);
    const T eps = (T)a.eps_reg;
    const T b1 = (T)a.adam_b1, b2 = (T)a.adam_b2, aeps = (T)a.adam_eps;
    const T c1 = (T)cf->adam_c1, c2 = (T)cf->adam_c2;
    for (int e = tid; e < FT * KP; e += kNT) {
        const int fl = e / KP, i = e % KP;
        const int64_t f = f0 + fl;
        T vn = 0, gn = 0;
        if (f < nf && i < a.k) {
            const int64_t gi = (fbase + f) * KP + i;
            const T vh = vt[e] * cInv[i];
            const T av = avt[e] * ib;
            T bv = bvt[e] * ib;
            if (KIND != kKindCCA)
                bv += eps * vh;
            T pen = 0;
            for (int j = 0; j < i; ++j)
                pen += Tl[i * KP + j] * gt[fl * KP + j];
            const T grad = (av - pen) * cMB[i] - bv * cMAc[i];
            if (OPT == kOptSGD) {
                vn = vh + eta * grad;
            } else {
                const T mm = b1 * Am[gi] + (T(1) - b1) * grad;
                const T ss = b2 * As[gi] + (T(1) - b2) * grad * grad;
                Am[gi] = mm;
                As[gi] = ss;
                vn = vh + eta * (mm / c1) / (sqrt(ss / c2) + aeps);
            }
            const T g0 = gt[e];
            gn = g0 + gam * (bv - g0);
            V[gi] = vn;
            G[gi] = gn;
        }
        avt[e] = vn; // own slot only: reused for the stats below
        bvt[e] = gn;
    }
    __syncthreads();

    // per-tile partials of v_i^T G_j (j <= i) and ||v_i||^2 of the new state
    for (int e = tid; e < SW; e += kNT) {
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
        a.stat_part[(int64_t)tile * SW + e] = s;
    }
    const unsigned n_tiles = (unsigned)(a.n_tx + a.n_ty);
    if (!arrive_last(&a.cnt[1], n_tiles, &s_flag))
        return;

    // ---- last tile: normalisation and parent terms for the next iteration ----
    __shared__ double ssum[SW];
    __shared__ double sinv[KP];
    for (int e = tid; e < SW; e += kNT) {
        double s = 0.0;
        for (unsigned tl = 0; tl < n_tiles; ++tl)
            s += a.stat_part[(int64_t)tl * SW + e];
        ssum[e] = s;
    }
    __syncthreads();
    Coef *cw = a.coef;
    if (tid < KP) {
        const int i = tid;
        double inv = 0.0;
        if (i < a.k) {
            const double n2 = ssum[TRI + i];
            inv = 1.0 / sqrt(n2);
            if (!(n2 > 0.0) || !isfinite(inv))
                atomicOr(&cw->status, kStatusNonFinite);
        }
        sinv[i] = inv;
        cw->inv_nrm[i] = inv;
    }
    __syncthreads();
    for (int e = tid; e < KP * KP; e += kNT) {
        const int i = e / KP, j = e % KP;
        double c = 0.0;
        if (i < a.k && j <= i)
            c = ssum[tri_idx(i, j)] * sinv[i];
        cw->C[e] = c;
    }
    if (tid < KP) {
        const int j = tid;
        double s = 1.0;
        if (j < a.k) {
            const double cjj = ssum[tri_idx(j, j)] * sinv[j];
            s = cjj;
            if (!(cjj >= a.rho)) {
                s = a.rho;
                atomicAdd(&cw->clip_count, 1);
            }
            if (!isfinite(cjj))
                atomicOr(&cw->status, kStatusNonFinite);
        }
        cw->s[j] = s;
    }
    if (tid == 0)
        atomicExch(&a.cnt[1], 0u);
}

// ---------------------------------------------------------------------------
// Initialisation (one workgroup; not on the hot path): normalise the supplied
// players to the unit sphere, set [Bv]_i = v_i (Alg. 2), and form the
// normalisation and parent terms of the first iteration.
// ---------------------------------------------------------------------------
template <typename T, int KP>
__global__ void __launch_bounds__(kNT) k_init(T *V, T *G, int64_t d, int k, double rho, Coef *cw)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    __shared__ double part[kNT];
    __shared__ double nrm[KP];
    const int tid = threadIdx.x;
    // column norms of the raw players
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
    // C = V^T G (= V^T V) lower triangle and the norms of the normalised V
    for (int e = tid; e < TRI; e += kNT) {
        int i, j;
        tri_ij(e, i, j);
        double s = 0.0;
        for (int64_t f = 0; f < d; ++f)
            s += (double)V[f * KP + i] * (double)G[f * KP + j];
        cw->C[i * KP + j] = s; // scaled by inv_nrm below
    }
    __syncthreads();
    if (tid < KP) {
        const int i = tid;
        double inv = 0.0;
        if (i < k) {
            const double n2 = cw->C[i * KP + i];
            inv = 1.0 / sqrt(n2);
            if (!(n2 > 0.0) || !isfinite(inv))
                atomicOr(&cw->status, kStatusNonFinite);
        }
        cw->inv_nrm[i] = inv;
    }
    __syncthreads();
    for (int e = tid; e < KP * KP; e += kNT) {
        const int i = e / KP, j = e % KP;
        cw->C[e] = (i < k && j <= i) ? cw->C[e] * cw->inv_nrm[i] : 0.0;
    }
    __syncthreads();
    if (tid < KP) {
        const int j = tid;
        double s = 1.0;
        if (j < k) {
            s = cw->C[j * KP + j];
            if (!(s >= rho))
                s = rho;
        }
        cw->s[j] = s;
    }
}

// Read-out: out[i*d + f] = scale_i * S[f*KP + i] (column-major FP64), with
// scale_i = inv_nrm_i (players) times 1/sqrt(s_i) when B-normalising, or 1
// (auxiliary variable).
template <typename T, int KP>
__global__ void __launch_bounds__(kNT) k_readout(const T *S, int64_t d, int k, const Coef *cf, int mode,
                                                 double *out)
{
    const int64_t n = d * (int64_t)k;
    for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kNT) {
        const int i = (int)(e / d);
        const int64_t f = e % d;
        double sc = 1.0;
        if (mode >= 1)
            sc = cf->inv_nrm[i];
        if (mode == 2)
            sc /= sqrt(cf->s[i]);
        out[e] = sc * (double)S[f * KP + i];
    }
}

} // namespace sgep
