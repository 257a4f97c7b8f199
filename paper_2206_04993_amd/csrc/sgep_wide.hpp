// sgep_wide.hpp -- CDNA4 (gfx950) kernels of the large-d form of the
// stochastic gamma-EigenGame step (Alg. 2, M = 1) for minibatches stored in
// BF16 or in FP8-e4m3 with per-column FP32 scales, problem kinds CCA (two
// views, Sec. 1) and LDA (between-class A, within-class B, Sec. 1).
//
// The minibatch is the only large operand and is read by two products per
// iteration, X V and X^T W.  Both run on the BF16 MFMA (16x16x32, FP32
// accumulate).  X enters exactly (FP8 codes decode exactly to BF16); the FP32
// right-hand operands V and W are split into BF16 hi + lo, so each product is
// X V_hi + X V_lo and the operand keeps 16 significand bits.  The FP8 column
// scale s_f is folded into the V operand (X V = X_q (diag(s) V)) and applied
// to the rows of X^T W.  State (V, [Bv], Adam moments) is FP32, the k x k
// reductions and norms FP64.
//
// One iteration is three launches:
//   k_wfwd  raw P = X V (CCA also Q = Y V) for a 64-row block over one slice of
//           the features (split-K, the minibatch width d >> b), eight waves
//           each over a contiguous feature range, FP32 partials per slice.
//   k_wmid  sums the slices (fixed order), writes the products transposed as
//           BF16 hi/lo operand rows W (CCA: P then Q; LDA: P then the one-hot
//           class indicator of the labels), advances the step counter, and
//           reduces the previous iteration's per-workgroup state statistics
//           (v_i^T [Bv]_j, ||v_i||^2, LDA: class means times v_i) to totals.
//   k_wbwd  for one view and a run of 64-feature subtiles: X^T W over all rows
//           (X transposed in registers), the k x k Gram terms of the minibatch
//           recomputed from the W fragments already in registers (identical in
//           every workgroup, so no extra reduction pass), the coefficients,
//           and the fused epilogue: update direction, retraction step (SGD or
//           Adam), auxiliary update, the BF16 hi/lo V operand of the next
//           iteration, and this workgroup's FP64 partial statistics.
// The stored V is lazily normalised as in sgep_kernels.hpp: P and W are raw
// products with the stored V, and the norm totals scale every use.
#pragma once

#include "sgep_kernels.hpp"

namespace sgep {
namespace wide {

constexpr int kWT = 512;       // threads per workgroup: eight wave64
constexpr int kNW = kWT / 64;  // waves per workgroup
constexpr int kFT = 64;        // features per backward subtile
constexpr int kRB = 64;        // minibatch rows per forward workgroup
constexpr int kMaxCls = 16;    // LDA classes
constexpr int kInBF16 = 0;
constexpr int kInFP8 = 1;
constexpr int kKindLDA = 2;
constexpr int kStatusBadLabel = 2;
constexpr int kStatCols = 16;  // statistics columns per reduction workgroup of k_wmid

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

struct WideArgs {
    const void *X, *Y;          // views (LDA: X only), row-major, 16-byte aligned rows
    const int32_t *labels;      // LDA: class of each row
    int64_t ldx, ldy, b;
    int64_t dv[2];              // view widths (multiples of 8)
    int64_t off[2];             // first state row of each view (multiples of kFT)
    int64_t dtot;               // state rows: views padded to multiples of kFT
    int32_t nview, k, ncls;
    // forward decomposition: block = (split, view, 64-row block), row blocks fastest
    int32_t n_rb, n_split;
    int32_t nA;                 // k_wmid row workgroups: 16 rows each, 4 n_rb
    int64_t fs, fw;             // features per split and per wave (multiples of 64)
    int64_t ldr;                // padded rows (multiple of kRB) of the partials and of W
    // backward decomposition: workgroups [0, nwg0) cover view 0, the rest view 1;
    // each covers nsub consecutive subtiles of its view (nsubv[v] subtiles in all)
    int32_t nwg0, nwg, nsub;
    int32_t nsubv[2];
    float *V, *G, *Am, *As;     // dtot x KP, feature-major
    uint16_t *Vh, *Vl;          // KP x dtot, player-major BF16 hi / lo of s_f V
    const float *colscale;      // dtot (FP8 only): s_f, 0 on padding
    float *Ppart;               // [n_split][nview][ldr][KP]
    uint16_t *Wh, *Wl;          // [MW][ldr]
    const float *M;             // LDA: ncls x dtot class means
    const float *Mbar;          // LDA: dtot, prior-weighted mean of the class means
    const double *prior;        // LDA: ncls
    double *spart;              // [Ws][lds], column = backward workgroup
    double *stot;               // [Ws]
    int32_t lds, Ws;
    Coef *coef;
    int32_t schedule;
    double eta0, eta_T, t0, t_c, T, gamma, rho, eps_reg, adam_b1, adam_b2, adam_eps;
};

__device__ inline double eta_sched(const WideArgs &a, double t)
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

// BF16 round-to-nearest-even bits of x, and the BF16 hi + lo split of x.
__device__ __forceinline__ uint32_t bf16_rne(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_val(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ void split_bf16(float x, uint32_t &hi, uint32_t &lo)
{
    hi = bf16_rne(x);
    lo = bf16_rne(x - bf16_val(hi));
}

__device__ __forceinline__ f32x4 mfma_bf16(u32x4 a, u32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Four FP8-e4m3 codes (one dword) to BF16: features 0,1 in d0 and 2,3 in d1.
__device__ __forceinline__ void fp8x4_to_bf16(uint32_t w, uint32_t &d0, uint32_t &d1)
{
    d0 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, 1.0f, false));
    d1 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, 1.0f, true));
}

template <int KP, int KIND> struct Shape {
    static constexpr int NT = KP / 16;                               // 16-player tiles
    static constexpr int MW = (KIND == kKindLDA) ? KP + 16 : 2 * KP; // rows of W
    static constexpr int NU = MW / 16;
    static constexpr int MWP = MW + 4;                               // LDS row of the products
    static constexpr int TRI = KP * (KP + 1) / 2;
    static constexpr int SLOT = kFT * MWP;                           // floats per reduction slot
    // Gram terms per wave and in total (CCA: P^T Q, then sum P^2, sum Q^2 per
    // lane group; LDA: L^T P, sum P^2 per lane group, class counts per group)
    static constexpr int GW = (KIND == kKindLDA) ? 16 * KP + 4 * KP + 4 * 16 : KP * KP + 8 * KP;
    static constexpr int GT = (KIND == kKindLDA) ? 16 * KP + KP + 16 : KP * KP + 2 * KP;
    // statistics tiles: lower 16x16 tiles of V^T G, then (LDA) M V tiles
    static constexpr int NST = NT * (NT + 1) / 2 + ((KIND == kKindLDA) ? NT : 0);
};

// ---------------------------------------------------------------------------
// Forward products.  Lane l (row r = l % 16 of a 16-row tile, group g = l / 16)
// holds features f0 + 16 g + 8 m + j (j < 8) of MFMA chunk m in {0, 1} of a
// 64-feature step, and the V operand holds the same features of player
// l % 16 of a 16-player tile, so every 16-byte load is one contiguous piece
// of a row of X or of the player-major V operand; the pairing of k-indices to
// features is the same in both operands, so the sum is unchanged.
// ---------------------------------------------------------------------------
template <int KP, int IN>
__global__ void __launch_bounds__(kWT) k_wfwd(WideArgs a)
{
    constexpr int NT = KP / 16;
    __shared__ float red[4][kRB * KP];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    int blk = blockIdx.x;
    const int rb = blk % a.n_rb;
    blk /= a.n_rb;
    const int v = blk % a.nview;
    const int s = blk / a.nview;
    const int64_t dv = a.dv[v];
    const int64_t ld = v ? a.ldy : a.ldx;
    const uint8_t *Xb = (const uint8_t *)(v ? a.Y : a.X);
    const int64_t row0 = (int64_t)rb * kRB;
    const int64_t fbeg = (int64_t)s * a.fs + (int64_t)w * a.fw;
    const int64_t fend = (fbeg + a.fw < dv) ? fbeg + a.fw : dv;
    const uint16_t *Vh = a.Vh + a.off[v] + (int64_t)r16 * a.dtot;
    const uint16_t *Vl = a.Vl + a.off[v] + (int64_t)r16 * a.dtot;

    f32x4 acc[4][NT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u)
            acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int64_t f0 = fbeg; f0 < fend; f0 += 64) {
        u32x4 xa[4][2], vh[NT][2], vl[NT][2];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t row = row0 + 16 * t + r16;
            const bool rok = row < a.b;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int64_t fu = f0 + 16 * g + 8 * m;
                const bool ok = rok && fu < dv;
                if (IN == kInBF16) {
                    xa[t][m] = ok ? *reinterpret_cast<const u32x4 *>(Xb + 2 * (row * ld + fu))
                                  : u32x4{0u, 0u, 0u, 0u};
                } else {
                    const u32x2 q = ok ? *reinterpret_cast<const u32x2 *>(Xb + row * ld + fu)
                                       : u32x2{0u, 0u};
                    uint32_t e0, e1, e2, e3;
                    fp8x4_to_bf16(q[0], e0, e1);
                    fp8x4_to_bf16(q[1], e2, e3);
                    xa[t][m] = u32x4{e0, e1, e2, e3};
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int64_t vo = (int64_t)16 * u * a.dtot + f0 + 16 * g + 8 * m;
                vh[u][m] = *reinterpret_cast<const u32x4 *>(Vh + vo);
                vl[u][m] = *reinterpret_cast<const u32x4 *>(Vl + vo);
            }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int u = 0; u < NT; ++u) {
                    acc[t][u] = mfma_bf16(xa[t][m], vh[u][m], acc[t][u]);
                    acc[t][u] = mfma_bf16(xa[t][m], vl[u][m], acc[t][u]);
                }
    }

    // eight waves -> one 64 x KP partial: waves 4..7 park, 0..3 add, four-slot sum
    // D layout: lane l, register q holds row 4 (l/16) + q, column l % 16
    if (w >= 4) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    red[w - 4][(16 * t + 4 * g + q) * KP + 16 * u + r16] = acc[t][u][q];
    }
    __syncthreads();
    if (w < 4) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float *p = &red[w][(16 * t + 4 * g + q) * KP + 16 * u + r16];
                    *p = acc[t][u][q] + *p;
                }
    }
    __syncthreads();
    float *out = a.Ppart + (((int64_t)s * a.nview + v) * a.ldr + row0) * KP;
    for (int e = tid; e < kRB * KP; e += kWT)
        out[e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// ---------------------------------------------------------------------------
// Middle pass.  Blocks [0, ldr / 16): 16 rows each -- sum the forward slices,
// write W (BF16 hi/lo, row m of W holds column m of [P | Q] or of [P | L]
// over the minibatch rows), advance the step counter (block 0).  The other
// blocks (all of them when stats_only): kStatCols statistics columns each,
// summed over the backward workgroups in a fixed order.
// ---------------------------------------------------------------------------
template <int KP, int KIND>
__global__ void __launch_bounds__(kWT) k_wmid(WideArgs a, int stats_only)
{
    constexpr int NV = (KIND == kKindLDA) ? 1 : 2;
    __shared__ float tile[16 * NV * KP];
    __shared__ double wsum[kNW][64];
    const int tid = threadIdx.x;
    const int nA = stats_only ? 0 : a.nA;
    if ((int)blockIdx.x < nA) {
        const int q = blockIdx.x;
        const int64_t r0 = (int64_t)q * 16;
        for (int e = tid; e < 16 * NV * KP; e += kWT) {
            const int rl = e / (NV * KP), rem = e % (NV * KP);
            const int vv = rem / KP, c = rem % KP;
            float s = 0.f;
            for (int sp = 0; sp < a.n_split; ++sp)
                s += a.Ppart[(((int64_t)sp * a.nview + vv) * a.ldr + r0 + rl) * KP + c];
            tile[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < NV * KP * 16; e += kWT) {
            const int m = e / 16, rl = e % 16;
            uint32_t hi, lo;
            split_bf16(tile[rl * NV * KP + m], hi, lo);
            a.Wh[(int64_t)m * a.ldr + r0 + rl] = (uint16_t)hi;
            a.Wl[(int64_t)m * a.ldr + r0 + rl] = (uint16_t)lo;
        }
        if (KIND == kKindLDA) {
            for (int e = tid; e < 16 * 16; e += kWT) {
                const int c = e / 16, rl = e % 16;
                const int64_t row = r0 + rl;
                uint16_t one = 0;
                if (row < a.b) {
                    const int lab = a.labels[row];
                    if (lab < 0 || lab >= a.ncls) {
                        if (c == 0)
                            atomicOr(&a.coef->status, kStatusBadLabel);
                    } else if (lab == c) {
                        one = 0x3F80; // 1.0
                    }
                }
                a.Wh[(int64_t)(KP + c) * a.ldr + row] = one;
            }
        }
        if (q == 0 && tid == 0)
            a.coef->t += 1.0;
        return;
    }
    // statistics columns: one wave per column, lanes over workgroups, fixed order
    const int qb = blockIdx.x - nA;
    const int lane = tid & 63, w = tid >> 6;
    for (int cc = w; cc < kStatCols; cc += kNW) {
        const int e = qb * kStatCols + cc;
        double s = 0.0;
        if (e < a.Ws)
            for (int j = lane; j < a.nwg; j += 64)
                s += a.spart[(int64_t)e * a.lds + j];
        wsum[w][lane] = s;
        __syncthreads();
        if (lane == 0 && e < a.Ws) {
            double tot = 0.0;
            for (int j = 0; j < 64; ++j)
                tot += wsum[w][j];
            a.stot[e] = tot;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Statistics of a finished 64-feature tile (new players Vn, new auxiliary Gn,
// LDS, feature-major, KP per row; LDA: class means Mt, 16 x 64): FP64 MFMA
// (16x16x4) over the tile's features, accumulated in sacc over the subtiles
// of a workgroup.  Wave w owns statistics tiles w and w + 8.
// ---------------------------------------------------------------------------
template <int KP, int KIND>
__device__ __forceinline__ void tile_stats(const float *Vn, const float *Gn, const float *Mt,
                                           f64x4 (&sacc)[2])
{
    typedef Shape<KP, KIND> S;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int l16 = lane & 15, g = lane >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int st = w + kNW * h;
        if (st >= S::NST)
            continue;
        int u, u2;
        bool mv = false;
        if (st < S::NT * (S::NT + 1) / 2) {
            // st -> (u, u2), u >= u2, row-major over the lower triangle
            u = 0;
            while ((u + 1) * (u + 2) / 2 <= st)
                ++u;
            u2 = st - u * (u + 1) / 2;
        } else {
            mv = true;
            u = 0;
            u2 = st - S::NT * (S::NT + 1) / 2;
        }
        f64x4 acc = sacc[h];
#pragma unroll 4
        for (int k4 = 0; k4 < kFT; k4 += 4) {
            const int fl = k4 + g;
            const double av = mv ? (double)Mt[l16 * kFT + fl] : (double)Vn[fl * KP + 16 * u + l16];
            const double bv = mv ? (double)Vn[fl * KP + 16 * u2 + l16] : (double)Gn[fl * KP + 16 * u2 + l16];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        sacc[h] = acc;
    }
}

template <int KP, int KIND>
__device__ __forceinline__ void write_stats(const WideArgs &a, int wg, const f64x4 (&sacc)[2],
                                            double nrm)
{
    typedef Shape<KP, KIND> S;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, g = lane >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int st = w + kNW * h;
        if (st >= S::NST)
            continue;
        if (st < S::NT * (S::NT + 1) / 2) {
            int u = 0;
            while ((u + 1) * (u + 2) / 2 <= st)
                ++u;
            const int u2 = st - u * (u + 1) / 2;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * u + g + 4 * r, j = 16 * u2 + l16; // FP64 D row (l/16) + 4 r
                if (j <= i)
                    a.spart[(int64_t)tri_idx(i, j) * a.lds + wg] = sacc[h][r];
            }
        } else {
            const int u2 = st - S::NT * (S::NT + 1) / 2;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = g + 4 * r, j = 16 * u2 + l16;
                if (c < a.ncls)
                    a.spart[(int64_t)(S::TRI + KP + c * KP + j) * a.lds + wg] = sacc[h][r];
            }
        }
    }
    if (tid < KP)
        a.spart[(int64_t)(S::TRI + tid) * a.lds + wg] = nrm;
}

// Player-major BF16 hi/lo operand of s_f Vn for the 64 features of a tile
// (two features per thread per pass, one 128-byte run per player).
template <int KP, int IN>
__device__ __forceinline__ void write_vop(const WideArgs &a, const float *Vn, int64_t frow)
{
    for (int e = threadIdx.x; e < KP * (kFT / 2); e += kWT) {
        const int i = e / (kFT / 2), fl = 2 * (e % (kFT / 2));
        float x0 = Vn[fl * KP + i], x1 = Vn[(fl + 1) * KP + i];
        if (IN == kInFP8) {
            x0 *= a.colscale[frow + fl];
            x1 *= a.colscale[frow + fl + 1];
        }
        uint32_t h0, l0, h1, l1;
        split_bf16(x0, h0, l0);
        split_bf16(x1, h1, l1);
        const int64_t o = (int64_t)i * a.dtot + frow + fl;
        *reinterpret_cast<uint32_t *>(a.Vh + o) = h0 | (h1 << 16);
        *reinterpret_cast<uint32_t *>(a.Vl + o) = l0 | (l1 << 16);
    }
}

__device__ __forceinline__ void wg_range(const WideArgs &a, int wg, int &v, int &sub0, int &sub1)
{
    if (wg < a.nwg0) {
        v = 0;
        sub0 = wg * a.nsub;
    } else {
        v = 1;
        sub0 = (wg - a.nwg0) * a.nsub;
    }
    sub1 = sub0 + a.nsub < a.nsubv[v] ? sub0 + a.nsub : a.nsubv[v];
}

// ---------------------------------------------------------------------------
// Backward products, coefficients and fused epilogue.
// Main loop over 32-row chunks (wave w takes chunks w, w + 8, ...): lane l
// (n = l % 16, g = l / 16) loads rows 8 g .. 8 g + 7 of the chunk at features
// 4 n .. 4 n + 3 of the subtile and transposes them in registers, so MFMA c
// (c < 4) gets the B operand B[8 g + j][n] = X[row 8 g + j][feature 4 n + c];
// the A operand is a 16-row tile of W, lane l holding W[l % 16][rows 8 g ..
// 8 g + 7] in one 16-byte load.  D[m][n] is then (X^T W^T)[4 n + c][m].
// ---------------------------------------------------------------------------
template <int KP, int IN, int KIND, int OPT>
__global__ void __launch_bounds__(kWT) k_wbwd(WideArgs a)
{
    typedef Shape<KP, KIND> S;
    constexpr int NT = S::NT, NU = S::NU, MWP = S::MWP, SLOT = S::SLOT, TRI = S::TRI;
    constexpr bool LDA = KIND == kKindLDA;
    constexpr int NC = LDA ? kMaxCls : 1;
    __shared__ __attribute__((aligned(16))) float red[4 * SLOT];
    __shared__ float Tl[KP * KP];
    __shared__ double gd[S::GT];
    __shared__ float cInv[KP], cMB[KP], cMAc[KP];
    __shared__ double dInv[KP], dS[KP];
    __shared__ float cMV[NC * KP], cSp[NC * KP], cU[NC * KP];
    __shared__ double dMc[NC * KP];
    __shared__ float Mt[NC * kFT], Mb[LDA ? kFT : 1];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int wg = xcd_tile(blockIdx.x, gridDim.x);
    int v, sub0, sub1;
    wg_range(a, wg, v, sub0, sub1);
    const int64_t dv = a.dv[v];
    const int64_t ld = v ? a.ldy : a.ldx;
    const uint8_t *Xb = (const uint8_t *)(v ? a.Y : a.X);
    const int nch = (int)((a.b + 31) / 32);
    const double t = a.coef->t; // this iteration's number, set by k_wmid
    const double ib = 1.0 / (double)a.b;

    f64x4 sacc[2] = {f64x4{0, 0, 0, 0}, f64x4{0, 0, 0, 0}};
    double nrm = 0.0;

    for (int sub = sub0; sub < sub1; ++sub) {
        const bool first = sub == sub0;
        const int64_t fv0 = (int64_t)sub * kFT;
        f32x4 acc[4][NU];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int u = 0; u < NU; ++u)
                acc[c][u] = f32x4{0.f, 0.f, 0.f, 0.f};
        f32x4 gacc[LDA ? NT : NT * NT];
#pragma unroll
        for (int u = 0; u < (LDA ? NT : NT * NT); ++u)
            gacc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        float dP[NT], dQ[NT], ncnt = 0.f;
#pragma unroll
        for (int u = 0; u < NT; ++u)
            dP[u] = dQ[u] = 0.f;

        const int64_t fu = fv0 + 4 * l16;
        const bool fok = fu < dv;
        for (int ch = w; ch < nch; ch += kNW) {
            const int64_t r0 = (int64_t)ch * 32;
            uint32_t d0[8], d1[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t row = r0 + 8 * g + j;
                const bool ok = fok && row < a.b;
                if (IN == kInBF16) {
                    const u32x2 q = ok ? *reinterpret_cast<const u32x2 *>(Xb + 2 * (row * ld + fu))
                                       : u32x2{0u, 0u};
                    d0[j] = q[0];
                    d1[j] = q[1];
                } else {
                    const uint32_t q = ok ? *reinterpret_cast<const uint32_t *>(Xb + row * ld + fu) : 0u;
                    fp8x4_to_bf16(q, d0[j], d1[j]);
                }
            }
            u32x4 wh[NU], wl[NU];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int64_t wo = (int64_t)(16 * u + l16) * a.ldr + r0 + 8 * g;
                wh[u] = *reinterpret_cast<const u32x4 *>(a.Wh + wo);
                if (!(LDA && u == NT))
                    wl[u] = *reinterpret_cast<const u32x4 *>(a.Wl + wo);
                else
                    wl[u] = u32x4{0u, 0u, 0u, 0u};
            }
            __builtin_amdgcn_sched_barrier(0);
            u32x4 bx[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t a0 = d0[2 * q], a1 = d0[2 * q + 1];
                const uint32_t b0 = d1[2 * q], b1 = d1[2 * q + 1];
                bx[0][q] = (a0 & 0xFFFFu) | (a1 << 16);
                bx[1][q] = (a0 >> 16) | (a1 & 0xFFFF0000u);
                bx[2][q] = (b0 & 0xFFFFu) | (b1 << 16);
                bx[3][q] = (b0 >> 16) | (b1 & 0xFFFF0000u);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    acc[c][u] = mfma_bf16(wh[u], bx[c], acc[c][u]);
                    if (!(LDA && u == NT))
                        acc[c][u] = mfma_bf16(wl[u], bx[c], acc[c][u]);
                }
            if (first) {
                // Gram terms from the W fragments: lane (m, g) holds rows 8g..8g+7 of
                // W row m, which is both the A layout (A[m][k]) and the B layout
                // (B[k][m]) of a 16x16x32 MFMA over those 32 rows.
                if (!LDA) {
#pragma unroll
                    for (int up = 0; up < NT; ++up)
#pragma unroll
                        for (int uq = 0; uq < NT; ++uq) {
                            f32x4 &ga = gacc[up * NT + uq];
                            ga = mfma_bf16(wh[up], wh[NT + uq], ga);
                            ga = mfma_bf16(wh[up], wl[NT + uq], ga);
                            ga = mfma_bf16(wl[up], wh[NT + uq], ga);
                        }
                } else {
#pragma unroll
                    for (int u = 0; u < NT; ++u) {
                        gacc[u] = mfma_bf16(wh[NT], wh[u], gacc[u]);
                        gacc[u] = mfma_bf16(wh[NT], wl[u], gacc[u]);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        ncnt += bf16_val(wh[NT][q] & 0xFFFFu) + bf16_val(wh[NT][q] >> 16);
                }
#pragma unroll
                for (int u = 0; u < NT; ++u)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float p0 = bf16_val(wh[u][q] & 0xFFFFu) + bf16_val(wl[u][q] & 0xFFFFu);
                        const float p1 = bf16_val(wh[u][q] >> 16) + bf16_val(wl[u][q] >> 16);
                        dP[u] += p0 * p0 + p1 * p1;
                        if (!LDA) {
                            const float q0 = bf16_val(wh[NT + u][q] & 0xFFFFu) + bf16_val(wl[NT + u][q] & 0xFFFFu);
                            const float q1 = bf16_val(wh[NT + u][q] >> 16) + bf16_val(wl[NT + u][q] >> 16);
                            dQ[u] += q0 * q0 + q1 * q1;
                        }
                    }
            }
        }

        // ---- products: eight waves -> prod = slot 0, element (feature, m) ----
        if (w >= 4) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int u = 0; u < NU; ++u)
                    *reinterpret_cast<f32x4 *>(&red[(w - 4) * SLOT + (4 * l16 + c) * MWP + 16 * u + 4 * g]) =
                        acc[c][u];
        }
        __syncthreads();
        if (w < 4) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    f32x4 *p = reinterpret_cast<f32x4 *>(&red[w * SLOT + (4 * l16 + c) * MWP + 16 * u + 4 * g]);
                    *p = acc[c][u] + *p;
                }
        }
        __syncthreads();
        for (int e = tid; e < kFT * S::MW; e += kWT) {
            const int idx = (e / S::MW) * MWP + e % S::MW;
            red[idx] = ((red[idx] + red[SLOT + idx]) + red[2 * SLOT + idx]) + red[3 * SLOT + idx];
        }
        __syncthreads();
        float *ext = red + SLOT; // three free slots from here on

        if (first) {
            // ---- Gram terms: eight waves x lane groups, fixed-order sum ----
            float *gw = ext + w * S::GW;
            if (!LDA) {
#pragma unroll
                for (int up = 0; up < NT; ++up)
#pragma unroll
                    for (int uq = 0; uq < NT; ++uq)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            gw[(16 * up + 4 * g + q) * KP + 16 * uq + l16] = gacc[up * NT + uq][q];
#pragma unroll
                for (int u = 0; u < NT; ++u) {
                    gw[KP * KP + g * KP + 16 * u + l16] = dP[u];
                    gw[KP * KP + 4 * KP + g * KP + 16 * u + l16] = dQ[u];
                }
            } else {
#pragma unroll
                for (int u = 0; u < NT; ++u)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        gw[(4 * g + q) * KP + 16 * u + l16] = gacc[u][q];
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    gw[16 * KP + g * KP + 16 * u + l16] = dP[u];
                gw[20 * KP + g * 16 + l16] = ncnt;
            }
            __syncthreads();
            for (int e = tid; e < S::GT; e += kWT) {
                double s = 0.0;
                if (!LDA) {
                    if (e < KP * KP) {
                        for (int ww = 0; ww < kNW; ++ww)
                            s += (double)ext[ww * S::GW + e];
                    } else {
                        const int which = (e - KP * KP) / KP, col = (e - KP * KP) % KP;
                        for (int ww = 0; ww < kNW; ++ww)
                            for (int gg = 0; gg < 4; ++gg)
                                s += (double)ext[ww * S::GW + KP * KP + which * 4 * KP + gg * KP + col];
                    }
                } else {
                    if (e < 16 * KP) {
                        for (int ww = 0; ww < kNW; ++ww)
                            s += (double)ext[ww * S::GW + e];
                    } else if (e < 17 * KP) {
                        const int col = e - 16 * KP;
                        for (int ww = 0; ww < kNW; ++ww)
                            for (int gg = 0; gg < 4; ++gg)
                                s += (double)ext[ww * S::GW + 16 * KP + gg * KP + col];
                    } else {
                        const int c = e - 17 * KP;
                        for (int ww = 0; ww < kNW; ++ww)
                            for (int gg = 0; gg < 4; ++gg)
                                s += (double)ext[ww * S::GW + 20 * KP + gg * 16 + c];
                    }
                }
                gd[e] = s;
            }
            __syncthreads();

            // ---- k x k coefficients (identical in every workgroup) ----
            double *ss = reinterpret_cast<double *>(ext);
            for (int e = tid; e < a.Ws; e += kWT)
                ss[e] = a.stot[e];
            __syncthreads();
            if (tid < KP) {
                const int i = tid;
                double inv = 0.0, s = 1.0;
                if (i < a.k) {
                    inv = 1.0 / sqrt(ss[TRI + i]);
                    s = ss[tri_idx(i, i)] * inv;
                    if (!(s >= a.rho))
                        s = a.rho;
                }
                dInv[i] = inv;
                dS[i] = s;
            }
            __syncthreads();
            if (LDA) {
                // raw M V, the class-sum terms, and the centred normalised class-mean
                // projections Mc_ci = (mu_c - mubar)^T v_i (FP64) with cU = pi_c Mc_ci
                for (int e = tid; e < kMaxCls * KP; e += kWT) {
                    const int c = e / KP, i = e % KP;
                    float mv = 0.f, sp = 0.f;
                    if (c < a.ncls && i < a.k) {
                        const double mvr = ss[TRI + KP + c * KP + i];
                        mv = (float)mvr;
                        sp = (float)(gd[c * KP + i] - gd[17 * KP + c] * mvr);
                    }
                    cMV[e] = mv;
                    cSp[e] = sp;
                }
                if (tid < KP) {
                    const int i = tid;
                    double mbar = 0.0;
                    if (i < a.k)
                        for (int c = 0; c < a.ncls; ++c)
                            mbar += a.prior[c] * ss[TRI + KP + c * KP + i] * dInv[i];
                    for (int c = 0; c < kMaxCls; ++c) {
                        double mc = 0.0;
                        if (c < a.ncls && i < a.k)
                            mc = ss[TRI + KP + c * KP + i] * dInv[i] - mbar;
                        dMc[c * KP + i] = mc;
                        cU[c * KP + i] = (float)((c < a.ncls ? a.prior[c] : 0.0) * mc);
                    }
                }
            }
            __syncthreads();
            // (M_A)_ij: CCA b^-1 inv_i inv_j (P^T Q + Q^T P)_ij; LDA sum_c pi_c Mc_ci Mc_cj
            auto MA = [&](int i, int j) -> double {
                if (!LDA)
                    return (gd[i * KP + j] + gd[j * KP + i]) * dInv[i] * dInv[j] * ib;
                double s = 0.0;
                for (int c = 0; c < a.ncls; ++c)
                    s += a.prior[c] * dMc[c * KP + i] * dMc[c * KP + j];
                return s;
            };
            for (int e = tid; e < KP * KP; e += kWT) {
                const int i = e / KP, j = e % KP;
                double val = 0.0;
                if (i < a.k && j < i)
                    val = MA(i, j) / dS[j];
                Tl[e] = (float)val;
            }
            Coef *cw = a.coef;
            if (tid < KP) {
                const int i = tid;
                double mA = 0.0, mB = 0.0, c = 0.0;
                if (i < a.k) {
                    const double ii2 = dInv[i] * dInv[i];
                    mA = MA(i, i);
                    if (!LDA) {
                        mB = (gd[KP * KP + i] + gd[KP * KP + KP + i]) * ii2 * ib;
                    } else {
                        double q = gd[16 * KP + i];
                        for (int cc = 0; cc < a.ncls; ++cc) {
                            const double mvr = ss[TRI + KP + cc * KP + i];
                            q += -2.0 * mvr * gd[cc * KP + i] + gd[17 * KP + cc] * mvr * mvr;
                        }
                        mB = q * ii2 * ib + a.eps_reg;
                    }
                    for (int j = 0; j < i; ++j)
                        c += MA(i, j) / dS[j] * (ss[tri_idx(i, j)] * dInv[i]); // T_ij C_ij
                }
                cMB[i] = (float)mB;
                cMAc[i] = (float)(mA - c);
                cInv[i] = (float)dInv[i];
                if (wg == 0) {
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
                        cw->eta = eta_sched(a, t);
                        cw->gamma = a.gamma;
                    }
                }
            }
            __syncthreads();
        }

        // ---- fused epilogue over the subtile's 64 features x KP players ----
        const int64_t frow = a.off[v] + fv0; // state row of the subtile's first feature
        float *Gold = ext, *Vn = ext + kFT * KP, *Gn = ext + 2 * kFT * KP;
        for (int e = tid; e < kFT * KP; e += kWT)
            Gold[e] = a.G[frow * KP + e];
        if (LDA) {
            for (int e = tid; e < kMaxCls * kFT; e += kWT) {
                const int c = e / kFT, fl = e % kFT;
                Mt[e] = c < a.ncls ? a.M[(int64_t)c * a.dtot + frow + fl] : 0.f;
            }
            for (int e = tid; e < kFT; e += kWT)
                Mb[e] = a.Mbar[frow + e];
        }
        __syncthreads();
        const float eta = (float)eta_sched(a, t), gam = (float)a.gamma, ibf = (float)ib;
        const float eps = (float)a.eps_reg;
        const float b1 = (float)a.adam_b1, b2 = (float)a.adam_b2, aeps = (float)a.adam_eps;
        const float c1 = (float)(1.0 - pow(a.adam_b1, t)), c2 = (float)(1.0 - pow(a.adam_b2, t));
        for (int e = tid; e < kFT * KP; e += kWT) {
            const int fl = e / KP, i = e % KP;
            const int64_t si = frow * KP + e;
            float vn = 0.f, gn = 0.f;
            if (fv0 + fl < dv && i < a.k) {
                const float inv = cInv[i];
                const float vh = a.V[si] * inv;
                const float *pr = red + fl * MWP;
                float av, bv;
                if (!LDA) {
                    const float sf = IN == kInFP8 ? a.colscale[frow + fl] : 1.f;
                    const float rawA = v == 0 ? pr[KP + i] : pr[i];
                    const float rawB = v == 0 ? pr[i] : pr[KP + i];
                    av = rawA * sf * inv * ibf;
                    bv = rawB * sf * inv * ibf;
                } else {
                    float corr = 0.f, ma = 0.f;
                    for (int c = 0; c < a.ncls; ++c) {
                        corr += pr[KP + c] * cMV[c * KP + i] + Mt[c * kFT + fl] * cSp[c * KP + i];
                        ma += (Mt[c * kFT + fl] - Mb[fl]) * cU[c * KP + i];
                    }
                    bv = (pr[i] - corr) * inv * ibf + eps * vh;
                    av = ma;
                }
                float pen = 0.f;
                for (int j = 0; j < i; ++j)
                    pen += Tl[i * KP + j] * Gold[fl * KP + j];
                const float grad = (av - pen) * cMB[i] - bv * cMAc[i];
                if (OPT == kOptSGD) {
                    vn = vh + eta * grad;
                } else {
                    const float mm = b1 * a.Am[si] + (1.f - b1) * grad;
                    const float sq = b2 * a.As[si] + (1.f - b2) * grad * grad;
                    a.Am[si] = mm;
                    a.As[si] = sq;
                    vn = vh + eta * (mm / c1) / (sqrtf(sq / c2) + aeps);
                }
                const float g0 = Gold[e];
                gn = g0 + gam * (bv - g0);
                a.V[si] = vn;
                a.G[si] = gn;
            }
            Vn[e] = vn;
            Gn[e] = gn;
        }
        __syncthreads();
        write_vop<KP, IN>(a, Vn, frow);
        tile_stats<KP, KIND>(Vn, Gn, Mt, sacc);
        if (tid < KP)
            for (int fl = 0; fl < kFT; ++fl)
                nrm += (double)Vn[fl * KP + tid] * (double)Vn[fl * KP + tid];
        __syncthreads();
    }
    write_stats<KP, KIND>(a, wg, sacc, nrm);
}

// ---------------------------------------------------------------------------
// Initialisation (same workgroups as k_wbwd): the stored players V (unit
// columns, written by the host) give [Bv] = V (Alg. 2), the V operand and the
// first statistics.
// ---------------------------------------------------------------------------
template <int KP, int IN, int KIND>
__global__ void __launch_bounds__(kWT) k_winit(WideArgs a)
{
    __shared__ float Vn[kFT * KP];
    __shared__ float Mt[(KIND == kKindLDA ? kMaxCls : 1) * kFT];
    const int tid = threadIdx.x;
    const int wg = blockIdx.x;
    int v, sub0, sub1;
    wg_range(a, wg, v, sub0, sub1);
    f64x4 sacc[2] = {f64x4{0, 0, 0, 0}, f64x4{0, 0, 0, 0}};
    double nrm = 0.0;
    for (int sub = sub0; sub < sub1; ++sub) {
        const int64_t frow = a.off[v] + (int64_t)sub * kFT;
        for (int e = tid; e < kFT * KP; e += kWT) {
            const float x = a.V[frow * KP + e];
            Vn[e] = x;
            a.G[frow * KP + e] = x;
        }
        if (KIND == kKindLDA)
            for (int e = tid; e < kMaxCls * kFT; e += kWT) {
                const int c = e / kFT, fl = e % kFT;
                Mt[e] = c < a.ncls ? a.M[(int64_t)c * a.dtot + frow + fl] : 0.f;
            }
        __syncthreads();
        write_vop<KP, IN>(a, Vn, frow);
        tile_stats<KP, KIND>(Vn, Vn, Mt, sacc);
        if (tid < KP)
            for (int fl = 0; fl < kFT; ++fl)
                nrm += (double)Vn[fl * KP + tid] * (double)Vn[fl * KP + tid];
        __syncthreads();
    }
    write_stats<KP, KIND>(a, wg, sacc, nrm);
}

// Read-out after k_wmid(stats_only): out[i * d + f] (column-major FP64) =
// scale_i * S[row(f) * KP + i], scale as in k_readout (mode 0: 1, 1: 1/||V_i||,
// 2: additionally 1/sqrt(s_i)); row(f) maps feature f of the concatenated
// views to its state row.
template <int KP>
__global__ void __launch_bounds__(256) k_wreadout(const float *S, const double *stot, int64_t d,
                                                  int64_t dx, int64_t off1, int k, double rho,
                                                  Coef *cw, int mode, double *out)
{
    constexpr int TRI = KP * (KP + 1) / 2;
    __shared__ double scale[KP];
    if (threadIdx.x < KP) {
        const int i = threadIdx.x;
        double sc = 1.0;
        if (i < k) {
            const double inv = 1.0 / sqrt(stot[TRI + i]);
            if (blockIdx.x == 0 && (!isfinite(inv) || !(stot[TRI + i] > 0.0)))
                atomicOr(&cw->status, kStatusNonFinite);
            if (mode >= 1)
                sc = inv;
            if (mode == 2) {
                double s = stot[tri_idx(i, i)] * inv;
                if (!(s >= rho))
                    s = rho;
                sc /= sqrt(s);
            }
        }
        scale[i] = sc;
    }
    __syncthreads();
    const int64_t n = d * (int64_t)k;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e / d);
        const int64_t f = e % d;
        const int64_t row = f < dx ? f : off1 + (f - dx);
        out[e] = scale[i] * (double)S[row * KP + i];
    }
}

} // namespace wide
} // namespace sgep
