// sgep_wide.hpp -- CDNA4 (gfx950) kernels of the large-d form of the
// stochastic gamma-EigenGame step (Alg. 2, M = 1) for minibatches stored in
// BF16 or in FP8-e4m3 with per-column FP32 scales, problem kinds CCA (two
// views, Sec. 1) and LDA (between-class A, within-class B, Sec. 1); and the
// same decomposition for FP32 minibatches (LDA), on the FP32 MFMA.
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
//           Extra workgroups reduce the previous iteration's per-workgroup
//           state statistics (v_i^T [Bv]_j, ||v_i||^2, LDA: class means times
//           v_i) to totals.
//   k_wmid  sums the slices (fixed order) and writes the backward operand W,
//           transposed, as BF16 hi/lo rows: CCA [P | Q]; LDA the within-class
//           residual R = X V - (M V)[labels] and the one-hot class indicator L;
//           advances the step counter.
//   k_wbwd  for one view and a run of 64-feature subtiles: X^T W over all rows
//           (X transposed in registers), the k x k Gram terms of the minibatch
//           recomputed from the W fragments already in registers (identical in
//           every workgroup, so no extra reduction pass), the coefficients,
//           and the fused epilogue on MFMA tiles: parent penalty (and the LDA
//           class terms) as small products, update direction, retraction step
//           (SGD or Adam), auxiliary update, the BF16 hi/lo V operand of the
//           next iteration, and this workgroup's FP64 partial statistics.
// The stored V is lazily normalised as in sgep_kernels.hpp: P and W are raw
// products with the stored V, and the norm totals scale every use.
//
// Both streaming loops are software-pipelined: the loads of the next chunk are
// issued before the MFMAs of the current one.
//
// FP32 minibatches (kInF32) use the same launches, partials and epilogue with
// the 16x16x4 FP32 MFMA: the operands V and W are FP32 (player-major V copy
// Vf, W rows Wf), with no hi/lo split, and a lane's eight consecutive
// k-values of a 32-wide chunk feed eight MFMAs, MFMA j taking the lane's
// element j (the k-index l / 16 of MFMA j stands for k-value 8 (l / 16) + j;
// both operands use the same assignment, so each product sums every k-value
// once).
#pragma once

#include "sgep_kernels.hpp"

namespace sgep {
namespace wide {

constexpr int kWT = 512;       // threads per workgroup: eight wave64
constexpr int kNW = kWT / 64;  // waves per workgroup
constexpr int kFT = 64;        // features per backward subtile
constexpr int kRB = 64;        // row granularity of the forward partials and the middle pass
constexpr int kRowPad = 128;   // padding of the row dimension (256 with the four-wave forward)
// minibatch rows per forward workgroup: 64, or 128 (eight 16-row tiles per
// wave, so each V operand load serves twice the rows) where the accumulators
// and the reduction buffer fit (KP <= 32) and the minibatch is large enough to
// keep >= 256 workgroups busy (chosen at init)
constexpr int kMaxCls = 16;    // LDA classes
constexpr int kMR = 4;         // minibatch rows per middle-pass workgroup
constexpr int kMT = 256;       // threads per middle-pass workgroup
constexpr int kInBF16 = 0;
constexpr int kInFP8 = 1;
constexpr int kInF32 = 2;
constexpr int kKindLDA = 2;
constexpr int kStatusBadLabel = 2;
constexpr int kStatCols = 16;  // statistics columns per reduction workgroup
constexpr int kBT = 256;       // threads per backward workgroup: four wave64, one per SIMD
constexpr int kBW = kBT / 64;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
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
    int32_t rbf;                // rows per forward workgroup: 64 or 128, or 256 (k_wfwd4)
    int32_t nA;                 // k_wmid workgroups: kMR rows each, over the 64-row blocks
    int64_t fs, fw;             // features per split and per wave (multiples of 64)
    int64_t ldr;                // padded rows (multiple of the forward row block) of the partials and of W
    // backward decomposition: workgroups [0, nwg0) cover view 0, the rest view 1;
    // each covers nsub consecutive subtiles of its view (nsubv[v] subtiles in all)
    int32_t nwg0, nwg, nsub;
    int32_t nsubv[2];
    int32_t ft;                 // features per backward subtile: 64 (one kernel) or 128
                                // (products k_wprod, then the epilogue k_wepi per 64)
    int32_t nstat;              // columns of the statistics partials (writing workgroups)
    float *prod;                // ft = 128: X^T W per state row, [dtot][rows of W in X^T W]
    float *ctile;               // ft = 128: the iteration's coefficient tile (k_wprod -> k_wepi)
    float *V, *G, *Am, *As;     // dtot x KP, feature-major
    uint16_t *Vh, *Vl;          // KP x dtot, player-major BF16 hi / lo of s_f V
    float *Vf;                  // FP32 input: KP x dtot, player-major copy of V
    const float *colscale;      // dtot (FP8 only): s_f, 0 on padding
    float *Ppart;               // [n_split][nview][ldr][KP]
    uint16_t *Wh, *Wl;          // BF16 W: 1 KB tiles of 16 rows x 32 minibatch rows (w_idx)
    float *Wf;                  // FP32 input: [rows of W][ldr]
    const float *M;             // LDA: ncls x dtot class means
    const float *Mbar;          // LDA: dtot, prior-weighted mean of the class means
    const double *prior;        // LDA: ncls
    double *spart;              // statistics partials, column = backward workgroup (sp_idx)
    double *stot;               // [Ws]
    int32_t lds, Ws;
    Coef *coef;
    int32_t schedule;
    double eta0, eta_T, t0, t_c, T, gamma, rho, eps_reg, adam_b1, adam_b2, adam_eps;
    int32_t smooth;          // Alg. 3 estimate of v_j^T B v_j instead of the clip
    double lrho, lspan;      // Alg. 3: log rho, log nu - log rho
    // running-mean centring (CCA): mu, FP32 running means of the views at the
    // state rows (s_f-scaled true values, zero on padding); xsum, the split
    // backward's minibatch column sums (raw codes) from k_wprod to k_wepi
    int32_t center;
    float *mu, *xsum;
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

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Eight k-values per lane (two f32x4 of A and of B) through eight 16x16x4
// MFMAs: MFMA j takes element j of both.
__device__ __forceinline__ f32x4 mfma_f32x8(const f32x4 (&a)[2], const f32x4 (&b)[2], f32x4 c)
{
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            c = mfma_f32(a[h][j], b[h][j], c);
    return c;
}

// Four FP8-e4m3 codes (one dword) to BF16: features 0,1 in d0 and 2,3 in d1.
__device__ __forceinline__ void fp8x4_to_bf16(uint32_t w, uint32_t &d0, uint32_t &d1)
{
    d0 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, 1.0f, false));
    d1 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, 1.0f, true));
}

template <int KP, int KIND> struct Shape {
    static constexpr bool LDA = KIND == kKindLDA;
    static constexpr int NT = KP / 16;                 // 16-player tiles
    static constexpr int MWA = LDA ? KP : 2 * KP;      // rows of W in the products X^T W
    static constexpr int NU = MWA / 16;
    static constexpr int MWP = MWA + 4;                // LDS row of the products
    static constexpr int TRI = KP * (KP + 1) / 2;
    static constexpr int SLOT = kFT * MWP;             // floats per reduction slot
    static constexpr int GLD = KP + 4;                 // LDS row of the old auxiliary tile
    static constexpr int VLD = KP + 1;                 // LDS row of the new V, G tiles
    // Gram terms per wave (CCA: P^T Q, then per lane group sum P^2, sum Q^2,
    // sum P and sum Q -- the column sums of the centring; LDA: L^T R, then
    // sum R^2 per lane group) and in total
    static constexpr int GW = LDA ? 16 * KP + 4 * KP : KP * KP + 16 * KP;
    static constexpr int GT = LDA ? 16 * KP + KP : KP * KP + 4 * KP;
    static constexpr int NG = LDA ? NT : NT * NT;      // Gram MFMA tiles per wave
    // statistics tiles: lower 16x16 tiles of V^T G, then the mean tiles: LDA
    // the class means times V (16 rows), CCA the view's running mean times V
    // (row 0; zero without centring)
    static constexpr int NST = NT * (NT + 1) / 2 + NT;
    // 16-row tiles of the BF16 backward operand W (LDA: R, then the one-hot
    // rows of the classes; CCA: P, then Q)
    static constexpr int MWT = (LDA ? KP + kMaxCls : 2 * KP) / 16;
};

// Position of element (row m, minibatch row r) of the BF16 backward operand
// W (Wh, Wl): 32-row chunks, within a chunk 16-row tiles of 16 x 32 elements
// (1 KB), row-major inside the tile.  A wave's fragment load of one tile --
// lane (m % 16, g) taking rows 8 g .. 8 g + 7 -- is then one contiguous 1 KB.
template <int MWT>
__device__ __forceinline__ int64_t w_idx(int m, int64_t r)
{
    return (((r >> 5) * MWT + (m >> 4)) * 16 + (m & 15)) * 32 + (r & 31);
}

// ---------------------------------------------------------------------------
// Statistics partials: statistic e of workgroup column j sits in group e / 16,
// a [lds][16] block, so the 16 consecutive statistics of one workgroup are
// one 128-byte run (written together; read 4 columns x 16 per wave).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t sp_idx(const WideArgs &a, int e, int j)
{
    return ((int64_t)(e >> 4) * a.lds + j) * 16 + (e & 15);
}

// Statistics totals of group qb (kStatCols = 16 statistics): the partials of
// the latest backward pass (or of k_winit) summed over the nstat columns in a
// fixed order -- lane (e, q) of wave w over the columns j = 4 w + q (mod 4 NW),
// ascending, then the four q by a butterfly, then the waves in order.
// ---------------------------------------------------------------------------
static_assert(kStatCols == 16, "one 16-statistic group per reduction workgroup");
template <int NW = kNW>
__device__ inline void reduce_stats(const WideArgs &a, int qb)
{
    __shared__ double part[NW][16];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6); // wave index, scalar
    const int el = lane & 15;
    const double *p = a.spart + (int64_t)qb * a.lds * 16 + el;
    constexpr int JS = 4 * NW; // column stride of a lane
    int j = 4 * w + (lane >> 4);
    double s = 0.0;
    for (; j + 3 * JS < a.nstat; j += 4 * JS) {
        const double x0 = p[(int64_t)j * 16], x1 = p[(int64_t)(j + JS) * 16];
        const double x2 = p[(int64_t)(j + 2 * JS) * 16], x3 = p[(int64_t)(j + 3 * JS) * 16];
        s += x0;
        s += x1;
        s += x2;
        s += x3;
    }
    for (; j < a.nstat; j += JS)
        s += p[(int64_t)j * 16];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (lane < 16)
        part[w][el] = s;
    __syncthreads();
    if (tid < 16) {
        double t = part[0][tid];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww)
            t += part[ww][tid];
        const int e = qb * 16 + tid;
        if (e < a.Ws)
            a.stot[e] = t;
    }
}

__global__ void __launch_bounds__(kWT) k_wstats(WideArgs a) { reduce_stats(a, blockIdx.x); }

// ---------------------------------------------------------------------------
// Forward products.  Lane l (row r = l % 16 of a 16-row tile, group g = l / 16)
// holds features f0 + 8 g .. f0 + 8 g + 7 of a 32-feature MFMA chunk, the V
// operand the same features of player l % 16 of a 16-player tile: one 16-byte
// (BF16) or 8-byte (FP8) load per row tile, one per player tile and half.
// ---------------------------------------------------------------------------
template <int KP, int IN, int RBF>
__global__ void __launch_bounds__(kWT) k_wfwd(WideArgs a)
{
    constexpr int NT = KP / 16;
    static_assert(RBF == 64 || (RBF == 128 && KP <= 32), "forward row block");
    constexpr int TR = RBF / 16;       // 16-row MFMA tiles
    __shared__ float red[4][RBF * KP];
    const int nfwd = a.n_rb * a.nview * a.n_split;
    if ((int)blockIdx.x >= nfwd) {
        reduce_stats(a, (int)blockIdx.x - nfwd);
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6); // wave index, scalar
    const int r16 = lane & 15, g = lane >> 4;
    // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin, so
    // XCD x runs blockIdx x, x + 8, ...; give it a contiguous range of
    // (slice, view) pairs with all their row blocks, so the V operand of
    // those feature slices stays in that XCD's L2 instead of every XCD
    // reading all of V
    int blk = blockIdx.x;
    if (nfwd % 8 == 0 && (a.nview * a.n_split) % 8 == 0)
        blk = (blk % 8) * (nfwd / 8) + blk / 8;
    const int rb = blk % a.n_rb;
    blk /= a.n_rb;
    const int v = blk % a.nview;
    const int s = blk / a.nview;
    const int64_t dv = a.dv[v];
    const int64_t ld = v ? a.ldy : a.ldx;
    const uint8_t *Xb = (const uint8_t *)(v ? a.Y : a.X);
    constexpr int ES = IN == kInBF16 ? 2 : (IN == kInF32 ? 4 : 1);
    const int64_t row0 = (int64_t)rb * RBF;
    const int64_t fbeg = (int64_t)s * a.fs + (int64_t)w * a.fw;
    const int64_t fend = (fbeg + a.fw < dv) ? fbeg + a.fw : dv;
    const int nst = fend > fbeg ? (int)((fend - fbeg + 31) / 32) : 0;
    // Loads are unconditional, from clamped in-bounds addresses (a row past the
    // minibatch reads the last row, a feature unit past the view the last
    // unit); the data are zeroed where they are consumed.  Branch-free loads
    // let the next chunk stay in flight while the current one is multiplied.
    const uint8_t *xr[TR];
    bool rok[TR];
#pragma unroll
    for (int t = 0; t < TR; ++t) {
        const int64_t row = row0 + 16 * t + r16;
        rok[t] = row < a.b;
        xr[t] = Xb + (rok[t] ? row : a.b - 1) * ld * ES;
    }

    f32x4 acc[TR][NT];
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u)
            acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};

    if constexpr (IN == kInF32) {
        // one 32-feature chunk: eight FP32 features of X per row tile and of V
        // per player tile (two 16-byte loads each)
        const float *Vf = a.Vf + a.off[v] + (int64_t)r16 * a.dtot + 8 * g;
        auto load = [&](int st, f32x4(&xa)[TR][2], f32x4(&va)[NT][2]) {
            const int64_t f0 = fbeg + 32 * (int64_t)(st < nst ? st : nst - 1);
            const int64_t fx = f0 + 8 * g < dv ? f0 + 8 * g : dv - 8;
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                const float *p = reinterpret_cast<const float *>(xr[t]) + fx;
                xa[t][0] = *reinterpret_cast<const f32x4 *>(p);
                xa[t][1] = *reinterpret_cast<const f32x4 *>(p + 4);
            }
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const float *q = Vf + (int64_t)16 * u * a.dtot + f0;
                va[u][0] = *reinterpret_cast<const f32x4 *>(q);
                va[u][1] = *reinterpret_cast<const f32x4 *>(q + 4);
            }
        };
        auto mma = [&](int st, const f32x4(&xa)[TR][2], const f32x4(&va)[NT][2]) {
            if (st >= nst)
                return; // wave-uniform
            const bool fok = fbeg + 32 * (int64_t)st + 8 * g < dv;
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                f32x4 x[2] = {xa[t][0], xa[t][1]};
                if (!(fok && rok[t]))
                    x[0] = x[1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    acc[t][u] = mfma_f32x8(x, va[u], acc[t][u]);
            }
        };
        f32x4 xa0[TR][2], va0[NT][2], xa1[TR][2], va1[NT][2];
        if (nst > 0) {
            load(0, xa0, va0);
            for (int st = 0; st < nst; st += 2) {
                load(st + 1, xa1, va1);
                __builtin_amdgcn_sched_barrier(0);
                mma(st, xa0, va0);
                load(st + 2, xa0, va0);
                __builtin_amdgcn_sched_barrier(0);
                mma(st + 1, xa1, va1);
            }
        }
    } else {
        // one 32-feature chunk: raw X (BF16: 4 dwords; FP8: 2 dwords) and V hi/lo
        const uint16_t *Vh = a.Vh + a.off[v] + (int64_t)r16 * a.dtot + 8 * g;
        const uint16_t *Vl = a.Vl + a.off[v] + (int64_t)r16 * a.dtot + 8 * g;
        auto load = [&](int st, u32x4(&xa)[TR], u32x4(&vh)[NT], u32x4(&vl)[NT]) {
            const int64_t f0 = fbeg + 32 * (int64_t)(st < nst ? st : nst - 1);
            const int64_t fx = f0 + 8 * g < dv ? f0 + 8 * g : dv - 8;
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                if (IN == kInBF16) {
                    xa[t] = *reinterpret_cast<const u32x4 *>(xr[t] + 2 * fx);
                } else {
                    const u32x2 q = *reinterpret_cast<const u32x2 *>(xr[t] + fx);
                    xa[t] = u32x4{q[0], q[1], 0u, 0u};
                }
            }
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const int64_t vo = (int64_t)16 * u * a.dtot + f0;
                vh[u] = *reinterpret_cast<const u32x4 *>(Vh + vo);
                vl[u] = *reinterpret_cast<const u32x4 *>(Vl + vo);
            }
        };
        auto mma = [&](int st, const u32x4(&xa)[TR], const u32x4(&vh)[NT], const u32x4(&vl)[NT]) {
            if (st >= nst)
                return; // wave-uniform
            const bool fok = fbeg + 32 * (int64_t)st + 8 * g < dv;
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                u32x4 x = xa[t];
                if (IN == kInFP8) {
                    uint32_t e0, e1, e2, e3;
                    fp8x4_to_bf16(xa[t][0], e0, e1);
                    fp8x4_to_bf16(xa[t][1], e2, e3);
                    x = u32x4{e0, e1, e2, e3};
                }
                if (!(fok && rok[t]))
                    x = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
                for (int u = 0; u < NT; ++u) {
                    acc[t][u] = mfma_bf16(x, vh[u], acc[t][u]);
                    acc[t][u] = mfma_bf16(x, vl[u], acc[t][u]);
                }
            }
        };
        u32x4 xa0[TR], vh0[NT], vl0[NT], xa1[TR], vh1[NT], vl1[NT];
        if (nst > 0) {
            load(0, xa0, vh0, vl0);
            for (int st = 0; st < nst; st += 2) {
                load(st + 1, xa1, vh1, vl1);
                __builtin_amdgcn_sched_barrier(0);
                mma(st, xa0, vh0, vl0);
                load(st + 2, xa0, vh0, vl0);
                __builtin_amdgcn_sched_barrier(0);
                mma(st + 1, xa1, vh1, vl1);
            }
        }
    }

    // eight waves -> one RBF x KP partial: waves 4..7 park, 0..3 add, four-slot
    // sum.  D layout: lane l, register q holds row 4 (l/16) + q, column l % 16
    if (w >= 4) {
#pragma unroll
        for (int t = 0; t < TR; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    red[w - 4][(16 * t + 4 * g + q) * KP + 16 * u + r16] = acc[t][u][q];
    }
    __syncthreads();
    if (w < 4) {
#pragma unroll
        for (int t = 0; t < TR; ++t)
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
    for (int e = tid; e < RBF * KP; e += kWT)
        out[e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// ---------------------------------------------------------------------------
// Forward products with four waves of RBF rows each (k_wfwd4, BF16 / FP8):
// one wave per SIMD holds an RBF x KP accumulator (registers up to 512 per
// lane: RBF = 256 for KP <= 32, 128 for KP = 64), so every V operand load
// serves RBF rows instead of 64 -- a quarter (half) of the V traffic per byte
// of X.  The four waves take consecutive feature
// ranges of the workgroup's slice; their partials are summed through two
// LDS slots in a fixed order ((wave 0 + wave 2) + (wave 1 + wave 3)).
// Lane layout, operands and MFMAs as k_wfwd.
// ---------------------------------------------------------------------------
template <int KP, int IN>
__global__ void __launch_bounds__(256) k_wfwd4(WideArgs a)
{
    static_assert(IN == kInBF16 || IN == kInFP8, "BF16 / FP8 codes");
    constexpr int NT = KP / 16;
    constexpr int RBF = KP <= 32 ? 256 : 128;
    constexpr int TR = RBF / 16;
    __shared__ float red[2][RBF * KP];
    const int nfwd = a.n_rb * a.nview * a.n_split;
    if ((int)blockIdx.x >= nfwd) {
        reduce_stats<4>(a, (int)blockIdx.x - nfwd);
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6); // wave index, scalar
    const int r16 = lane & 15, g = lane >> 4;
    int blk = blockIdx.x; // XCD-aware order, as k_wfwd
    if (nfwd % 8 == 0 && (a.nview * a.n_split) % 8 == 0)
        blk = (blk % 8) * (nfwd / 8) + blk / 8;
    const int rb = blk % a.n_rb;
    blk /= a.n_rb;
    const int v = blk % a.nview;
    const int s = blk / a.nview;
    const int64_t dv = a.dv[v];
    const int64_t ld = v ? a.ldy : a.ldx;
    const uint8_t *Xb = (const uint8_t *)(v ? a.Y : a.X);
    constexpr int ES = IN == kInBF16 ? 2 : 1;
    const int64_t row0 = (int64_t)rb * RBF;
    const int64_t fbeg = (int64_t)s * a.fs + (int64_t)w * a.fw;
    const int64_t fend = (fbeg + a.fw < dv) ? fbeg + a.fw : dv;
    const int nst = fend > fbeg ? (int)((fend - fbeg + 31) / 32) : 0;
    // row t of the lane (16 t + r16 of the block), clamped to the minibatch
    const int64_t rlast = a.b - 1;
    uint32_t rok = 0; // bit t: row valid
#pragma unroll
    for (int t = 0; t < TR; ++t)
        if (row0 + 16 * t + r16 < a.b)
            rok |= 1u << t;
    const uint16_t *Vh = a.Vh + a.off[v] + (int64_t)r16 * a.dtot + 8 * g;
    const uint16_t *Vl = a.Vl + a.off[v] + (int64_t)r16 * a.dtot + 8 * g;

    f32x4 acc[TR][NT];
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u)
            acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};

    // one 32-feature chunk: raw X (BF16: 4 dwords; FP8: 2 dwords) and V hi/lo
    auto load = [&](int st, u32x4(&xa)[TR], u32x4(&vh)[NT], u32x4(&vl)[NT]) {
        const int64_t f0 = fbeg + 32 * (int64_t)(st < nst ? st : nst - 1);
        const int64_t fx = f0 + 8 * g < dv ? f0 + 8 * g : dv - 8;
#pragma unroll
        for (int t = 0; t < TR; ++t) {
            const int64_t row = (rok >> t) & 1u ? row0 + 16 * t + r16 : rlast;
            const uint8_t *p = Xb + (row * ld + fx) * ES;
            if (IN == kInBF16) {
                xa[t] = *reinterpret_cast<const u32x4 *>(p);
            } else {
                const u32x2 q = *reinterpret_cast<const u32x2 *>(p);
                xa[t] = u32x4{q[0], q[1], 0u, 0u};
            }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int64_t vo = (int64_t)16 * u * a.dtot + f0;
            vh[u] = *reinterpret_cast<const u32x4 *>(Vh + vo);
            vl[u] = *reinterpret_cast<const u32x4 *>(Vl + vo);
        }
    };
    auto mma = [&](int st, const u32x4(&xa)[TR], const u32x4(&vh)[NT], const u32x4(&vl)[NT]) {
        if (st >= nst)
            return; // wave-uniform
        const bool fok = fbeg + 32 * (int64_t)st + 8 * g < dv;
#pragma unroll
        for (int t = 0; t < TR; ++t) {
            u32x4 x = xa[t];
            if (IN == kInFP8) {
                uint32_t e0, e1, e2, e3;
                fp8x4_to_bf16(xa[t][0], e0, e1);
                fp8x4_to_bf16(xa[t][1], e2, e3);
                x = u32x4{e0, e1, e2, e3};
            }
            if (!(fok && ((rok >> t) & 1u)))
                x = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                acc[t][u] = mfma_bf16(x, vh[u], acc[t][u]);
                acc[t][u] = mfma_bf16(x, vl[u], acc[t][u]);
            }
        }
    };
    u32x4 xa0[TR], vh0[NT], vl0[NT], xa1[TR], vh1[NT], vl1[NT];
    if (nst > 0) {
        load(0, xa0, vh0, vl0);
        for (int st = 0; st < nst; st += 2) {
            load(st + 1, xa1, vh1, vl1);
            __builtin_amdgcn_sched_barrier(0);
            mma(st, xa0, vh0, vl0);
            load(st + 2, xa0, vh0, vl0);
            __builtin_amdgcn_sched_barrier(0);
            mma(st + 1, xa1, vh1, vl1);
        }
    }

    // four waves -> one RBF x KP partial.  D layout: lane l, register q holds
    // row 4 (l/16) + q, column l % 16 of each 16 x 16 tile
    float *slot = red[w & 1];
    if (w < 2) {
#pragma unroll
        for (int t = 0; t < TR; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    slot[(16 * t + 4 * g + q) * KP + 16 * u + r16] = acc[t][u][q];
    }
    __syncthreads();
    if (w >= 2) {
#pragma unroll
        for (int t = 0; t < TR; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float *p = &slot[(16 * t + 4 * g + q) * KP + 16 * u + r16];
                    *p = *p + acc[t][u][q];
                }
    }
    __syncthreads();
    float *out = a.Ppart + (((int64_t)s * a.nview + v) * a.ldr + row0) * KP;
    for (int e = tid; e < RBF * KP; e += 256)
        out[e] = red[0][e] + red[1][e];
}

// rows per workgroup of k_wfwd4
template <int KP> constexpr int fwd4_rows() { return KP <= 32 ? 256 : 128; }

// ---------------------------------------------------------------------------
// Forward products for KP = 32 and 64 with the V operand shared through LDS
// (k_wfwdv, BF16 or FP8 minibatches; FP8 codes decode exactly to BF16, the
// column scales folded into V): eight waves of 64 rows each (512 rows per
// workgroup) walk the same feature slice in 64-feature chunks, so each row's
// 128-byte line is read whole by one chunk (two 32-feature halves, issued
// together) instead of half now and half after it may have left L2.  For
// every chunk the waves fetch the 4 KP / 16 V fragments (player tile x hi/lo
// x 32-feature half) into a double-buffered LDS ring -- KP = 64: wave w
// fragment w (player tile w / 2, hi for even w, lo for odd) of both halves;
// KP = 32: fragment w % 4 of half w / 4 -- so one fragment read from L2
// serves 512 rows (k_wfwd4: 128 or 256); every wave then reads them all from
// LDS.  The minibatch loads run one chunk ahead.  Each wave owns
// its rows, so the partials go straight from the accumulators to memory (no
// cross-wave sum).  Within a half: lane layout, operands and MFMAs as k_wfwd.
// ---------------------------------------------------------------------------
constexpr int kFwdVRows = 512; // rows per k_wfwdv workgroup
template <int KP, int IN>
__global__ void __launch_bounds__(512) k_wfwdv(WideArgs a)
{
    static_assert(IN == kInBF16 || IN == kInFP8, "BF16 / FP8 codes");
    static_assert(KP == 32 || KP == 64, "two or four player tiles");
    constexpr int ES = IN == kInBF16 ? 2 : 1;
    constexpr int NT = KP / 16, TR = 4, NWV = 8;
    constexpr int NH = KP == 64 ? 2 : 1; // halves fetched per wave
    __shared__ u32x4 vb[2][2][2 * NT][64]; // [buffer][half][fragment][lane]
    const int nfwd = a.n_rb * a.nview * a.n_split;
    if ((int)blockIdx.x >= nfwd) {
        reduce_stats<NWV>(a, (int)blockIdx.x - nfwd);
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6); // wave index, scalar
    const int r16 = lane & 15, g = lane >> 4;
    int blk = blockIdx.x; // XCD-aware order, as k_wfwd
    if (nfwd % 8 == 0 && (a.nview * a.n_split) % 8 == 0)
        blk = (blk % 8) * (nfwd / 8) + blk / 8;
    const int rb = blk % a.n_rb;
    blk /= a.n_rb;
    const int v = blk % a.nview;
    const int s = blk / a.nview;
    const int64_t dv = a.dv[v];
    const int64_t ld = v ? a.ldy : a.ldx;
    const uint8_t *Xb = (const uint8_t *)(v ? a.Y : a.X);
    const int64_t row0 = (int64_t)rb * kFwdVRows + 64 * w; // this wave's 64 rows
    const int64_t fbeg = (int64_t)s * a.fs;                  // a multiple of 64
    const int64_t fend = (fbeg + a.fs < dv) ? fbeg + a.fs : dv;
    const int nst = fend > fbeg ? (int)((fend - fbeg + 63) / 64) : 0; // workgroup-uniform
    const int64_t rlast = a.b - 1;
    uint32_t rok = 0; // bit t: row valid
#pragma unroll
    for (int t = 0; t < TR; ++t)
        if (row0 + 16 * t + r16 < a.b)
            rok |= 1u << t;
    // the V fragments this wave fetches: fragment wf (player tile wf / 2, hi
    // or lo) of both halves (KP = 64) or of half w / 4 (KP = 32)
    const int wf = KP == 64 ? w : (w & 3);
    const int h0 = KP == 64 ? 0 : (w >> 2);
    const uint16_t *Vsrc = ((wf & 1) ? a.Vl : a.Vh) + a.off[v] +
                           (int64_t)(16 * (wf >> 1) + r16) * a.dtot + 8 * g + 32 * h0;

    f32x4 acc[TR][NT];
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u)
            acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};

    // chunk st: features f0 + 32 h + 8 g .. + 7 of the lane's rows (clamped
    // in-bounds: a row past the minibatch reads the last row, a feature unit
    // past the view the last unit; zeroed where consumed) and the wave's two
    // V fragments.  The V rows are padded to 64 features, so f0 + 64 stays
    // inside the view's state rows.
    auto load = [&](int st, u32x4(&xa)[2][TR], u32x4(&vg)[NH]) {
        const int64_t f0 = fbeg + 64 * (int64_t)(st < nst ? st : nst - 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t fx = f0 + 32 * h + 8 * g < dv ? f0 + 32 * h + 8 * g : dv - 8;
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                const int64_t row = (rok >> t) & 1u ? row0 + 16 * t + r16 : rlast;
                const uint8_t *p = Xb + (row * ld + fx) * ES;
                if (IN == kInBF16) {
                    xa[h][t] = *reinterpret_cast<const u32x4 *>(p);
                } else { // eight codes, decoded where consumed
                    const u32x2 q = *reinterpret_cast<const u32x2 *>(p);
                    xa[h][t] = u32x4{q[0], q[1], 0u, 0u};
                }
            }
        }
#pragma unroll
        for (int h = 0; h < NH; ++h)
            vg[h] = *reinterpret_cast<const u32x4 *>(Vsrc + f0 + 32 * h);
    };
    auto step = [&](int st, const u32x4(&xa)[2][TR], const u32x4(&vg)[NH]) {
        // every wave reaches every barrier: nst is workgroup-uniform
        u32x4(&buf)[2][2 * NT][64] = vb[st & 1];
#pragma unroll
        for (int h = 0; h < NH; ++h)
            buf[h0 + h][wf][lane] = vg[h];
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool fok = fbeg + 64 * (int64_t)st + 32 * h + 8 * g < dv;
            u32x4 x[TR];
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                u32x4 xt = xa[h][t];
                if (IN == kInFP8) {
                    uint32_t e0, e1, e2, e3;
                    fp8x4_to_bf16(xa[h][t][0], e0, e1);
                    fp8x4_to_bf16(xa[h][t][1], e2, e3);
                    xt = u32x4{e0, e1, e2, e3};
                }
                x[t] = (fok && ((rok >> t) & 1u)) ? xt : u32x4{0u, 0u, 0u, 0u};
            }
            // one player tile at a time: its hi / lo fragments from LDS
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const u32x4 vh = buf[h][2 * u][lane], vl = buf[h][2 * u + 1][lane];
#pragma unroll
                for (int t = 0; t < TR; ++t)
                    acc[t][u] = mfma_bf16(x[t], vh, acc[t][u]);
#pragma unroll
                for (int t = 0; t < TR; ++t)
                    acc[t][u] = mfma_bf16(x[t], vl, acc[t][u]);
            }
        }
    };
    // two register stages: chunk st + 1 is in flight while st is multiplied
    // (one loop exit, so the loads stay in flight across the back edge)
    u32x4 xa0[2][TR], xa1[2][TR], vg0[NH], vg1[NH];
    if (nst > 0) {
        load(0, xa0, vg0);
        int st = 0;
        for (; st + 2 <= nst; st += 2) {
            load(st + 1, xa1, vg1);
            __builtin_amdgcn_sched_barrier(0);
            step(st, xa0, vg0);
            load(st + 2, xa0, vg0);
            __builtin_amdgcn_sched_barrier(0);
            step(st + 1, xa1, vg1);
        }
        if (st < nst)
            step(st, xa0, vg0);
    }

    // this wave's 64 x KP partial.  D layout: lane l, register q holds row
    // 4 (l/16) + q, column l % 16 of each 16 x 16 tile
    float *out = a.Ppart + (((int64_t)s * a.nview + v) * a.ldr + row0) * KP;
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                out[(16 * t + 4 * g + q) * KP + 16 * u + r16] = acc[t][u][q];
}

// ---------------------------------------------------------------------------
// Middle pass, kMR rows per workgroup: sum the forward slices in a fixed order
// and write row m of W (BF16 hi/lo over the minibatch rows; FP32 input: FP32)
// = column m of [P | Q] (CCA) or of R = P - (M V)[labels] followed by the
// one-hot L (LDA, M V from the statistics totals of this iteration); block 0
// advances t.  One output element per thread; the slice loads of a thread
// are issued eight at a time and added in slice order.
// ---------------------------------------------------------------------------
template <int KP, int IN, int KIND>
__global__ void __launch_bounds__(kMT) k_wmid(WideArgs a)
{
    constexpr bool LDA = KIND == kKindLDA;
    constexpr int NV = LDA ? 1 : 2;
    constexpr int TRI = KP * (KP + 1) / 2;
    constexpr int NE = kMR * NV * KP; // output elements per workgroup
    __shared__ float tile[NE];
    __shared__ int lab[kMR];
    const int tid = threadIdx.x;
    const int q = blockIdx.x;
    const int64_t r0 = (int64_t)q * kMR;
    if (LDA && tid < kMR) {
        const int64_t row = r0 + tid;
        int l = -1;
        if (row < a.b) {
            l = a.labels[row];
            if (l < 0 || l >= a.ncls) {
                atomicOr(&a.coef->status, kStatusBadLabel);
                l = -1;
            }
        }
        lab[tid] = l;
    }
    __syncthreads();
    for (int e = tid; e < NE; e += kMT) {
        const int rl = e / (NV * KP), rem = e % (NV * KP);
        const int vv = rem / KP, c = rem % KP;
        const float *pp = a.Ppart + ((int64_t)vv * a.ldr + r0 + rl) * KP + c;
        const int64_t sstep = (int64_t)a.nview * a.ldr * KP; // between slices
        float s = 0.f;
        int sp = 0;
        for (; sp + 8 <= a.n_split; sp += 8) {
            float p[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                p[j] = pp[(sp + j) * sstep];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                s += p[j];
        }
        for (; sp < a.n_split; ++sp)
            s += pp[sp * sstep];
        if (LDA && lab[rl] >= 0)
            s = (float)((double)s - a.stot[TRI + KP + lab[rl] * KP + c]);
        if (!LDA && a.center && r0 + rl < a.b) // (X - 1 mu^T) V = X V - 1 (mu^T V)
            s = (float)((double)s - a.stot[TRI + KP + vv * KP + c]);
        tile[e] = s;
    }
    __syncthreads();
    if constexpr (IN == kInF32) {
        for (int e = tid; e < NE; e += kMT) {
            const int m = e / kMR, rl = e % kMR;
            a.Wf[(int64_t)m * a.ldr + r0 + rl] = tile[rl * NV * KP + m];
        }
        if (LDA) {
            for (int e = tid; e < kMaxCls * kMR; e += kMT) {
                const int c = e / kMR, rl = e % kMR;
                a.Wf[(int64_t)(KP + c) * a.ldr + r0 + rl] = lab[rl] == c ? 1.f : 0.f;
            }
        }
    } else {
        constexpr int MWT = Shape<KP, KIND>::MWT;
        for (int e = tid; e < NE; e += kMT) {
            const int m = e / kMR, rl = e % kMR;
            uint32_t hi, lo;
            split_bf16(tile[rl * NV * KP + m], hi, lo);
            a.Wh[w_idx<MWT>(m, r0 + rl)] = (uint16_t)hi;
            a.Wl[w_idx<MWT>(m, r0 + rl)] = (uint16_t)lo;
        }
        if (LDA) {
            for (int e = tid; e < kMaxCls * kMR; e += kMT) {
                const int c = e / kMR, rl = e % kMR;
                a.Wh[w_idx<MWT>(KP + c, r0 + rl)] = lab[rl] == c ? (uint16_t)0x3F80 : (uint16_t)0;
            }
        }
    }
    if (q == 0 && tid == 0)
        a.coef->t += 1.0;
}

// ---------------------------------------------------------------------------
// Statistics of a finished 64-feature tile (new players Vn, new auxiliary Gn,
// LDS, feature-major with row stride VLD; LDA: class means Mt, 16 x 64): FP64
// MFMA (16x16x4) over the tile's features, accumulated in sacc over the
// subtiles of a workgroup (kBW waves).  Wave w owns statistics tiles w,
// w + kBW, w + 2 kBW, ...
// ---------------------------------------------------------------------------
template <int KP, int KIND> struct StatTiles {
    static constexpr int H = (Shape<KP, KIND>::NST + kBW - 1) / kBW; // tiles per wave
};

template <int KP, int KIND>
__device__ __forceinline__ void tile_stats(const float *Vn, const float *Gn, const float *Mt,
                                           f64x4 (&sacc)[StatTiles<KP, KIND>::H], bool mv_on)
{
    typedef Shape<KP, KIND> S;
    constexpr int VLD = S::VLD;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l16 = lane & 15, g = lane >> 4;
#pragma unroll
    for (int h = 0; h < StatTiles<KP, KIND>::H; ++h) {
        const int st = w + kBW * h;
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
            if (!mv_on)
                continue; // wave-uniform: CCA without centring (its mean terms stay 0)
        }
        f64x4 acc = sacc[h];
#pragma unroll 4
        for (int k4 = 0; k4 < kFT; k4 += 4) {
            const int fl = k4 + g;
            // mean tiles: LDA rows are the 16 class means; CCA has row 0 only
            const double av = mv ? ((S::LDA || l16 == 0) ? (double)Mt[(S::LDA ? l16 : 0) * kFT + fl] : 0.0)
                                 : (double)Vn[fl * VLD + 16 * u + l16];
            const double bv = mv ? (double)Vn[fl * VLD + 16 * u2 + l16] : (double)Gn[fl * VLD + 16 * u2 + l16];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        sacc[h] = acc;
    }
}

template <int KP, int KIND>
__device__ __forceinline__ void write_stats(const WideArgs &a, int wg,
                                            const f64x4 (&sacc)[StatTiles<KP, KIND>::H], double nrm,
                                            int v)
{
    typedef Shape<KP, KIND> S;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6); // wave index, scalar
    const int l16 = lane & 15, g = lane >> 4;
#pragma unroll
    for (int h = 0; h < StatTiles<KP, KIND>::H; ++h) {
        const int st = w + kBW * h;
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
                    a.spart[sp_idx(a, tri_idx(i, j), wg)] = sacc[h][r];
            }
        } else {
            const int u2 = st - S::NT * (S::NT + 1) / 2;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = g + 4 * r, j = 16 * u2 + l16;
                if (S::LDA) {
                    if (c < a.ncls)
                        a.spart[sp_idx(a, S::TRI + KP + c * KP + j, wg)] = sacc[h][r];
                } else if (c == 0) { // CCA: mu_v^T v_j of this view, 0 for the other view
                    a.spart[sp_idx(a, S::TRI + KP + v * KP + j, wg)] = sacc[h][r];
                    a.spart[sp_idx(a, S::TRI + KP + (1 - v) * KP + j, wg)] = 0.0;
                }
            }
        }
    }
    if (tid < KP)
        a.spart[sp_idx(a, S::TRI + tid, wg)] = nrm;
}

// Player-major BF16 hi/lo operand of s_f Vn for the 64 features of a tile
// (two features per thread per pass, one 128-byte run per player); FP32
// input: the FP32 copy of Vn.
template <int KP, int KIND, int IN>
__device__ __forceinline__ void write_vop(const WideArgs &a, const float *Vn, int64_t frow)
{
    constexpr int VLD = Shape<KP, KIND>::VLD;
    if constexpr (IN == kInF32) { // player-major FP32 copy, one 256-byte run per player
        for (int e = threadIdx.x; e < KP * kFT; e += kBT) {
            const int i = e / kFT, fl = e % kFT;
            a.Vf[(int64_t)i * a.dtot + frow + fl] = Vn[fl * VLD + i];
        }
        return;
    }
    for (int e = threadIdx.x; e < KP * (kFT / 2); e += kBT) {
        const int i = e / (kFT / 2), fl = 2 * (e % (kFT / 2));
        float x0 = Vn[fl * VLD + i], x1 = Vn[(fl + 1) * VLD + i];
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

// |Vn_i|^2 over the tile (threads i < KP), FP64
template <int KP, int KIND>
__device__ __forceinline__ void tile_norms(const float *Vn, double &nrm)
{
    constexpr int VLD = Shape<KP, KIND>::VLD;
    if ((int)threadIdx.x < KP)
        for (int fl = 0; fl < kFT; ++fl)
            nrm += (double)Vn[fl * VLD + threadIdx.x] * (double)Vn[fl * VLD + threadIdx.x];
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

// One 32-row chunk of the backward stream held in registers: X (8 rows x NCF
// features per lane, raw: XD dwords per row), the W tiles (hi, lo), and the
// one-hot tile (LDA).
template <int NU, int XD> struct BwdChunk {
    uint32_t x[8][XD];
    u32x4 wh[NU], wl[NU];
    u32x4 lh;
};

// The same chunk for FP32 input: X (8 rows x 4 features per lane), the W
// tiles and the one-hot tile, eight rows per lane each.
template <int NU> struct BwdChunk32 {
    f32x4 x[8];
    f32x4 w[NU][2];
    f32x4 l[2];
};

// ---------------------------------------------------------------------------
// Backward products, coefficients and fused epilogue.
// A workgroup takes subtiles of FT features (64, or 128 where the view is
// wide enough to keep >= 256 workgroups: fewer W loads per X byte).
// Main loop over 32-row chunks (wave w takes chunks w, w + 4, ...): lane l
// (n = l % 16, g = l / 16) loads rows 8 g .. 8 g + 7 of the chunk at features
// NCF n .. NCF n + NCF - 1 of the subtile (NCF = FT / 16; one 16-byte load per
// row for BF16 at FT = 128) and transposes them in registers, so MFMA c
// (c < NCF) gets the B operand B[8 g + j][n] = X[row 8 g + j][feature NCF n + c];
// the A operand is a 16-row tile of W, lane l holding W[l % 16][rows 8 g ..
// 8 g + 7] in one 16-byte load.  D[m][n] is then (X^T W^T)[NCF n + c][m].
// With PART (k_wprod, 128-feature subtiles, one per workgroup) the summed
// products go to memory instead of an epilogue, and workgroup 0 alone forms
// the Gram terms and the coefficients, publishing them as the coefficient
// tile; k_wepi then runs the epilogue per 64-feature tile.
// ---------------------------------------------------------------------------
template <int KP, int IN, int KIND, int OPT, int FT = kFT, bool PART = false>
__device__ __forceinline__ void wbwd_body(WideArgs a)
{
    static_assert(FT == kFT || (FT == 2 * kFT && IN != kInF32 && PART), "backward subtile");
    constexpr int NCF = FT / 16;  // features per lane
    constexpr int NH = FT / kFT;  // 64-feature halves of a subtile
    constexpr int XD = NCF * (IN == kInBF16 ? 2 : 1) / 4; // dwords of X per lane and row
    typedef Shape<KP, KIND> S;
    constexpr int NT = S::NT, NU = S::NU, MWP = S::MWP, SLOT = S::SLOT, TRI = S::TRI;
    constexpr int GLD = S::GLD, VLD = S::VLD, NG = S::NG;
    constexpr bool LDA = S::LDA;
    constexpr int NC = LDA ? kMaxCls : 1;
    __shared__ __attribute__((aligned(16))) float red[4 * SLOT];
    __shared__ float Tt[KP * KP];   // Tt[j * KP + i] = T_ij (j < i), else 0
    __shared__ double Td[KP * KP];  // the same T_ij in FP64, row i: Td[i * KP + j]
    __shared__ double gd[S::GT];
    __shared__ double sprior[NC];   // LDA class priors
    __shared__ float cInv[KP], cMB[KP], cMAc[KP], cUc[KP];
    __shared__ double dInv[KP], dS[KP];
    __shared__ float cSp[NC * KP], cU[NC * KP];
    __shared__ double dMc[NC * KP];
    __shared__ float Mt[NC * kFT], Mb[LDA ? kFT : 1];
    // centring (CCA): the tile's running means, the W column sums, the
    // minibatch column sums of the subtile (per wave and lane group, then total)
    __shared__ float muT[LDA ? 1 : kFT], cP[LDA ? 1 : KP], cQ[LDA ? 1 : KP];
    __shared__ float xsp[LDA ? 1 : kBW * 4 * FT], xcs[LDA ? 1 : FT];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6); // wave index, scalar
    const int l16 = lane & 15, g = lane >> 4;
    const int wg = xcd_tile(blockIdx.x, gridDim.x);
    const bool CEN = !LDA && a.center != 0; // workgroup-uniform
    int v, sub0, sub1;
    wg_range(a, wg, v, sub0, sub1);
    const int64_t dv = a.dv[v];
    const int64_t ld = v ? a.ldy : a.ldx;
    const uint8_t *Xb = (const uint8_t *)(v ? a.Y : a.X);
    constexpr int ES = IN == kInBF16 ? 2 : (IN == kInF32 ? 4 : 1);
    const int nch = (int)((a.b + 31) / 32);
    const double t = a.coef->t; // this iteration's number, set by k_wmid
    const double ib = 1.0 / (double)a.b;
    // terms that depend only on t, once per workgroup
    const float eta = (float)eta_sched(a, t), gam = (float)a.gamma, ibf = (float)ib;
    const float eps = (float)a.eps_reg;
    const float b1 = (float)a.adam_b1, b2 = (float)a.adam_b2, aeps = (float)a.adam_eps;
    const float c1 = (float)(1.0 - pow(a.adam_b1, t)), c2 = (float)(1.0 - pow(a.adam_b2, t));
    if (LDA && tid < NC)
        sprior[tid] = tid < a.ncls ? a.prior[tid] : 0.0; // read after the loop's barriers
    // BF16 W in 1 KB tiles (w_idx): this lane's 16 bytes of a tile
    const uint16_t *Wh = IN == kInF32 ? nullptr : a.Wh + l16 * 32 + 8 * g;
    const uint16_t *Wl = IN == kInF32 ? nullptr : a.Wl + l16 * 32 + 8 * g;
    const float *Wf = IN == kInF32 ? a.Wf + (int64_t)l16 * a.ldr + 8 * g : nullptr;

    f64x4 sacc[StatTiles<KP, KIND>::H];
#pragma unroll
    for (int h = 0; h < StatTiles<KP, KIND>::H; ++h)
        sacc[h] = f64x4{0, 0, 0, 0};
    double nrm = 0.0;

    for (int sub = sub0; sub < sub1; ++sub) {
        const bool first = PART ? wg == 0 : sub == sub0; // forms the Gram terms
        const int64_t fv0 = (int64_t)sub * FT;
        f32x4 acc[NCF][NU];
#pragma unroll
        for (int c = 0; c < NCF; ++c)
#pragma unroll
            for (int u = 0; u < NU; ++u)
                acc[c][u] = f32x4{0.f, 0.f, 0.f, 0.f};
        f32x4 gacc[NG];
#pragma unroll
        for (int u = 0; u < NG; ++u)
            gacc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        float dP[NT], dQ[NT], sP[NT], sQ[NT]; // sums of squares; column sums (centring)
#pragma unroll
        for (int u = 0; u < NT; ++u)
            dP[u] = dQ[u] = sP[u] = sQ[u] = 0.f;
        float xs[NCF]; // centring: this lane's column sums of the minibatch (raw codes)
#pragma unroll
        for (int c = 0; c < NCF; ++c)
            xs[c] = 0.f;

        // Loads are unconditional, from clamped in-bounds addresses (a chunk past
        // the minibatch reads the last chunk, a row past it the last row, a
        // feature unit past the view the last unit); invalid X is zeroed where
        // it is consumed and an invalid chunk is skipped (wave-uniform), so the
        // ring of chunks stays in flight.
        const int64_t fu = fv0 + NCF * l16;
        const bool fok = fu < dv;
        const uint8_t *xc = Xb + (fok ? fu : dv - NCF) * ES;

        if constexpr (IN == kInF32) {
            auto loadc = [&](int ch, BwdChunk32<NU> &B) {
                const int64_t r0 = (int64_t)(ch < nch ? ch : nch - 1) * 32;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int64_t row = r0 + 8 * g + j < a.b ? r0 + 8 * g + j : a.b - 1;
                    B.x[j] = *reinterpret_cast<const f32x4 *>(xc + row * ld * 4);
                }
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const float *q = Wf + (int64_t)16 * u * a.ldr + r0;
                    B.w[u][0] = *reinterpret_cast<const f32x4 *>(q);
                    B.w[u][1] = *reinterpret_cast<const f32x4 *>(q + 4);
                }
                if (LDA && first) { // the one-hot rows only feed the Gram terms
                    const float *q = Wf + (int64_t)KP * a.ldr + r0;
                    B.l[0] = *reinterpret_cast<const f32x4 *>(q);
                    B.l[1] = *reinterpret_cast<const f32x4 *>(q + 4);
                }
            };
            auto compute = [&](int ch, const BwdChunk32<NU> &B) {
                if (ch >= nch)
                    return; // wave-uniform
                const int64_t r0 = (int64_t)ch * 32;
                // B operand of feature column c: xb[c][h][j] = X[row 8 g + 4 h + j][4 n + c]
                f32x4 xb[4][2];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bool ok = fok && r0 + 8 * g + j < a.b;
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        xb[c][j >> 2][j & 3] = ok ? B.x[j][c] : 0.f;
                }
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int u = 0; u < NU; ++u)
                        acc[c][u] = mfma_f32x8(B.w[u], xb[c], acc[c][u]);
                if (first) {
                    // Gram terms from the W fragments (lane (m, g): rows 8g..8g+7 of
                    // W row m, the A and the B layout of the eight MFMAs)
                    if (!LDA) {
#pragma unroll
                        for (int up = 0; up < NT; ++up)
#pragma unroll
                            for (int uq = 0; uq < NT; ++uq)
                                gacc[up * NT + uq] =
                                    mfma_f32x8(B.w[up], B.w[NT + uq], gacc[up * NT + uq]);
                    } else {
#pragma unroll
                        for (int u = 0; u < NT; ++u)
                            gacc[u] = mfma_f32x8(B.l, B.w[u], gacc[u]);
                    }
#pragma unroll
                    for (int u = 0; u < NT; ++u)
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const float p = B.w[u][h][j];
                                dP[u] += p * p;
                                if (!LDA) {
                                    const float q = B.w[NT + u][h][j];
                                    dQ[u] += q * q;
                                }
                            }
                }
            };
            // two chunks in flight (the FP32 products are MFMA-bound)
            constexpr int NB = 2;
            BwdChunk32<NU> cb[NB];
            loadc(w, cb[0]);
            for (int ch = w; ch < nch; ch += NB * kBW) {
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    loadc(ch + kBW * (q + 1), cb[(q + 1) % NB]);
                    __builtin_amdgcn_sched_barrier(0);
                    compute(ch + kBW * q, cb[q]);
                }
            }
        } else {
            auto loadc = [&](int ch, BwdChunk<NU, XD> &B) {
                const int64_t cc = ch < nch ? ch : nch - 1;
                const int64_t r0 = cc * 32;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int64_t row = r0 + 8 * g + j < a.b ? r0 + 8 * g + j : a.b - 1;
                    const uint8_t *px = xc + row * ld * ES;
                    if constexpr (XD == 4) {
                        const u32x4 q = *reinterpret_cast<const u32x4 *>(px);
                        B.x[j][0] = q[0]; B.x[j][1] = q[1]; B.x[j][2] = q[2]; B.x[j][3] = q[3];
                    } else if constexpr (XD == 2) {
                        const u32x2 q = *reinterpret_cast<const u32x2 *>(px);
                        B.x[j][0] = q[0]; B.x[j][1] = q[1];
                    } else {
                        B.x[j][0] = *reinterpret_cast<const uint32_t *>(px);
                    }
                }
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const int64_t wo = (cc * S::MWT + u) * 512;
                    B.wh[u] = *reinterpret_cast<const u32x4 *>(Wh + wo);
                    B.wl[u] = *reinterpret_cast<const u32x4 *>(Wl + wo);
                }
                if (LDA && first) // the one-hot rows only feed the Gram terms
                    B.lh = *reinterpret_cast<const u32x4 *>(Wh + (cc * S::MWT + KP / 16) * 512);
            };
            auto compute = [&](int ch, const BwdChunk<NU, XD> &B) {
                if (ch >= nch)
                    return; // wave-uniform
                const int64_t r0 = (int64_t)ch * 32;
                // feature pairs p: column c = 2 p, 2 p + 1 of the transposed chunk;
                // row j's BF16 pair is dword p of the row (FP8 codes decode exactly)
                bool rvalid[8];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    rvalid[j] = fok && r0 + 8 * g + j < a.b;
#pragma unroll
                for (int p = 0; p < NCF / 2; ++p) {
                    uint32_t col[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        uint32_t x;
                        if (IN == kInBF16) {
                            x = B.x[j][p];
                        } else {
                            uint32_t e0, e1;
                            fp8x4_to_bf16(B.x[j][p >> 1], e0, e1);
                            x = (p & 1) ? e1 : e0;
                        }
                        col[j] = rvalid[j] ? x : 0u;
                    }
                    if (CEN) {
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            xs[2 * p] += bf16_val(col[j] & 0xFFFFu);
                            xs[2 * p + 1] += bf16_val(col[j] >> 16);
                        }
                    }
                    // B operands: the BF16 of rows 2q, 2q + 1 in dword q
                    u32x4 b0, b1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t a0 = col[2 * q], a1 = col[2 * q + 1];
                        b0[q] = (a0 & 0xFFFFu) | (a1 << 16);
                        b1[q] = (a0 >> 16) | (a1 & 0xFFFF0000u);
                    }
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        acc[2 * p][u] = mfma_bf16(B.wh[u], b0, acc[2 * p][u]);
                        acc[2 * p][u] = mfma_bf16(B.wl[u], b0, acc[2 * p][u]);
                        acc[2 * p + 1][u] = mfma_bf16(B.wh[u], b1, acc[2 * p + 1][u]);
                        acc[2 * p + 1][u] = mfma_bf16(B.wl[u], b1, acc[2 * p + 1][u]);
                    }
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
                                ga = mfma_bf16(B.wh[up], B.wh[NT + uq], ga);
                                ga = mfma_bf16(B.wh[up], B.wl[NT + uq], ga);
                                ga = mfma_bf16(B.wl[up], B.wh[NT + uq], ga);
                            }
                    } else {
#pragma unroll
                        for (int u = 0; u < NT; ++u) {
                            gacc[u] = mfma_bf16(B.lh, B.wh[u], gacc[u]);
                            gacc[u] = mfma_bf16(B.lh, B.wl[u], gacc[u]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < NT; ++u)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const float p0 = bf16_val(B.wh[u][q] & 0xFFFFu) + bf16_val(B.wl[u][q] & 0xFFFFu);
                            const float p1 = bf16_val(B.wh[u][q] >> 16) + bf16_val(B.wl[u][q] >> 16);
                            dP[u] += p0 * p0 + p1 * p1;
                            if (!LDA) {
                                const float q0 = bf16_val(B.wh[NT + u][q] & 0xFFFFu) +
                                                 bf16_val(B.wl[NT + u][q] & 0xFFFFu);
                                const float q1 = bf16_val(B.wh[NT + u][q] >> 16) + bf16_val(B.wl[NT + u][q] >> 16);
                                dQ[u] += q0 * q0 + q1 * q1;
                                if (CEN) {
                                    sP[u] += p0 + p1;
                                    sQ[u] += q0 + q1;
                                }
                            }
                        }
                }
            };
            // ring of NB chunks in flight: the loads of chunk i + NB - 1 are issued
            // before the MFMAs of chunk i (wave w takes chunks w, w + kBW, ...)
            constexpr int NB = FT == kFT ? 3 : 2; // 128-feature chunks hold twice the X
            BwdChunk<NU, XD> cb[NB];
#pragma unroll
            for (int p = 0; p < NB - 1; ++p)
                loadc(w + kBW * p, cb[p]);
            for (int ch = w; ch < nch; ch += NB * kBW) {
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    loadc(ch + kBW * (q + NB - 1), cb[(q + NB - 1) % NB]);
                    __builtin_amdgcn_sched_barrier(0);
                    compute(ch + kBW * q, cb[q]);
                }
            }
        }

        if (CEN) { // the subtile's minibatch column sums: waves in order, then lane groups
#pragma unroll
            for (int c = 0; c < NCF; ++c)
                xsp[(w * 4 + g) * FT + NCF * l16 + c] = xs[c];
            __syncthreads();
            for (int f = tid; f < FT; f += kBT) {
                float t = 0.f;
                for (int q = 0; q < kBW * 4; ++q)
                    t += xsp[q * FT + f];
                xcs[f] = t;
                if (PART)
                    a.xsum[a.off[v] + fv0 + f] = t;
            }
            __syncthreads();
        }
        for (int hh = 0; hh < NH; ++hh) { // 64-feature halves
            // the old auxiliary tile of this subtile, into registers now (written
            // to LDS once the products and Gram terms no longer need the space)
            const int64_t fvh = fv0 + (int64_t)kFT * hh; // the half's first feature
            const int64_t frow = a.off[v] + fvh;          // and its state row
            constexpr int GPT = kFT * KP / kBT;
            float gpre[GPT];
            if constexpr (!PART) {
#pragma unroll
                for (int q = 0; q < GPT; ++q)
                    gpre[q] = a.G[frow * KP + tid + q * kBT];
            }
            if constexpr (PART) {
                // ---- products of the whole subtile: waves 0, 1 write slots A, B
                // (FT features each), waves 2, 3 add theirs, A + B to memory ----
                float *slot = red + (w & 1) * 2 * SLOT;
                if (w < 2) {
#pragma unroll
                    for (int c = 0; c < NCF; ++c)
#pragma unroll
                        for (int u = 0; u < NU; ++u)
                            *reinterpret_cast<f32x4 *>(&slot[(NCF * l16 + c) * MWP + 16 * u + 4 * g]) =
                                acc[c][u];
                }
                __syncthreads();
                if (w >= 2) {
#pragma unroll
                    for (int c = 0; c < NCF; ++c)
#pragma unroll
                        for (int u = 0; u < NU; ++u) {
                            f32x4 *q = reinterpret_cast<f32x4 *>(
                                &slot[(NCF * l16 + c) * MWP + 16 * u + 4 * g]);
                            *q = *q + acc[c][u];
                        }
                }
                __syncthreads();
                float *out = a.prod + (a.off[v] + fv0) * S::MWA;
                for (int e = tid; e < FT * S::MWA; e += kBT) {
                    const int idx = (e / S::MWA) * MWP + e % S::MWA;
                    out[e] = red[idx] + red[2 * SLOT + idx];
                }
                if (!first)
                    return;
                __syncthreads();
            } else {
                // ---- products: four waves -> prod = slot 0, element (feature, m); the
                // lanes holding this half's features write ----
                if ((NCF * l16) / kFT == hh) {
                    const int fl0 = NCF * l16 - kFT * hh;
#pragma unroll
                    for (int c = 0; c < NCF; ++c)
#pragma unroll
                        for (int u = 0; u < NU; ++u)
                            *reinterpret_cast<f32x4 *>(
                                &red[w * SLOT + (fl0 + c) * MWP + 16 * u + 4 * g]) = acc[c][u];
                }
                __syncthreads();
                for (int e = tid; e < kFT * S::MWA; e += kBT) {
                    const int idx = (e / S::MWA) * MWP + e % S::MWA;
                    red[idx] =
                        ((red[idx] + red[SLOT + idx]) + red[2 * SLOT + idx]) + red[3 * SLOT + idx];
                }
                __syncthreads();
            }
            float *ext = red + SLOT; // three free slots from here on

            if (first && hh == 0) {
                // ---- Gram terms: four waves x lane groups, fixed-order sum ----
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
                        gw[KP * KP + 8 * KP + g * KP + 16 * u + l16] = sP[u];
                        gw[KP * KP + 12 * KP + g * KP + 16 * u + l16] = sQ[u];
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
                }
                __syncthreads();
                for (int e = tid; e < S::GT; e += kBT) {
                    double s = 0.0;
                    const int base = LDA ? 16 * KP : KP * KP;
                    if (e < base) {
                        for (int ww = 0; ww < kBW; ++ww)
                            s += (double)ext[ww * S::GW + e];
                    } else {
                        const int which = (e - base) / KP, col = (e - base) % KP;
                        for (int ww = 0; ww < kBW; ++ww)
                            for (int gg = 0; gg < 4; ++gg)
                                s += (double)ext[ww * S::GW + base + which * 4 * KP + gg * KP + col];
                    }
                    gd[e] = s;
                }
                __syncthreads();
                if (!LDA && tid < KP) { // centring: column sums of P and Q over the rows
                    cP[tid] = (float)gd[KP * KP + 2 * KP + tid];
                    cQ[tid] = (float)gd[KP * KP + 3 * KP + tid];
                }

                // ---- k x k coefficients (identical in every workgroup) ----
                double *ss = reinterpret_cast<double *>(ext);
                // four loads of a thread in flight before its stores
                for (int e0 = 0; e0 < a.Ws; e0 += 4 * kBT) {
                    double r[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int e = e0 + tid + q * kBT;
                        r[q] = e < a.Ws ? a.stot[e] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int e = e0 + tid + q * kBT;
                        if (e < a.Ws)
                            ss[e] = r[q];
                    }
                }
                __syncthreads();
                if (tid < KP) {
                    const int i = tid;
                    double inv = 0.0, s = 1.0;
                    if (i < a.k) {
                        inv = 1.0 / sqrt(ss[TRI + i]);
                        if (a.smooth) { // Alg. 3: exp(log rho + (log nu - log rho) sigmoid(z_i))
                            const double z = a.coef->z[(int64_t)t & 1][i];
                            s = exp(a.lrho + a.lspan / (1.0 + exp(-z)));
                        } else {        // Alg. 2: max(v_i^T G_i, rho)
                            s = ss[tri_idx(i, i)] * inv;
                            if (!(s >= a.rho))
                                s = a.rho;
                        }
                    }
                    dInv[i] = inv;
                    dS[i] = s;
                }
                __syncthreads();
                if (LDA) {
                    // class sums S = L^T R (raw) and the centred normalised class-mean
                    // projections Mc_ci = (mu_c - mubar)^T v_i (FP64), cU = pi_c Mc_ci
                    for (int e = tid; e < kMaxCls * KP; e += kBT) {
                        const int c = e / KP, i = e % KP;
                        cSp[e] = (c < a.ncls && i < a.k) ? (float)gd[e] : 0.f;
                    }
                    if (tid < KP) {
                        const int i = tid;
                        double mbar = 0.0, usum = 0.0;
                        if (i < a.k)
                            for (int c = 0; c < a.ncls; ++c)
                                mbar += sprior[c] * ss[TRI + KP + c * KP + i] * dInv[i];
                        for (int c = 0; c < kMaxCls; ++c) {
                            double mc = 0.0;
                            if (c < a.ncls && i < a.k)
                                mc = ss[TRI + KP + c * KP + i] * dInv[i] - mbar;
                            dMc[c * KP + i] = mc;
                            const float u = (float)((c < a.ncls ? sprior[c] : 0.0) * mc);
                            cU[c * KP + i] = u;
                            usum += (double)u;
                        }
                        cUc[i] = (float)usum;
                    }
                }
                __syncthreads();
                // (M_A)_ij: CCA b^-1 inv_i inv_j (P^T Q + Q^T P)_ij; LDA sum_c pi_c Mc_ci Mc_cj
                auto MA = [&](int i, int j) -> double {
                    if (!LDA)
                        return (gd[i * KP + j] + gd[j * KP + i]) * dInv[i] * dInv[j] * ib;
                    double s = 0.0;
                    for (int c = 0; c < a.ncls; ++c)
                        s += sprior[c] * dMc[c * KP + i] * dMc[c * KP + j];
                    return s;
                };
                for (int e = tid; e < KP * KP; e += kBT) {
                    const int j = e / KP, i = e % KP;
                    double val = 0.0;
                    if (i < a.k && j < i)
                        val = MA(i, j) / dS[j];
                    Tt[e] = (float)val;
                    Td[i * KP + j] = val;
                }
                __syncthreads();
                Coef *cw = a.coef;
                if (tid < KP) {
                    const int i = tid;
                    double mA = 0.0, mB = 0.0, c = 0.0;
                    if (i < a.k) {
                        const double ii2 = dInv[i] * dInv[i];
                        mA = MA(i, i);
                        if (!LDA)
                            mB = (gd[KP * KP + i] + gd[KP * KP + KP + i]) * ii2 * ib;
                        else
                            mB = gd[16 * KP + i] * ii2 * ib + a.eps_reg;
                        for (int j = 0; j < i; ++j)
                            c += Td[i * KP + j] * (ss[tri_idx(i, j)] * dInv[i]); // T_ij C_ij
                    }
                    cMB[i] = (float)mB;
                    cMAc[i] = (float)(mA - c);
                    cInv[i] = (float)dInv[i];
                    if (wg == 0) {
                        if (i < a.k) {
                            cw->ema_a[i] += a.gamma * (mA - cw->ema_a[i]);
                            cw->ema_b[i] += a.gamma * (mB - cw->ema_b[i]);
                            const double craw = ss[tri_idx(i, i)] * dInv[i];
                            if (a.smooth) {
                                // Alg. 3 z step at rate gamma, into the other buffer
                                const double z = cw->z[(int64_t)t & 1][i];
                                const double sg = 1.0 / (1.0 + exp(-z));
                                const double zn = z + a.gamma * (craw - dS[i]) * dS[i] * a.lspan *
                                                          sg * (1.0 - sg);
                                cw->z[((int64_t)t + 1) & 1][i] = zn;
                                if (!isfinite(zn))
                                    atomicOr(&cw->status, kStatusNonFinite);
                            } else if (!(craw >= a.rho)) {
                                atomicAdd(&cw->clip_count, 1);
                            }
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
            if constexpr (PART) { // the coefficient tile for k_wepi; no epilogue here
                float *ct = a.ctile;
                for (int e = tid; e < KP * KP; e += kBT)
                    ct[e] = Tt[e];
                if (tid < KP) {
                    ct[KP * KP + tid] = cInv[tid];
                    ct[KP * KP + KP + tid] = cMB[tid];
                    ct[KP * KP + 2 * KP + tid] = cMAc[tid];
                    ct[KP * KP + 3 * KP + tid] = cUc[tid];
                }
                if (LDA)
                    for (int e = tid; e < NC * KP; e += kBT) {
                        ct[KP * KP + 4 * KP + e] = cSp[e];
                        ct[KP * KP + 4 * KP + NC * KP + e] = cU[e];
                    }
                else if (tid < KP) { // the column sums for the centring
                    ct[KP * KP + 4 * KP + tid] = cP[tid];
                    ct[KP * KP + 5 * KP + tid] = cQ[tid];
                }
                return;
            }

            // ---- fused epilogue on 16 x 16 tiles (feature block fb, player block pb) ----
            float *Gold = ext, *Vn = ext + kFT * GLD, *Gn = Vn + kFT * VLD;
#pragma unroll
            for (int q = 0; q < GPT; ++q) {
                const int e = tid + q * kBT;
                Gold[(e / KP) * GLD + e % KP] = gpre[q];
            }
            if (LDA) {
                for (int e = tid; e < kMaxCls * kFT; e += kBT) {
                    const int c = e / kFT, fl = e % kFT;
                    Mt[e] = c < a.ncls ? a.M[(int64_t)c * a.dtot + frow + fl] : 0.f;
                }
                for (int e = tid; e < kFT; e += kBT)
                    Mb[e] = a.Mbar[frow + e];
            }
            if (CEN && tid < kFT)
                muT[tid] = a.mu[frow + tid];
            __syncthreads();
            for (int tt = w; tt < 4 * NT; tt += kBW) {
                const int fb = tt / NT, pb = tt % NT;
                // parent penalty sum_j G_old[fl][j] T_ij, and (LDA) the class terms
                // sum_c M[c][fl] S_ci and sum_c M[c][fl] U_ci: FP32 MFMA 16x16x4
                f32x4 pen = {0.f, 0.f, 0.f, 0.f}, e2 = pen, e3 = pen;
#pragma unroll 4
                for (int j0 = 0; j0 < KP; j0 += 4)
                    pen = __builtin_amdgcn_mfma_f32_16x16x4f32(Gold[(16 * fb + l16) * GLD + j0 + g],
                                                              Tt[(j0 + g) * KP + 16 * pb + l16], pen, 0, 0, 0);
                if (LDA) {
#pragma unroll
                    for (int c0 = 0; c0 < kMaxCls; c0 += 4) {
                        const float mA_ = Mt[(c0 + g) * kFT + 16 * fb + l16];
                        e2 = __builtin_amdgcn_mfma_f32_16x16x4f32(mA_, cSp[(c0 + g) * KP + 16 * pb + l16], e2, 0, 0, 0);
                        e3 = __builtin_amdgcn_mfma_f32_16x16x4f32(mA_, cU[(c0 + g) * KP + 16 * pb + l16], e3, 0, 0, 0);
                    }
                }
                const int i = 16 * pb + l16;
                // the state of this tile's four rows, loaded together
                float vold[4], mold[4], sold[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t si = (frow + 16 * fb + 4 * g + r) * KP + i;
                    vold[r] = a.V[si];
                    if (OPT != kOptSGD) {
                        mold[r] = a.Am[si];
                        sold[r] = a.As[si];
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int fl = 16 * fb + 4 * g + r; // FP32 D row 4 (l/16) + r
                    const int64_t si = (frow + fl) * KP + i;
                    float vn = 0.f, gn = 0.f;
                    if (fvh + fl < dv && i < a.k) {
                        const float inv = cInv[i];
                        const float vh = vold[r] * inv;
                        const float *pr = red + fl * MWP;
                        float av, bv;
                        if (!LDA) {
                            const float sf = IN == kInFP8 ? a.colscale[frow + fl] : 1.f;
                            const float rawA = v == 0 ? pr[KP + i] : pr[i];
                            const float rawB = v == 0 ? pr[i] : pr[KP + i];
                            float rA = rawA * sf, rB = rawB * sf;
                            if (CEN) { // (X - 1 mu^T)^T W = X^T W - mu (1^T W)
                                rA -= muT[fl] * (v == 0 ? cQ[i] : cP[i]);
                                rB -= muT[fl] * (v == 0 ? cP[i] : cQ[i]);
                            }
                            av = rA * inv * ibf;
                            bv = rB * inv * ibf;
                        } else {
                            bv = (pr[i] - e2[r]) * inv * ibf + eps * vh;
                            av = e3[r] - Mb[fl] * cUc[i];
                        }
                        const float grad = (av - pen[r]) * cMB[i] - bv * cMAc[i];
                        if (OPT == kOptSGD) {
                            vn = vh + eta * grad;
                        } else {
                            const float mm = b1 * mold[r] + (1.f - b1) * grad;
                            const float sq = b2 * sold[r] + (1.f - b2) * grad * grad;
                            a.Am[si] = mm;
                            a.As[si] = sq;
                            vn = vh + eta * (mm / c1) / (sqrtf(sq / c2) + aeps);
                        }
                        const float g0 = Gold[fl * GLD + i];
                        gn = g0 + gam * (bv - g0);
                        a.V[si] = vn;
                        a.G[si] = gn;
                    }
                    Vn[fl * VLD + i] = vn;
                    Gn[fl * VLD + i] = gn;
                }
            }
            if (CEN && tid < kFT) { // mu += gamma (column mean - mu); Mt row 0 for the statistics
                float mn = 0.f;
                if (fvh + tid < dv) {
                    const float sf = IN == kInFP8 ? a.colscale[frow + tid] : 1.f;
                    mn = muT[tid] + gam * (xcs[kFT * hh + tid] * sf * ibf - muT[tid]);
                }
                a.mu[frow + tid] = mn;
                Mt[tid] = mn;
            }
            __syncthreads();
            write_vop<KP, KIND, IN>(a, Vn, frow);
            tile_stats<KP, KIND>(Vn, Gn, Mt, sacc, LDA || CEN);
            tile_norms<KP, KIND>(Vn, nrm);
            __syncthreads();
        }
    }
    write_stats<KP, KIND>(a, wg, sacc, nrm, v);
}

template <int KP, int IN, int KIND, int OPT>
__global__ void __launch_bounds__(kBT) k_wbwd(WideArgs a)
{
    wbwd_body<KP, IN, KIND, OPT>(a);
}

template <int KP, int IN, int KIND>
__global__ void __launch_bounds__(kBT) k_wprod(WideArgs a)
{
    wbwd_body<KP, IN, KIND, kOptSGD, 2 * kFT, true>(a);
}

// Size in floats of the coefficient tile: T (KP x KP), 1/||v||, m_B,
// m_A - c, sum_c pi_c U (KP each), and (LDA) the class sums S and U.
template <int KP, int KIND> constexpr int ctile_floats()
{
    return KP * KP + 4 * KP + (KIND == kKindLDA ? 2 * kMaxCls * KP : 2 * KP);
}

// ---------------------------------------------------------------------------
// Epilogue of the split backward: one workgroup per 64-feature tile of the
// state (both views), from the products k_wprod left in memory and its
// coefficient tile: update direction, retraction step (SGD or Adam),
// auxiliary update, the V operand of the next iteration and this tile's
// statistics partials (column = workgroup).  The same arithmetic as the
// epilogue of k_wbwd.
// ---------------------------------------------------------------------------
template <int KP, int IN, int KIND, int OPT>
__global__ void __launch_bounds__(kBT) k_wepi(WideArgs a)
{
    typedef Shape<KP, KIND> S;
    constexpr int NT = S::NT, GLD = S::GLD, VLD = S::VLD, MWA = S::MWA;
    constexpr bool LDA = S::LDA;
    constexpr int NC = LDA ? kMaxCls : 1;
    __shared__ float Gold[kFT * GLD], Vn[kFT * VLD], Gn[kFT * VLD];
    __shared__ float Tt[KP * KP];
    __shared__ float cInv[KP], cMB[KP], cMAc[KP], cUc[KP];
    __shared__ float cSp[NC * KP], cU[NC * KP];
    __shared__ float Mt[NC * kFT], Mb[LDA ? kFT : 1];
    __shared__ float muT[LDA ? 1 : kFT], xcs[LDA ? 1 : kFT], cP[LDA ? 1 : KP], cQ[LDA ? 1 : KP];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6); // wave index, scalar
    const int l16 = lane & 15, g = lane >> 4;
    const int wg = xcd_tile(blockIdx.x, gridDim.x);
    const int nt0 = a.nsubv[0] * (a.ft / kFT); // 64-feature tiles of view 0
    const int v = wg < nt0 ? 0 : 1;
    const int64_t fvh = (int64_t)kFT * (v ? wg - nt0 : wg);
    const int64_t dv = a.dv[v];
    const int64_t frow = a.off[v] + fvh;
    const bool CEN = !LDA && a.center != 0; // centring (CCA): rank-one corrections
    const double t = a.coef->t;
    const double ib = 1.0 / (double)a.b;
    const float eta = (float)eta_sched(a, t), gam = (float)a.gamma, ibf = (float)ib;
    const float eps = (float)a.eps_reg;
    const float b1 = (float)a.adam_b1, b2 = (float)a.adam_b2, aeps = (float)a.adam_eps;
    const float c1 = (float)(1.0 - pow(a.adam_b1, t)), c2 = (float)(1.0 - pow(a.adam_b2, t));

    // ---- everything the tile needs, in one round of loads: every load of a
    // thread is issued before its first LDS store ----
    constexpr int NTT = 4 * NT / kBW;      // epilogue tiles per wave
    constexpr int PT = KP * KP / kBT;      // T
    constexpr int PG = kFT * KP / kBT;     // old auxiliary tile
    constexpr int PS = LDA ? NC * KP / kBT : 1; // class terms S, U
    constexpr int PM = LDA ? NC * kFT / kBT : 1; // class means
    constexpr int NPR = LDA ? 1 : 2;       // products per element: B_t V (LDA); X^T Q, X^T P
    const float *ct = a.ctile;
    float rT[PT], rG[PG], rS[PS], rU[PS], rM[PM], rMb = 0.f, rc[4] = {0.f, 0.f, 0.f, 0.f};
    float rmu = 0.f, rxs = 0.f, rcs = 0.f; // centring: mean, column sum, W column sum
    float vold_[NTT][4], prr[NTT][4][NPR];
#pragma unroll
    for (int q = 0; q < PT; ++q)
        rT[q] = ct[tid + q * kBT];
    if (tid < KP) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            rc[j] = ct[KP * KP + j * KP + tid]; // 1/||v||, m_B, m_A - c, sum_c pi_c U
    }
    if (CEN) {
        if (tid < kFT) {
            rmu = a.mu[frow + tid];
            rxs = a.xsum[frow + tid];
        }
        if (tid < 2 * KP) // sum P (tid < KP), then sum Q
            rcs = ct[KP * KP + 4 * KP + tid];
    }
    if (LDA) {
#pragma unroll
        for (int q = 0; q < PS; ++q) {
            rS[q] = ct[KP * KP + 4 * KP + tid + q * kBT];
            rU[q] = ct[KP * KP + 4 * KP + NC * KP + tid + q * kBT];
        }
#pragma unroll
        for (int q = 0; q < PM; ++q) {
            const int e = tid + q * kBT, c = e / kFT, fl = e % kFT;
            rM[q] = c < a.ncls ? a.M[(int64_t)c * a.dtot + frow + fl] : 0.f;
        }
        if (tid < kFT)
            rMb = a.Mbar[frow + tid];
    }
#pragma unroll
    for (int q = 0; q < PG; ++q)
        rG[q] = a.G[frow * KP + tid + q * kBT];
    // this lane's own elements of its epilogue tiles: old players and products
    const float *pin = a.prod + frow * MWA;
#pragma unroll
    for (int h = 0; h < NTT; ++h) {
        const int tt = w + kBW * h, fb = tt / NT, pb = tt % NT, i = 16 * pb + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int fl = 16 * fb + 4 * g + r;
            vold_[h][r] = a.V[(frow + fl) * KP + i];
            if (LDA) {
                prr[h][r][0] = pin[fl * MWA + i];
            } else { // view x: A_t from X^T Q (second half of the row), B_t from X^T P
                prr[h][r][0] = pin[fl * MWA + KP + i];
                prr[h][r][NPR - 1] = pin[fl * MWA + i];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PT; ++q)
        Tt[tid + q * kBT] = rT[q];
    if (tid < KP) {
        cInv[tid] = rc[0];
        cMB[tid] = rc[1];
        cMAc[tid] = rc[2];
        cUc[tid] = rc[3];
    }
    if (LDA) {
#pragma unroll
        for (int q = 0; q < PS; ++q) {
            cSp[tid + q * kBT] = rS[q];
            cU[tid + q * kBT] = rU[q];
        }
#pragma unroll
        for (int q = 0; q < PM; ++q)
            Mt[tid + q * kBT] = rM[q];
        if (tid < kFT)
            Mb[tid] = rMb;
    }
#pragma unroll
    for (int q = 0; q < PG; ++q) {
        const int e = tid + q * kBT;
        Gold[(e / KP) * GLD + e % KP] = rG[q];
    }
    if (CEN) {
        if (tid < kFT) {
            muT[tid] = rmu;
            xcs[tid] = rxs;
        }
        if (tid < KP)
            cP[tid] = rcs;
        else if (tid < 2 * KP)
            cQ[tid - KP] = rcs;
    }
    __syncthreads();

#pragma unroll
    for (int h = 0; h < NTT; ++h) {
        const int tt = w + kBW * h, fb = tt / NT, pb = tt % NT;
        f32x4 pen = {0.f, 0.f, 0.f, 0.f}, e2 = pen, e3 = pen;
#pragma unroll 4
        for (int j0 = 0; j0 < KP; j0 += 4)
            pen = __builtin_amdgcn_mfma_f32_16x16x4f32(Gold[(16 * fb + l16) * GLD + j0 + g],
                                                      Tt[(j0 + g) * KP + 16 * pb + l16], pen, 0, 0, 0);
        if (LDA) {
#pragma unroll
            for (int c0 = 0; c0 < kMaxCls; c0 += 4) {
                const float mA_ = Mt[(c0 + g) * kFT + 16 * fb + l16];
                e2 = __builtin_amdgcn_mfma_f32_16x16x4f32(mA_, cSp[(c0 + g) * KP + 16 * pb + l16], e2, 0, 0, 0);
                e3 = __builtin_amdgcn_mfma_f32_16x16x4f32(mA_, cU[(c0 + g) * KP + 16 * pb + l16], e3, 0, 0, 0);
            }
        }
        const int i = 16 * pb + l16;
        float vold[4], mold[4], sold[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t si = (frow + 16 * fb + 4 * g + r) * KP + i;
            vold[r] = vold_[h][r];
            if (OPT != kOptSGD) {
                mold[r] = a.Am[si];
                sold[r] = a.As[si];
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int fl = 16 * fb + 4 * g + r; // FP32 D row 4 (l/16) + r
            const int64_t si = (frow + fl) * KP + i;
            float vn = 0.f, gn = 0.f;
            if (fvh + fl < dv && i < a.k) {
                const float inv = cInv[i];
                const float vh = vold[r] * inv;
                float av, bv;
                if (!LDA) {
                    const float sf = IN == kInFP8 ? a.colscale[frow + fl] : 1.f;
                    // view x: A from X^T Q, B from X^T P; view y: the reverse
                    const float rawA = v == 0 ? prr[h][r][0] : prr[h][r][NPR - 1];
                    const float rawB = v == 0 ? prr[h][r][NPR - 1] : prr[h][r][0];
                    float rA = rawA * sf, rB = rawB * sf;
                    if (CEN) { // (X - 1 mu^T)^T W = X^T W - mu (1^T W)
                        rA -= muT[fl] * (v == 0 ? cQ[i] : cP[i]);
                        rB -= muT[fl] * (v == 0 ? cP[i] : cQ[i]);
                    }
                    av = rA * inv * ibf;
                    bv = rB * inv * ibf;
                } else {
                    bv = (prr[h][r][0] - e2[r]) * inv * ibf + eps * vh;
                    av = e3[r] - Mb[fl] * cUc[i];
                }
                const float grad = (av - pen[r]) * cMB[i] - bv * cMAc[i];
                if (OPT == kOptSGD) {
                    vn = vh + eta * grad;
                } else {
                    const float mm = b1 * mold[r] + (1.f - b1) * grad;
                    const float sq = b2 * sold[r] + (1.f - b2) * grad * grad;
                    a.Am[si] = mm;
                    a.As[si] = sq;
                    vn = vh + eta * (mm / c1) / (sqrtf(sq / c2) + aeps);
                }
                const float g0 = Gold[fl * GLD + i];
                gn = g0 + gam * (bv - g0);
                a.V[si] = vn;
                a.G[si] = gn;
            }
            Vn[fl * VLD + i] = vn;
            Gn[fl * VLD + i] = gn;
        }
    }
    if (CEN && tid < kFT) { // mu += gamma (column mean - mu); Mt row 0 for the statistics
        float mn = 0.f;
        if (fvh + tid < dv) {
            const float sf = IN == kInFP8 ? a.colscale[frow + tid] : 1.f;
            mn = muT[tid] + gam * (xcs[tid] * sf * ibf - muT[tid]);
        }
        a.mu[frow + tid] = mn;
        Mt[tid] = mn;
    }
    __syncthreads();
    f64x4 sacc[StatTiles<KP, KIND>::H];
#pragma unroll
    for (int h = 0; h < StatTiles<KP, KIND>::H; ++h)
        sacc[h] = f64x4{0, 0, 0, 0};
    double nrm = 0.0;
    write_vop<KP, KIND, IN>(a, Vn, frow);
    tile_stats<KP, KIND>(Vn, Gn, Mt, sacc, LDA || CEN);
    tile_norms<KP, KIND>(Vn, nrm);
    write_stats<KP, KIND>(a, wg, sacc, nrm, v);
}

// ---------------------------------------------------------------------------
// Initialisation (same workgroups as k_wbwd): the stored players V (unit
// columns, written by the host) give [Bv] = V (Alg. 2), the V operand and the
// first statistics.
// ---------------------------------------------------------------------------
template <int KP, int IN, int KIND>
__global__ void __launch_bounds__(kBT) k_winit(WideArgs a)
{
    constexpr int VLD = Shape<KP, KIND>::VLD;
    __shared__ float Vn[kFT * VLD];
    __shared__ float Mt[(KIND == kKindLDA ? kMaxCls : 1) * kFT];
    const bool CEN = KIND != kKindLDA && a.center != 0;
    const int tid = threadIdx.x;
    const int wg = blockIdx.x;
    int v, sub0, sub1;
    wg_range(a, wg, v, sub0, sub1);
    f64x4 sacc[StatTiles<KP, KIND>::H];
#pragma unroll
    for (int h = 0; h < StatTiles<KP, KIND>::H; ++h)
        sacc[h] = f64x4{0, 0, 0, 0};
    double nrm = 0.0;
    const int nh = a.ft / kFT;
    for (int sh = sub0 * nh; sh < sub1 * nh; ++sh) { // 64-feature halves of the subtiles
        const int64_t frow = a.off[v] + (int64_t)sh * kFT;
        for (int e = tid; e < kFT * KP; e += kBT) {
            const float x = a.V[frow * KP + e];
            Vn[(e / KP) * VLD + e % KP] = x;
            a.G[frow * KP + e] = x;
        }
        if (KIND == kKindLDA)
            for (int e = tid; e < kMaxCls * kFT; e += kBT) {
                const int c = e / kFT, fl = e % kFT;
                Mt[e] = c < a.ncls ? a.M[(int64_t)c * a.dtot + frow + fl] : 0.f;
            }
        else if (CEN && tid < kFT) // the running means (zero at the start)
            Mt[tid] = a.mu[frow + tid];
        __syncthreads();
        write_vop<KP, KIND, IN>(a, Vn, frow);
        tile_stats<KP, KIND>(Vn, Vn, Mt, sacc, KIND == kKindLDA || CEN);
        tile_norms<KP, KIND>(Vn, nrm);
        __syncthreads();
    }
    write_stats<KP, KIND>(a, wg, sacc, nrm, v);
}

// Read-out after k_wstats: out[i * d + f] (column-major FP64) =
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
