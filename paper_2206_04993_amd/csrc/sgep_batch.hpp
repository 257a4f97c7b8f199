// sgep_batch.hpp -- batched execution of many independent stochastic
// gamma-EigenGame instances (Alg. 2 per instance, M = 1) that share k, the
// problem kind, the element type and the hyperparameters but not the width d.
//
// One iteration of the whole batch is a short, fixed sequence of launches
// (capturable in one hipGraph).  The instances are split into groups; per
// group there is one forward launch (sgep_kernels.hpp fwd_body for every row
// tile of every instance of the group), one coefficient launch (coef_body,
// one workgroup per instance) and one backward launch per feature-tile height
// in use (bwd_body for every feature tile).  Running the groups
// one after the other keeps each group's minibatches small enough to still
// sit in the last-level cache when the backward launch reads them again.
//
// Within a launch a workgroup finds its (instance, tile) from its index.
// Workgroups are dealt to the eight XCDs round-robin (index % 8), so the
// host assigns every instance to one XCD (largest instances first, each to
// the XCD with the least work so far) and lays the tiles of each XCD's
// instances out in slots index / 8: all tiles of an instance share one L2,
// which holds its players V, its projections P, Q and its Gram partials.
//
// The arithmetic is exactly that of a single handle: an instance advanced by
// the batch holds the same bits as the same instance advanced alone with the
// same feature-tile height.  The batch kernels keep fewer loads in flight per
// wave (LOWREG) so that more workgroups share a CU; that changes when values
// arrive, not the order in which they are summed.
#pragma once

#include "sgep_kernels.hpp"

namespace sgep {
namespace batch {

constexpr uint32_t kNoTile = 0xffffffffu;

struct Launch {
    const StepArgs *args;      // per instance: every field except X, Y, b and n_fwd
    const void *const *X;      // per instance: device pointer of its minibatch view x
    const void *const *Y;      // per instance: view y
    const uint32_t *map;       // forward: instance per (XCD, slot / tiles); backward:
                               // (instance << 16) | tile per (XCD, slot)
    int32_t per_xcd;           // entries per XCD in map
    int64_t b;
};

// the per-instance arguments of this iteration; vector loads also need
// 16-byte aligned views (the table's vec_ok covers the leading dimensions)
__device__ __forceinline__ StepArgs instance_args(const Launch &L,
                                                  const StepArgs *__restrict__ args,
                                                  const void *const *__restrict__ Xs,
                                                  const void *const *__restrict__ Ys,
                                                  uint32_t inst)
{
    StepArgs a = args[inst];
    a.X = Xs[inst];
    a.Y = Ys[inst];
    a.b = L.b;
    a.n_fwd = (int32_t)((L.b + 15) / 16);
    if (((uintptr_t)a.X & 15u) != 0 || ((uintptr_t)a.Y & 15u) != 0)
        a.vec_ok = 0;
    return a;
}

// Forward launch: 8 * per_xcd * (n_fwd + 1) workgroups.  Slot s of XCD x
// takes instance map[x * per_xcd + s / (n_fwd + 1)], row tile s % (n_fwd + 1)
// (the last one of each instance reduces its norm / parent partials).
template <typename T, int KP, int KIND, bool CENTER = false>
__global__ void __launch_bounds__(kNT) k_bfwd(Launch L, const StepArgs *__restrict__ args,
                                        const void *const *__restrict__ Xs,
                                        const void *const *__restrict__ Ys)
{
    const int nf = (int)((L.b + 15) / 16);
    const int x = blockIdx.x & 7, s = blockIdx.x >> 3;
    const int q = s / (nf + 1);
    if (q >= L.per_xcd)
        return;
    const uint32_t inst = L.map[x * L.per_xcd + q];
    if (inst == kNoTile)
        return;
    const StepArgs a = instance_args(L, args, Xs, Ys, inst);
    fwd_body<T, KP, KIND, true, CENTER>(a, s - q * (nf + 1));
}

// Coefficient launch: 8 * per_xcd workgroups over the forward map (one
// instance per entry); each computes its instance's coefficient block.
template <typename T, int KP, int KIND>
__global__ void __launch_bounds__(kNT) k_bcoef(Launch L, const StepArgs *__restrict__ args,
                                        const void *const *__restrict__ Xs,
                                        const void *const *__restrict__ Ys)
{
    const int x = blockIdx.x & 7, s = blockIdx.x >> 3;
    const uint32_t inst = L.map[x * L.per_xcd + s];
    if (inst == kNoTile)
        return;
    const StepArgs a = instance_args(L, args, Xs, Ys, inst);
    coef_body<T, KP, KIND>(a);
}

// Backward launch: 8 * per_xcd workgroups; slot s of XCD x takes the feature
// tile map[x * per_xcd + s] (kNoTile: nothing); coefficients from k_bcoef.
template <typename T, int KP, int MB, int KIND, int OPT, bool CENTER = false>
__global__ void __launch_bounds__(kNT) k_bbwd(Launch L, const StepArgs *__restrict__ args,
                                        const void *const *__restrict__ Xs,
                                        const void *const *__restrict__ Ys)
{
    const int x = blockIdx.x & 7, s = blockIdx.x >> 3;
    const uint32_t e = L.map[x * L.per_xcd + s];
    if (e == kNoTile)
        return;
    const StepArgs a = instance_args(L, args, Xs, Ys, e >> 16);
    bwd_body<T, KP, MB, KIND, OPT, kModePre, true, CENTER>(a, (int)(e & 0xffffu));
}

// ---------------------------------------------------------------------------
// Persistent form: the whole iteration of every instance in one launch.
//
// The host gives every instance to one XCC (largest first, each to the XCC
// with the least total width so far) and writes one work queue per XCC: the
// forward items of an instance (its row tiles, then the workgroup that sums
// the norm / parent partials and advances t), its coefficient item and its
// backward items (feature tiles), with the forward items of the next `lag`
// instances placed between an instance's forward and its coefficient item:
//     F(i1) .. F(i_lag)  F(i_lag+1) C(i1) B(i1)  F(i_lag+2) C(i2) B(i2) ..
// so that the backward of an instance reads its minibatch shortly after its
// forward did (from the last-level cache rather than from HBM) while the
// other workgroups keep streaming the next instances.
//
// Every workgroup reads the XCC it runs on from the hardware register and
// claims the items of that XCC's queue in order by an atomic increment of the
// queue's head (one claim ahead of the item it works on).  A coefficient
// item waits until all forward items of its instance are done, a backward
// item until the coefficient item is.  An item only ever waits for items
// earlier in its queue; every item below the head is held by a running
// workgroup and the smallest unfinished one waits for nothing unfinished, so
// every wait ends without the grid being resident at once.  Waits are bounded
// besides (one poll budget per workgroup for all its waits of the launch; a
// give-up sets kStatusSync in the instance's status word).
//
// Producer and consumer of every exchange run on the same XCC and so share
// its L2: a producer waits for its stores to complete (vmcnt 0) before the
// device-scope increment that publishes them; a consumer, once the count is
// reached, invalidates its CU's L1 before reading, so its loads are served by
// the L2 that holds the producer's data.  The counters are only touched with
// device-scope atomics.  The last workgroup to finish resets every counter
// for the next launch (so a captured graph can be replayed) and flags every
// instance if some queue was left unclaimed (no workgroup on that XCC).
//
// Items run fwd_body, coef_body and bwd_body (kModePre, 16-feature tiles)
// exactly as the grouped launches do: an instance holds the same bits under
// either plan.  The bodies' LDS arrays add up in one kernel, so the form is
// built for up to 32 padded players.
// ---------------------------------------------------------------------------
constexpr int kItemFwd = 0, kItemCoef = 1, kItemBwd = 2;
constexpr int kMaxQueues = 16;                 // the XCC id is a 4-bit field
constexpr int kSyncExit = 16 * kMaxQueues;     // sync[16 q]: claim head of queue q
constexpr int kSyncInst = kSyncExit + 16;      // sync[kSyncInst + 2 i]: forward items of
                                               // instance i done; + 1: coefficients done

struct Queues {
    const unsigned long long *items; // (kind << 48) | (instance << 32) | tile
    const int32_t *meta;             // device: queue q is items[meta[q] .. meta[q] + meta[nq + q])
    int32_t nq;                      // queues: the number of XCCs
    int32_t nf_max;                  // row tiles at b_max; forward item tile nf_max is the
                                     // norm-totals workgroup
    int32_t n;                       // instances
    uint32_t *sync;
};

__device__ __forceinline__ unsigned xcc_id()
{
    // hardware register XCC_ID (gfx942 / gfx950), bits 3:0
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
}

// bounded wait (one thread) for *w >= target; false if the budget ran out
__device__ __forceinline__ bool wait_count(uint32_t *w, uint32_t target, int &budget)
{
    while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (--budget < 0) {
            budget = 0;
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// (at least three waves per SIMD: the bodies on their own need at most ~160
// registers, but together the compiler would take them all and leave one
// workgroup per CU)
// publish the workgroup's results: every store complete, then count
__device__ __forceinline__ void publish(uint32_t *cnt)
{
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// wait (thread 0) for *cnt >= target, then drop this CU's L1 so that the
// workgroup's loads are served by the XCC's L2; a give-up sets kStatusSync
__device__ __forceinline__ void acquire(uint32_t *cnt, uint32_t target, int &budget,
                                        int *status)
{
    if (threadIdx.x == 0) {
        if (!wait_count(cnt, target, budget))
            atomicOr(status, kStatusSync);
        asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
}

template <typename T, int KP, int OPT, bool CENTER = false>
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(2))) k_bpers(Launch L, Queues Q,
                                         const StepArgs *__restrict__ args,
                                         const void *const *__restrict__ Xs,
                                         const void *const *__restrict__ Ys)
{
    constexpr int GEN = kKindGeneral;
    __shared__ unsigned long long s_item;
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    // a workgroup on an XCC without a queue takes no items (the last
    // workgroup out then flags the instances of any queue left unclaimed)
    const unsigned qx = xcc_id();
    const bool mine = qx < (unsigned)Q.nq;
    const int q = mine ? (int)qx : 0;
    const unsigned long long *items = Q.items + Q.meta[q];
    const uint32_t qlen = mine ? (uint32_t)Q.meta[Q.nq + q] : 0u;
    uint32_t *head = Q.sync + 16 * q;
    int budget = kSpinMax; // thread 0's polls for all of this workgroup's waits
    uint32_t nxt = 0;
    if (tid == 0 && mine)
        nxt = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (tid == 0) {
            const uint32_t cur = nxt;
            if (cur < qlen)
                nxt = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
            s_item = cur < qlen ? items[cur] : ~0ull;
        }
        __syncthreads();
        const unsigned long long it = s_item;
        if (it == ~0ull)
            break;
        const int kind = (int)(it >> 48);
        const uint32_t inst = (uint32_t)(it >> 32) & 0xffffu;
        const int tile = (int)(it & 0xffffffffu);
        uint32_t *cnt = Q.sync + kSyncInst + 2 * inst;
        // each kind loads its instance's arguments itself, so that only the
        // fields its body uses are live in it
        if (kind == kItemFwd) {
            const StepArgs a = instance_args(L, args, Xs, Ys, inst);
            // row tiles past this minibatch's rows do nothing but count
            if (tile == Q.nf_max)
                fwd_body<T, KP, GEN, true, CENTER>(a, a.n_fwd);
            else if (tile < a.n_fwd)
                fwd_body<T, KP, GEN, true, CENTER>(a, tile);
            publish(cnt);
        } else if (kind == kItemCoef) {
            // every forward item of the instance done
            acquire(cnt, (uint32_t)Q.nf_max + 1, budget, &args[inst].coef->status);
            const StepArgs a = instance_args(L, args, Xs, Ys, inst);
            coef_body<T, KP, GEN>(a);
            publish(cnt + 1);
        } else {
            // the instance's coefficient block written
            acquire(cnt + 1, 1u, budget, &args[inst].coef->status);
            const StepArgs a = instance_args(L, args, Xs, Ys, inst);
            bwd_body<T, KP, 1, GEN, OPT, kModePre, true, CENTER>(a, tile);
        }
        __syncthreads(); // s_item is rewritten next
    }
    // the last workgroup out resets the counters for the next launch
    if (tid == 0)
        s_flag = __hip_atomic_fetch_add(Q.sync + kSyncExit, 1u, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    __syncthreads();
    if (!s_flag)
        return;
    __shared__ int s_lost;
    if (tid == 0) {
        int lost = 0;
        for (int j = 0; j < Q.nq; ++j)
            if (__hip_atomic_load(Q.sync + 16 * j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                (uint32_t)Q.meta[Q.nq + j])
                lost = 1;
        s_lost = lost;
    }
    __syncthreads();
    for (int j = tid; j < kSyncInst + 2 * Q.n; j += kNT)
        __hip_atomic_store(Q.sync + j, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (s_lost)
        for (int i = tid; i < Q.n; i += kNT)
            atomicOr(&((Coef *)args[i].coef)->status, kStatusSync);
}

} // namespace batch
} // namespace sgep
