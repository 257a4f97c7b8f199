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
template <typename T, int KP, int KIND>
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
    fwd_body<T, KP, KIND, true>(a, s - q * (nf + 1));
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
template <typename T, int KP, int MB, int KIND, int OPT>
__global__ void __launch_bounds__(kNT) k_bbwd(Launch L, const StepArgs *__restrict__ args,
                                        const void *const *__restrict__ Xs,
                                        const void *const *__restrict__ Ys)
{
    const int x = blockIdx.x & 7, s = blockIdx.x >> 3;
    const uint32_t e = L.map[x * L.per_xcd + s];
    if (e == kNoTile)
        return;
    const StepArgs a = instance_args(L, args, Xs, Ys, e >> 16);
    bwd_body<T, KP, MB, KIND, OPT, kModePre, true>(a, (int)(e & 0xffffu));
}

} // namespace batch
} // namespace sgep
