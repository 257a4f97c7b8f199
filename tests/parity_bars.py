"""Element-wise comparison of the GPU players with the oracle's, shared by the
parity tests.

With Adam (App. H) an element's first steps are about eta_t g / (|g| + eps):
where the gradient g is at the rounding level (|g| comparable to adam_eps)
the two sides may step in opposite directions, so such an element can differ
by up to 2 sum_t eta_t.  Only elements whose oracle gradient scale, the root
of the bias-corrected second moment, stays below GRAD_TINY may exceed the plain
bar, and by no more than that; every other element must meet the plain bar."""
import numpy as np

GRAD_TINY = 1e-6  # gradient scale of a "rounding-level" element (typical |g| ~ 1e-3)


def assert_players_close(Vg, st, tol, adam=False, eta_sum=0.0, b2=0.999):
    """Vg: GPU players (d, k); st: oracle State after the same t steps."""
    D = np.abs(np.asarray(Vg) - st.V)
    over = D > tol
    if not adam:
        assert not over.any(), float(D.max())
        return
    scale = np.sqrt(st.s2 / (1.0 - b2 ** st.t))
    bad = over & ~(scale <= GRAD_TINY)
    assert not bad.any(), (float(D[bad].max()), float(scale[bad].min()))
    assert float(D.max()) <= 2.0 * eta_sum + tol, float(D.max())
    assert int(over.sum()) <= max(4, 1e-4 * D.size), int(over.sum())
