"""The read-out entry point that allocates no device memory
(sgep_vectors_noalloc), through the C ABI, against sgep_vectors: two calls
in a row on different handles, the second with the smaller read-out, so the
fixed staging array holds the first call's (larger) contents when the second
runs; both bitwise equal to sgep_vectors (the same kernels), with and without
the read-out flags; a read-out larger than the staging array is rejected."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _bf16_dev(X):
    import torch
    bits = synth.bf16_bits(X)
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).cuda().view(torch.bfloat16)


def _lda_solver(sg, d, k, dtype, steps):
    import torch
    gen = synth.LDAClasses(d=d, c=6, r=min(16, d), seed=7)
    cfg = sg.make_config(sg.SGEP_KIND_LDA, dtype, k, d, 0, 96, eta0=0.01, eps_reg=1e-3,
                         n_classes=6)
    s = sg.Solver(cfg, synth.initial_players(d, k, 3), class_means=gen.means,
                  class_priors=np.full(6, 1.0 / 6))
    for t in range(1, steps + 1):
        X, lab = gen.batch(t, 96)
        Xd = (_bf16_dev(X) if dtype == sg.SGEP_BF16
              else torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda())
        s.step(Xd, torch.from_numpy(lab.astype(np.int32)).cuda())
    return s


def _cca_solver(sg, dx, dy, k, steps):
    import torch
    gen = synth.CCAPlanted(dx, dy, np.linspace(0.9, 0.4, 4), sigma=0.5, seed=5)
    cfg = sg.make_config(sg.SGEP_KIND_CCA, sg.SGEP_F32, k, dx, dy, 128, eta0=0.05, gamma=0.5)
    s = sg.Solver(cfg, synth.initial_players(dx + dy, k, 4))
    for t in range(1, steps + 1):
        X, Y = gen.batch(t, 128)
        s.step(torch.from_numpy(X.astype(np.float32)).cuda(),
               torch.from_numpy(Y.astype(np.float32)).cuda())
    return s


def test_noalloc_readout_equals_readout_on_two_calls():
    import paper_2206_04993_amd as sg
    sg.load()
    big = _lda_solver(sg, 4096, 64, sg.SGEP_BF16, 3)      # d k = 262,144
    small = _cca_solver(sg, 520, 300, 12, 3)             # d k = 9,840
    print("no-alloc read-out: LDA BF16 d=4096 k=64, then CCA F32 d=820 k=12", flush=True)
    for s in (big, small):
        for flags in (0, sg.SGEP_VEC_BNORM | sg.SGEP_VEC_CANONICAL):
            a = sg.sgep_vectors_noalloc(s.h, s.d, s.k, flags)
            b = sg.sgep_vectors(s.h, s.d, s.k, flags)
            assert np.array_equal(a, b), (s.d, flags)
            assert np.all(np.isfinite(a))
    # and back to the large one after the small one
    a = sg.sgep_vectors_noalloc(big.h, big.d, big.k, 0)
    assert np.array_equal(a, big.vectors(0))
    with pytest.raises(sg.SgepError) as e:
        sg.sgep_vectors_noalloc(small.h, small.d, small.k, 4)
    assert e.value.status == sg.SGEP_EINVAL
    big.close()
    small.close()


def test_noalloc_readout_rejects_more_than_the_staging_array():
    import paper_2206_04993_amd as sg
    sg.load()
    s = _lda_solver(sg, 65600, 64, sg.SGEP_F32, 0)       # d k = 4,198,400 > 4,194,304
    with pytest.raises(sg.SgepError) as e:
        sg.sgep_vectors_noalloc(s.h, s.d, s.k, 0)
    assert e.value.status == sg.SGEP_EUNSUPPORTED
    assert np.all(np.isfinite(s.vectors(0)))             # the allocating read-out still works
    s.close()
