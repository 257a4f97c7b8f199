"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
include/sgep.h declares, the header compiles as C and C++, the ctypes config
mirrors the C struct layout, and argument validation answers synchronously
without touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgep.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sgep_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2206_04993_amd as sg
    lib = sg.load()
    names = _declared()
    assert "sgep_init" in names and "sgep_step" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sg.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", sg.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sgep_[a-z_]+)\b", out))
    assert set(names) <= exported


def test_header_compiles_as_c_and_cpp_and_layout_matches(tmp_path):
    import paper_2206_04993_amd as sg
    prog = tmp_path / "lay.c"
    fields = [f[0] for f in sg.sgep_config._fields_]
    body = "\n".join(f'printf("%zu\\n", offsetof(sgep_config, {f}));' for f in fields)
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "sgep.h"\n'
                    'int main(void){' + body + 'printf("%zu\\n", sizeof(sgep_config));return 0;}\n')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                    str(prog), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    offs = [getattr(sg.sgep_config, f).offset for f in fields]
    assert vals[:-1] == offs
    assert vals[-1] == ctypes.sizeof(sg.sgep_config)
    cpp = tmp_path / "h.cpp"
    cpp.write_text('#include "sgep.h"\nint main(){ sgep_config c{}; (void)c; return 0; }\n')
    subprocess.run(["g++", "-std=c++11", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                    "-c", str(cpp), "-o", str(tmp_path / "h.o")], check=True)


def _init_status(cfg, V0=None):
    import paper_2206_04993_amd as sg
    lib = sg.load()
    d = cfg.dx + cfg.dy if cfg.kind == sg.SGEP_KIND_CCA else cfg.dx
    if V0 is None:
        V0 = np.ones((cfg.k, max(d, 1)))
    V0 = np.ascontiguousarray(V0, dtype=np.float64)
    h = ctypes.c_void_p()
    return lib.sgep_init(ctypes.byref(h), ctypes.byref(cfg),
                         V0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)


def test_config_validation_is_synchronous():
    import paper_2206_04993_amd as sg
    mk = sg.make_config
    C, G, L = sg.SGEP_KIND_CCA, sg.SGEP_KIND_GENERAL, sg.SGEP_KIND_LDA
    cases = [
        (mk(C, sg.SGEP_F32, 0, 8, 8, 16), sg.SGEP_EINVAL),          # k = 0
        (mk(C, sg.SGEP_F32, 65, 64, 64, 16), sg.SGEP_EUNSUPPORTED),  # k > 64
        (mk(C, sg.SGEP_F64, 33, 64, 64, 16), sg.SGEP_EUNSUPPORTED),  # F64 k > 32
        (mk(C, sg.SGEP_F32, 4, 0, 8, 16), sg.SGEP_ESHAPE),           # empty view
        (mk(C, sg.SGEP_F32, 4, 8, 8, 0), sg.SGEP_ESHAPE),            # b_max = 0
        (mk(C, sg.SGEP_F32, 20, 8, 8, 16), sg.SGEP_ESHAPE),          # k > d
        (mk(G, sg.SGEP_F32, 4, 8, 9, 16), sg.SGEP_ESHAPE),           # general needs dx == dy
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, gamma=0.0), sg.SGEP_EINVAL),
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, gamma=1.5), sg.SGEP_EINVAL),
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, rho=-1.0), sg.SGEP_EINVAL),
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, eps_reg=1e-3), sg.SGEP_EINVAL),  # ridge is GENERAL only
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, schedule=sg.SGEP_SCHED_INV, t0=0.0), sg.SGEP_EINVAL),
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, schedule=7), sg.SGEP_EINVAL),
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, optimizer=sg.SGEP_ADAM, adam_b1=1.0), sg.SGEP_EINVAL),
        (mk(G, sg.SGEP_BF16, 4, 8, 8, 16), sg.SGEP_EUNSUPPORTED),    # BF16: CCA and LDA only
        (mk(C, sg.SGEP_BF16, 40, 64, 64, 16), sg.SGEP_EUNSUPPORTED),  # BF16 CCA: k <= 32
        (mk(C, sg.SGEP_BF16, 4, 12, 8, 16), sg.SGEP_ESHAPE),         # BF16 widths: multiples of 8
        (mk(C, sg.SGEP_FP8_E4M3, 4, 8, 8, 16), sg.SGEP_EINVAL),      # FP8 needs column scales
        (mk(C, 4, 4, 8, 8, 16), sg.SGEP_EINVAL),                     # unknown dtype
        (mk(L, sg.SGEP_F64, 4, 8, 0, 16, n_classes=3), sg.SGEP_EUNSUPPORTED),  # LDA: BF16, F32
        (mk(L, sg.SGEP_F32, 4, 12, 0, 16, n_classes=3), sg.SGEP_ESHAPE),  # LDA: d multiple of 8
        (mk(L, sg.SGEP_FP8_E4M3, 4, 8, 0, 16, n_classes=3), sg.SGEP_EUNSUPPORTED),
        (mk(L, sg.SGEP_BF16, 4, 8, 0, 16, n_classes=1), sg.SGEP_EINVAL),   # >= 2 classes
        (mk(L, sg.SGEP_BF16, 4, 8, 0, 16, n_classes=17), sg.SGEP_EINVAL),  # <= 16 classes
        (mk(L, sg.SGEP_BF16, 4, 8, 8, 16, n_classes=3), sg.SGEP_ESHAPE),   # LDA: dy = 0
        (mk(L, sg.SGEP_BF16, 4, 8, 0, 16, n_classes=3), sg.SGEP_EINVAL),   # no class means
        (mk(9, sg.SGEP_F32, 4, 8, 8, 16), sg.SGEP_EINVAL),
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, smooth=2, nu=10.0), sg.SGEP_EINVAL),    # Alg. 2 or 3
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, center=2), sg.SGEP_EINVAL),
        (mk(sg.SGEP_KIND_ICA, sg.SGEP_BF16, 4, 16, 0, 16), sg.SGEP_EUNSUPPORTED),  # ICA: F64/F32
        (mk(sg.SGEP_KIND_ICA, sg.SGEP_F32, 4, 16, 8, 16), sg.SGEP_ESHAPE),         # one stream
        (mk(sg.SGEP_KIND_ICA, sg.SGEP_F32, 4, 16, 0, 16, center=1), sg.SGEP_EUNSUPPORTED),
        (mk(sg.SGEP_KIND_ICA, sg.SGEP_F32, 4, 16, 0, 16, n_classes=3), sg.SGEP_EINVAL),
        (mk(L, sg.SGEP_BF16, 4, 8, 0, 16, n_classes=3, center=1), sg.SGEP_EUNSUPPORTED),
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, smooth=1, rho=0.0, nu=10.0), sg.SGEP_EINVAL),  # rho > 0
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, smooth=1, rho=1e-2, nu=1e-2), sg.SGEP_EINVAL),  # nu > rho
        (mk(C, sg.SGEP_F32, 4, 8, 8, 16, smooth=1, rho=1e-2, nu=float("inf")), sg.SGEP_EINVAL),
    ]
    for cfg, want in cases:
        assert _init_status(cfg) == want, (cfg.kind, cfg.dtype, cfg.k, want)


def test_auxiliary_data_validation_is_synchronous():
    """Missing, extra or non-finite FP8 scales / LDA class data are refused
    before any device work."""
    import paper_2206_04993_amd as sg
    mk = sg.make_config
    C, L = sg.SGEP_KIND_CCA, sg.SGEP_KIND_LDA
    fp8 = mk(C, sg.SGEP_FP8_E4M3, 4, 8, 8, 16)
    bf16 = mk(C, sg.SGEP_BF16, 4, 8, 8, 16)
    lda = mk(L, sg.SGEP_BF16, 4, 8, 0, 16, n_classes=3)
    ones8 = np.ones(8)
    means, priors = np.zeros((3, 8)), np.full(3, 1.0 / 3)
    cases = [
        (fp8, dict(x_col_scale=ones8), sg.SGEP_EINVAL),                       # y scales missing
        (fp8, dict(x_col_scale=ones8, y_col_scale=-ones8), sg.SGEP_EINVAL),    # non-positive
        (fp8, dict(x_col_scale=np.r_[ones8[:7], np.inf], y_col_scale=ones8), sg.SGEP_EINVAL),
        (bf16, dict(x_col_scale=ones8, y_col_scale=ones8), sg.SGEP_EINVAL),    # BF16 has no scales
        (lda, dict(class_means=means), sg.SGEP_EINVAL),                        # priors missing
        (lda, dict(class_means=means, class_priors=np.array([0.5, 0.5, 0.0])), sg.SGEP_EINVAL),
        (lda, dict(class_means=means * np.nan, class_priors=priors), sg.SGEP_EINVAL),
        (bf16, dict(class_means=means, class_priors=priors), sg.SGEP_EINVAL),  # CCA has no classes
    ]
    for cfg, aux, want in cases:
        with pytest.raises(sg.SgepError) as ei:
            sg.sgep_init_ex(cfg, np.ones((8 if cfg.kind == L else 16, 4)), **aux)
        assert ei.value.status == want, (cfg.kind, cfg.dtype, sorted(aux))


def test_null_arguments_rejected():
    import paper_2206_04993_amd as sg
    lib = sg.load()
    assert lib.sgep_init(None, None, None, None) == sg.SGEP_EINVAL
    cfg = sg.make_config(sg.SGEP_KIND_CCA, sg.SGEP_F32, 4, 8, 8, 16)
    h = ctypes.c_void_p()
    assert lib.sgep_init(ctypes.byref(h), ctypes.byref(cfg), None, None) == sg.SGEP_EINVAL
    for fn in ("sgep_sync", "sgep_destroy"):
        assert getattr(lib, fn)(None) == sg.SGEP_EINVAL
    assert lib.sgep_step(None, None, 0, None, 0, 1) == sg.SGEP_EINVAL
    assert lib.sgep_step_lda(None, None, 0, None, 1) == sg.SGEP_EINVAL
    assert lib.sgep_kernels_per_step(None, None) == sg.SGEP_EINVAL
    assert lib.sgep_step_kernel_name(None, 0) is None
    assert lib.sgep_means(None, None) == sg.SGEP_EINVAL
    assert lib.sgep_step_profiled(None, None, 0, None, 0, None, 1, None, 0) == sg.SGEP_EINVAL
    assert lib.sgep_init_ex(None, None, None, None, None) == sg.SGEP_EINVAL
    assert sg.sgep_status_string(sg.SGEP_EPOISONED).startswith("handle poisoned")
    assert sg.sgep_version() >= 100


def test_batch_validation_is_synchronous():
    """Batch creation refuses bad arguments before any device work."""
    import paper_2206_04993_amd as sg
    lib = sg.load()
    mk = sg.make_config

    def status(n, d, ld, cfg, V0s):
        bt = ctypes.c_void_p()
        d64 = (ctypes.c_int64 * max(1, n))(*d)
        ld64 = (ctypes.c_int64 * max(1, n))(*ld)
        cols = [np.ascontiguousarray(v, dtype=np.float64) for v in V0s]
        ptrs = (ctypes.POINTER(ctypes.c_double) * max(1, n))(
            *[c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if c.size else None
              for c in cols])
        return lib.sgep_batch_init(ctypes.byref(bt), n, d64, ld64, ctypes.byref(cfg), ptrs,
                                   None)

    G = sg.SGEP_KIND_GENERAL
    ok = mk(G, sg.SGEP_F32, 4, 0, 0, 16)
    V = [np.ones((4, 32)), np.ones((4, 40))]
    assert status(0, [32], [32], ok, V[:1]) == sg.SGEP_EINVAL                  # n = 0
    assert status(2, [32, 40], [32, 39], ok, V) == sg.SGEP_ESHAPE              # ld < d
    assert status(2, [32, 0], [32, 40], ok, V) == sg.SGEP_ESHAPE               # d = 0
    assert status(2, [32, 40], [32, 40], ok, [V[0], np.zeros(0)]) == sg.SGEP_EINVAL  # V0 NULL
    assert status(1, [32], [32], mk(sg.SGEP_KIND_CCA, sg.SGEP_F32, 4, 16, 16, 16),
                  V[:1]) == sg.SGEP_EUNSUPPORTED                                # GENERAL only
    assert status(1, [32], [32], mk(G, sg.SGEP_BF16, 4, 0, 0, 16),
                  V[:1]) == sg.SGEP_EUNSUPPORTED                                # F32 / F64 only
    assert lib.sgep_batch_init(None, 1, None, None, None, None, None) == sg.SGEP_EINVAL
    for fn in ("sgep_batch_sync", "sgep_batch_destroy"):
        assert getattr(lib, fn)(None) == sg.SGEP_EINVAL
    assert lib.sgep_batch_step(None, None, None, 1) == sg.SGEP_EINVAL
    assert lib.sgep_batch_tune(None, None, None, 1, 1, None) == sg.SGEP_EINVAL
    assert lib.sgep_batch_plan(None, None, None) == sg.SGEP_EINVAL
    assert lib.sgep_batch_launches(None, None, None, 0) == sg.SGEP_EINVAL
