"""Host-only checks of the C ABI (no GPU): the library loads, exports every
entry point that include/nrng.h declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import pytest

from paper_1004_3105_amd import binding as nb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "nrng.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nrng_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    fns = header_functions()
    for name in ("nrng_boxmuller", "nrng_polar", "nrng_batched", "nrng_polar_dev", "nrng_strerror"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    L = nb.lib()
    missing = [f for f in header_functions() if not hasattr(L, f)]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    assert sorted(header_functions()) == nb.EXPORTED
    for f in header_functions():
        assert callable(getattr(nb, f))


def test_strerror_and_version():
    L = nb.lib()
    for code in range(-7, 1):
        assert isinstance(L.nrng_strerror(code), bytes) and len(L.nrng_strerror(code)) > 0
    assert L.nrng_strerror(-99) == b"unknown status"
    assert L.nrng_version() >= 10000


def test_argument_errors_return_before_any_launch():
    L = nb.lib()
    p = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
    # unknown dtype
    assert L.nrng_boxmuller(1, 0, 10, 0.0, 1.0, p, 7, None) == nb.NRNG_EDTYPE
    assert L.nrng_polar(1, 0, 10, 0.0, 1.0, p, -1, None, None) == nb.NRNG_EDTYPE
    assert L.nrng_batched(0, 4, p, p, p, None, p, p, p, 100, 9, None, None) == nb.NRNG_EDTYPE
    # bad mu / sigma
    for mu, sigma in ((0.0, -1.0), (float("nan"), 1.0), (0.0, float("inf")), (float("-inf"), 1.0)):
        assert L.nrng_boxmuller(1, 0, 10, mu, sigma, p, 1, None) == nb.NRNG_EINVAL
        assert L.nrng_polar(1, 0, 10, mu, sigma, p, 1, None, None) == nb.NRNG_EINVAL
        assert L.nrng_test_b1_words(p, 4, mu, sigma, p, 1, None) == nb.NRNG_EINVAL
    # null output with n > 0
    assert L.nrng_boxmuller(1, 0, 10, 0.0, 1.0, None, 1, None) == nb.NRNG_EINVAL
    assert L.nrng_polar(1, 0, 10, 0.0, 1.0, None, 1, None, None) == nb.NRNG_EINVAL
    assert L.nrng_polar_dev(1, None, 10, 0.0, 1.0, p, 1, None) == nb.NRNG_EINVAL
    # n = 0 is a no-op
    assert L.nrng_boxmuller(1, 0, 0, 0.0, 1.0, None, 1, None) == nb.NRNG_OK
    assert L.nrng_polar(1, 0, 0, 0.0, 1.0, None, 1, None, None) == nb.NRNG_OK
    # batched: bad method, zero streams, null arrays
    assert L.nrng_batched(6, 4, p, p, p, None, p, p, p, 100, 1, None, None) == nb.NRNG_EINVAL
    assert L.nrng_batched(0, 0, None, None, None, None, None, None, None, 0, 1, None, None) == nb.NRNG_OK
    assert L.nrng_batched(1, 4, None, p, p, None, p, p, p, 100, 1, None, None) == nb.NRNG_EINVAL
    assert L.nrng_batched(1, 4, p, p, p, None, p, p, None, 100, 1, None, None) == nb.NRNG_EINVAL
    # the timed exec needs both events
    for e0, e1 in ((None, p), (p, None), (None, None)):
        assert L.nrng_batched_exec_timed(0, 0, 4, p, p, p, None, p, p, p, 1, None, None, e0, e1) == nb.NRNG_EINVAL
    # ... and a part with a main kernel (0 or 2)
    for part in (-1, 1, 3):
        assert L.nrng_batched_exec_timed(part, 0, 4, p, p, p, None, p, p, p, 1, None, None, p, p) == nb.NRNG_EINVAL
    # sizes beyond the supported range: 2^41 values for the rejection methods
    # and for a batch's output, 2^62 for the Box-Muller family
    assert L.nrng_polar(1, 0, (1 << 41) + 1, 0.0, 1.0, p, 1, None, None) == nb.NRNG_ERANGE
    assert L.nrng_polar2(1, 0, (1 << 41) + 1, 0.0, 1.0, p, 1, None, None) == nb.NRNG_ERANGE
    assert L.nrng_ratio(1, 0, (1 << 41) + 1, 0.0, 1.0, p, 1, None, None) == nb.NRNG_ERANGE
    for fn in (L.nrng_boxmuller, L.nrng_b3, L.nrng_b2):
        assert fn(1, 0, (1 << 62) + 1, 0.0, 1.0, p, 1, None) == nb.NRNG_ERANGE
    # the allocation-free Polar call serves at most 2^26 normals (its fixed
    # scratch), and checks its arguments as nrng_polar does
    assert L.nrng_polar_noalloc(1, 0, (1 << 26) + 1, 0.0, 1.0, p, 1, None, None) == nb.NRNG_ERANGE
    assert L.nrng_polar_noalloc(1, 0, 10, 0.0, 1.0, p, 5, None, None) == nb.NRNG_EDTYPE
    assert L.nrng_polar_noalloc(1, 0, 10, 0.0, -1.0, p, 1, None, None) == nb.NRNG_EINVAL
    assert L.nrng_polar_noalloc(1, 0, 10, 0.0, 1.0, None, 1, None, None) == nb.NRNG_EINVAL
    assert L.nrng_polar_noalloc(1, 0, 0, 0.0, 1.0, None, 1, None, None) == nb.NRNG_OK
    for m in range(6):
        assert L.nrng_batched(m, 4, p, p, p, None, p, p, p, (1 << 41) + 1, 1, None, None) == nb.NRNG_ERANGE
    # test hooks
    assert L.nrng_test_polar_budget(1, 0, 10, 0.0, 1.0, p, 1, 0, None, None) == nb.NRNG_EINVAL
    assert L.nrng_test_polar_xy(None, 8, 0.0, 1.0, p, 1, p, p, None) == nb.NRNG_EINVAL
    assert L.nrng_polar_trace(1, 0, 64, None, p, None) == nb.NRNG_EINVAL
    assert L.nrng_probe_store(p, 17, None) == nb.NRNG_EINVAL
    # graph helpers
    assert L.nrng_fillgraph_launch(None, None) == nb.NRNG_EINVAL
    assert L.nrng_fillgraph_destroy(None) == nb.NRNG_OK


def test_tune_table_validation():
    L = nb.lib()
    assert nb.nrng_tune_variants(nb.KERNEL_POLAR)
    assert nb.nrng_tune_variants(nb.KERNEL_B1)
    assert L.nrng_tune_set(1, 1, 257, 3, 0) == nb.NRNG_EINVAL
    assert L.nrng_tune_set(7, 1, 256, 4, 0) == nb.NRNG_EINVAL
    assert L.nrng_tune_set(1, 9, 256, 4, 0) == nb.NRNG_EDTYPE
    wg, un, g = nb.nrng_tune_get(nb.KERNEL_POLAR, nb.NRNG_F32)
    assert (wg, un) in nb.nrng_tune_variants(nb.KERNEL_POLAR)
    nb.nrng_tune_set(nb.KERNEL_POLAR, nb.NRNG_F32, wg, un, g)


def test_binding_raises_on_error_status():
    with pytest.raises(nb.NrngError):
        nb.nrng_boxmuller(1, 0, 10, 0.0, -1.0, 0x1000, nb.NRNG_F32, 0)


def test_binding_checks_tensor_sizes_before_calling():
    import torch
    small = torch.empty(10, dtype=torch.float32)
    with pytest.raises(ValueError):
        nb.nrng_boxmuller(1, 0, 11, 0.0, 1.0, small, nb.NRNG_F32, 0)
    with pytest.raises(ValueError):
        nb.nrng_polar(1, 0, 6, 0.0, 1.0, small, nb.NRNG_F64, 0)
    with pytest.raises(ValueError):
        nb.nrng_batched(nb.NRNG_METHOD_POLAR, 2, None, None, None, None, None, None, small, 11, nb.NRNG_F32, 0)
    with pytest.raises(ValueError):
        nb.nrng_test_polar_xy(torch.empty(3, dtype=torch.int32), 2, 0.0, 1.0, small, nb.NRNG_F32, None, None, 0)


def test_timed_exec_binding_needs_created_events():
    """The timed exec takes hipEvent_t handles: an int handle passes through,
    and anything without a created event (None, a plain object) is refused
    before the call; a null handle is the library's argument error."""
    assert nb._event(0x1234) == 0x1234
    for bad in (None, object()):
        with pytest.raises(ValueError):
            nb._event(bad)
    p = 0x1000
    with pytest.raises(nb.NrngError) as e:
        nb.nrng_batched_exec_timed(0, nb.NRNG_METHOD_B1, 4, p, p, p, None, p, p, p, nb.NRNG_F32, 0, None, 0, p)
    assert e.value.status == nb.NRNG_EINVAL


def test_b2_kernel_coefficients_equal_the_oracles():
    """Method B2's coefficients are derived twice, independently: by the
    kernels' generator (mpmath quadrature of the Chebyshev coefficients,
    csrc/gen_b2_poly.py) and by the oracle (the truncated series from the
    Taylor series, in long double).  Both round the same truncated series to
    double, so the FP64 values must agree bit for bit; the FP32 ones are
    those doubles rounded to single precision."""
    import numpy as np
    import oracle as O
    text = open(os.path.join(ROOT, "paper_1004_3105_amd", "csrc", "nrng_b2_poly.hpp")).read()

    def arr(name):
        body = re.search(name + r"\[4\] = \{([^}]*)\}", text).group(1)
        return [float.fromhex(x.strip().rstrip("f")) for x in body.split(",")]

    s, c = O.b2_coef()
    assert arr("kB2SinF64") == list(s)
    assert arr("kB2CosF64") == list(c)
    assert arr("kB2SinF32") == [float(np.float32(x)) for x in s]
    assert arr("kB2CosF32") == [float(np.float32(x)) for x in c]


def test_b2_argument_errors():
    L = nb.lib()
    p = ctypes.c_void_p(0x1000)
    assert L.nrng_b2(1, 0, 10, 0.0, 1.0, p, 7, None) == nb.NRNG_EDTYPE
    assert L.nrng_b2(1, 0, 10, 0.0, -1.0, p, 1, None) == nb.NRNG_EINVAL
    assert L.nrng_b2(1, 0, 10, 0.0, 1.0, None, 1, None) == nb.NRNG_EINVAL
    assert L.nrng_b2(1, 0, 0, 0.0, 1.0, None, 1, None) == nb.NRNG_OK
    assert L.nrng_test_b2_words(None, 4, 0.0, 1.0, p, 1, None) == nb.NRNG_EINVAL
    assert L.nrng_batched(nb.NRNG_METHOD_B2, 4, p, p, p, None, p, p, p, 100, 9, None, None) == nb.NRNG_EDTYPE
    assert L.nrng_batched(6, 4, p, p, p, None, p, p, p, 100, 1, None, None) == nb.NRNG_EINVAL


def test_probe_valu_argument_errors():
    L = nb.lib()
    p = ctypes.c_void_p(0x1000)
    assert L.nrng_probe_valu(-1, 16, p, 64, None) == nb.NRNG_EINVAL
    assert L.nrng_probe_valu(len(nb.VALU_PROBE_OPS), 16, p, 64, None) == nb.NRNG_EINVAL
    assert L.nrng_probe_valu(0, 16, None, 64, None) == nb.NRNG_EINVAL
    assert L.nrng_probe_valu(0, 16, p, 0, None) == nb.NRNG_EINVAL


def test_tune_load_applies_a_valid_table_and_rejects_a_bad_one(tmp_path):
    from paper_1004_3105_amd import autotune
    saved = {(k, d): nb.nrng_tune_get(k, d) for k in (0, 1, 2) for d in (0, 1, 2, 3)}
    try:
        good = tmp_path / "t.txt"
        good.write_text("# comment\npolar f32 512 32 3\n\nb1_batched bf16 256 2 0  # trailing\n")
        nb.nrng_tune_load(str(good))
        assert nb.nrng_tune_get(1, nb.NRNG_F32) == (512, 32, 3)
        assert nb.nrng_tune_get(2, nb.NRNG_BF16) == (256, 2, 0)
        assert nb.nrng_tune_get(0, nb.NRNG_F32) == saved[(0, nb.NRNG_F32)]      # untouched
        for text in ("polar f32 512 33 0\n", "polar f99 256 32 0\n", "nope f32 256 32 0\n", "polar f32 256\n"):
            bad = tmp_path / "bad.txt"
            bad.write_text("b1 f64 256 1 0\n" + text)
            before = nb.nrng_tune_get(0, nb.NRNG_F64)
            with pytest.raises(nb.NrngError):
                nb.nrng_tune_load(str(bad))
            assert nb.nrng_tune_get(0, nb.NRNG_F64) == before                  # nothing applied
        with pytest.raises(nb.NrngError):
            nb.nrng_tune_load(str(tmp_path / "missing.txt"))
        assert nb.lib().nrng_tune_load(None) == nb.NRNG_EINVAL
        # the autotuner's text form round-trips through the C loader
        tab = {"arch": "gfx950", "entries": [{"kernel": "b1", "dtype": "f16", "wg": 512, "unroll": 2,
                                              "grid_per_cu": 4}]}
        rt = tmp_path / "rt.txt"
        rt.write_text(autotune.text_table(tab))
        assert autotune.apply(str(rt))
        assert nb.nrng_tune_get(0, nb.NRNG_F16) == (512, 2, 4)
    finally:
        for (k, d), v in saved.items():
            nb.nrng_tune_set(k, d, *v)


def test_compiled_defaults_equal_the_committed_tune_table():
    """The library's compiled launch defaults are the table the autotuner
    wrote for the current kernels (paper_1004_3105_amd/tune_gfx950.txt)."""
    path = os.path.join(ROOT, "paper_1004_3105_amd", "tune_gfx950.txt")
    kid = {"b1": nb.KERNEL_B1, "polar": nb.KERNEL_POLAR, "b1_batched": nb.KERNEL_B1_BATCHED}
    did = {"f64": nb.NRNG_F64, "f32": nb.NRNG_F32, "bf16": nb.NRNG_BF16, "f16": nb.NRNG_F16}
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 12
    for k, d, wg, un, gpc in rows:
        assert nb.nrng_tune_get(kid[k], did[d]) == (int(wg), int(un), int(gpc)), (k, d)
