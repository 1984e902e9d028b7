"""GPU parity of the HIP path against the FP64 oracle (Algorithms B1 and P,
Section 2 of the paper), through the C ABI.

Bars: FP64 kernels within 4 ulp of the oracle; FP32 within
2e-6 * max(1, |z|) (widened by |mu| and sigma |n| when mu != 0); BF16/FP16
within one unit of the format plus the FP32 bar; Polar accept masks, output
indices and consumed counts bit-exact."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import NAME, TDT, assert_close, case, dev, host, run, u64
from paper_1004_3105_amd import binding as nb

pytestmark = pytest.mark.gpu

FLOAT_DTYPES = [nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_BF16, nb.NRNG_F16]


# ------------------------------------------------------------------ B1
@pytest.mark.parametrize("n", [1 << 20, (1 << 20) + 1])
def test_b1_f64_stream(n):
    ref, _ = O.b1(1, 0, n)
    z = host(run("b1", 1, 0, n, nb.NRNG_F64))
    assert_close(z, ref, nb.NRNG_F64, what="b1 f64")


@pytest.mark.parametrize("seed,offset,mu,sigma", [(1, 0, 0.0, 1.0), (0xDEADBEEF, 12345, 3.5, 2.25),
                                                   ((1 << 64) - 7, 3, -10.0, 0.1)])
def test_b1_f32_stream(seed, offset, mu, sigma):
    n = (1 << 20) + 3
    ref, _ = O.b1(seed, offset, n, mu, sigma)
    z = host(run("b1", seed, offset, n, nb.NRNG_F32, mu, sigma))
    assert_close(z, ref, nb.NRNG_F32, mu, sigma, what="b1 f32")


@pytest.mark.parametrize("dtype", [nb.NRNG_BF16, nb.NRNG_F16])
def test_b1_half_stream(dtype):
    n = (1 << 18) + 5
    ref, _ = O.b1(11, 0, n, 0.5, 1.5)
    zt = run("b1", 11, 0, n, dtype, 0.5, 1.5)
    assert_close(host(zt), ref, dtype, 0.5, 1.5, what="b1 half")
    # the narrow output is the round-to-nearest-even of the kernel's FP32 value
    z32 = run("b1", 11, 0, n, nb.NRNG_F32, 0.5, 1.5)
    assert torch.equal(zt, z32.to(TDT[dtype]))


@pytest.mark.parametrize("dtype", FLOAT_DTYPES)
def test_b1_words_edge_cases(dtype):
    w = synth.b1_edge_words()
    ref = O.b1_words(w)
    d = dev()
    wt = torch.from_numpy(w.view(np.int64)).to(d)
    out = torch.empty(w.size, dtype=TDT[dtype], device=d)
    case("b1 words", w.size)
    nb.nrng_test_b1_words(wt, w.size // 2, 0.0, 1.0, out, dtype)
    torch.cuda.synchronize()
    assert_close(host(out), ref, dtype, what="b1 words")


def test_b1_offsets_alignment_small_n():
    d = dev()
    for dtype in FLOAT_DTYPES:
        full = run("b1", 5, 100, 4099, dtype)
        # the stream from offset + 2k continues the same values
        part = run("b1", 5, 100 + 2 * 37, 4099 - 74, dtype)
        assert torch.equal(part, full[74:])
        # unaligned output pointer gives identical values
        buf = torch.zeros(4099 + 3, dtype=TDT[dtype], device=d)
        for sh in (1, 2, 3):
            o = buf[sh:sh + 4099]
            run("b1", 5, 100, 4099, dtype, out=o)
            assert torch.equal(o, full)
        # small and odd n: the last pair keeps only its first value
        for n in (1, 2, 3, 5, 31):
            z = run("b1", 5, 100, n, dtype)
            assert torch.equal(z, full[:n])
    # sigma = 0: every value is mu
    z = run("b1", 5, 0, 1001, nb.NRNG_F32, 2.5, 0.0)
    assert torch.all(z == 2.5)


# ------------------------------------------------------------------ Polar
def test_polar_f64_stream():
    n = 1 << 24
    ref, used = O.polar(7, 0, n)
    zt, cons = run("polar", 7, 0, n, nb.NRNG_F64, with_consumed=True)
    assert cons == used
    assert_close(host(zt), ref, nb.NRNG_F64, what="polar f64")


@pytest.mark.parametrize("seed,offset,mu,sigma", [(7, 0, 0.0, 1.0), (0xC0FFEE, 999, -4.0, 3.0)])
def test_polar_f32_stream(seed, offset, mu, sigma):
    n = (1 << 24) + 1
    ref, used = O.polar(seed, offset, n, mu, sigma)
    zt, cons = run("polar", seed, offset, n, nb.NRNG_F32, mu, sigma, with_consumed=True)
    assert cons == used
    assert_close(host(zt), ref, nb.NRNG_F32, mu, sigma, what="polar f32")


@pytest.mark.parametrize("dtype", [nb.NRNG_BF16, nb.NRNG_F16])
def test_polar_half_stream(dtype):
    n = (1 << 18) + 1
    ref, used = O.polar(17, 4, n, -1.0, 0.75)
    zt, cons = run("polar", 17, 4, n, dtype, -1.0, 0.75, with_consumed=True)
    assert cons == used
    assert_close(host(zt), ref, dtype, -1.0, 0.75, what="polar half")
    z32 = run("polar", 17, 4, n, nb.NRNG_F32, -1.0, 0.75)
    assert torch.equal(zt, z32.to(TDT[dtype]))


def test_polar_trace_bit_exact():
    n = 1 << 24
    _, used = O.polar(7, 0, n)
    ncand = used // 2 + 777
    masks, pref, _ = O.polar_trace(7, 0, ncand)
    d = dev()
    nw = (ncand + 63) // 64
    gm = torch.zeros(nw, dtype=torch.int64, device=d)
    gp = torch.zeros(nw, dtype=torch.int64, device=d)
    case("polar trace", ncand)
    nb.nrng_polar_trace(7, 0, ncand, gm, gp)
    torch.cuda.synchronize()
    assert np.array_equal(u64(gm), masks)
    assert np.array_equal(u64(gp), pref)


@pytest.mark.parametrize("dtype", FLOAT_DTYPES)
def test_polar_xy_edge_cases(dtype):
    xy = synth.polar_edge_xy()
    ncand = xy.size // 2
    ref, masks, a = O.polar_xy(xy)
    d = dev()
    xt = torch.from_numpy(xy).to(d)
    out = torch.empty(2 * ncand, dtype=TDT[dtype], device=d)
    gm = torch.zeros((ncand + 63) // 64, dtype=torch.int64, device=d)
    cnt = torch.zeros(1, dtype=torch.int64, device=d)
    case("polar xy", ncand)
    nb.nrng_test_polar_xy(xt, ncand, 0.0, 1.0, out, dtype, gm, cnt)
    torch.cuda.synchronize()
    assert np.array_equal(u64(gm), masks)
    assert int(cnt.item()) == a
    assert_close(host(out[:2 * a]), ref, dtype, what="polar xy")


def test_polar_budget_continuation():
    """A stream that outgrows its candidate budget continues serially past it
    in its last tile; the result is the same stream.  Budgets below, at and
    above the need (about 995 words of 64 candidates here), ending inside and
    at the end of a tile."""
    d = dev()
    n = 100001
    ref, cons = run("polar", 3, 1, n, nb.NRNG_F32, with_consumed=True)
    for words in (1, 2, 33, 500, 990, 994, 995, 996, 1024, 1100):
        out = torch.empty(n, dtype=torch.float32, device=d)
        c = torch.zeros(1, dtype=torch.int64, device=d)
        case("polar budget", words)
        nb.nrng_test_polar_budget(3, 1, n, 0.0, 1.0, out, nb.NRNG_F32, words, None, c)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), words
        assert int(c.item()) == cons


def test_polar_offsets_alignment_small_n():
    d = dev()
    for dtype in FLOAT_DTYPES:
        full, used = run("polar", 9, 50, 5001, dtype, with_consumed=True)
        head, u1 = run("polar", 9, 50, 1000, dtype, with_consumed=True)
        tail, u2 = run("polar", 9, 50 + u1, 4001, dtype, with_consumed=True)
        assert torch.equal(torch.cat([head, tail]), full) and u1 + u2 == used
        buf = torch.zeros(5001 + 3, dtype=TDT[dtype], device=d)
        for sh in (1, 2, 3):
            o = buf[sh:sh + 5001]
            run("polar", 9, 50, 5001, dtype, out=o)
            assert torch.equal(o, full)
        for n in (1, 2, 3, 7):
            z, c = run("polar", 9, 50, n, dtype, with_consumed=True)
            r, uc = O.polar(9, 50, n)
            assert c == uc
            assert torch.equal(z, full[:n])
    z = run("polar", 9, 0, 999, nb.NRNG_F32, -2.0, 0.0)
    assert torch.all(z == -2.0)


def test_counter_wraps_mod_2_64():
    seed = (1 << 64) - 100
    for method, fn in (("b1", O.b1), ("polar", O.polar)):
        ref, _ = fn(seed, 37, 4001)
        z = host(run(method, seed, 37, 4001, nb.NRNG_F64))
        assert_close(z, ref, nb.NRNG_F64, what=method + " wrap")


# ------------------------------------------------------------------ launch variants
def test_results_do_not_depend_on_launch_variant():
    for kernel, method in ((nb.KERNEL_B1, "b1"), (nb.KERNEL_POLAR, "polar")):
        for dtype in (nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_BF16):
            saved = nb.nrng_tune_get(kernel, dtype)
            outs = []
            try:
                for wg, un in nb.nrng_tune_variants(kernel):
                    for gpc in (0, 1):
                        nb.nrng_tune_set(kernel, dtype, wg, un, gpc)
                        outs.append(run(method, 21, 8, 300007, dtype, with_consumed=(method == "polar")))
            finally:
                nb.nrng_tune_set(kernel, dtype, *saved)
            if method == "polar":
                assert len({c for _, c in outs}) == 1
                outs = [o for o, _ in outs]
            for o in outs[1:]:
                assert torch.equal(o, outs[0])


# ------------------------------------------------------------------ statistics of GPU output
@pytest.mark.parametrize("method", ["b1", "polar"])
def test_gpu_output_distribution(method):
    from scipy import stats

    from helpers import stat_bounds
    n = 1 << 22
    z = host(run(method, 12345, 0, n, nb.NRNG_F32))
    bd = stat_bounds(n)
    assert abs(z.mean()) < bd["mean"]
    assert abs(z.var() - 1) < bd["var"]
    assert abs(stats.skew(z)) < bd["skew"]
    assert abs(stats.kurtosis(z, fisher=False) - 3) < bd["kurt"]
    assert stats.kstest(z, "norm").statistic < bd["ks"]


# ------------------------------------------------------------------ error report per dtype
def test_error_report_per_dtype(capsys):
    """The error against the FP64 oracle, per method and output dtype, on the
    first 2^22 normals of the seed-1 (B1) and seed-7 (Polar) streams and on a
    mu != 0 stream: FP64 as the largest ulp distance; FP32, BF16 and FP16 as
    the largest |dz| / max(1, |z|) and as the largest fraction of the bar.
    Printed as one line per case (and asserted within the bars)."""
    n = 1 << 22
    rows = []
    for method, seed, mu, sigma in (("b1", 1, 0.0, 1.0), ("polar", 7, 0.0, 1.0),
                                    ("b1", 5, -3.5, 2.0), ("polar", 5, -3.5, 2.0)):
        ref, _ = (O.b1 if method == "b1" else O.polar)(seed, 0, n, mu, sigma)
        for dtype in FLOAT_DTYPES:
            z = host(run(method, seed, 0, n, dtype, mu, sigma))
            frac = assert_close(z, ref, dtype, mu, sigma, what="%s %s" % (method, NAME[dtype]))
            rel = float(np.max(np.abs(z - ref) / np.maximum(1.0, np.abs(ref))))
            rows.append("%-5s mu=%5.1f sigma=%.1f %-4s max|dz|/max(1,|z|) %.3e  %s" % (
                method, mu, sigma, NAME[dtype], rel,
                ("max ulp %d" % frac) if dtype == nb.NRNG_F64 else ("max err/bar %.3f" % frac)))
    with capsys.disabled():
        print("\n[error report, n = 2^22 per case]\n" + "\n".join(rows), flush=True)
