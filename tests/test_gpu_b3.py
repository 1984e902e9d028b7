"""GPU parity of method B3 (Section 3 of the paper: Box-Muller with
m = max(u1, u2), u = m^2, r = sigma m h(v) for u <= 8/9 and
sigma sqrt(-ln(1 - u)) above, angle 2 pi u3 - pi, outputs cos then sin)
against the FP64 oracle, through the C ABI.

Bars: FP64 within 4 ulp plus 4e-15 sigma |n| (helpers.fp64_poly_tol: the
two sides evaluate the degree-15 polynomial by different schemes); FP32
within 2e-6 max(1, |z|) (widened by |mu| and sigma |n| when mu != 0);
BF16/FP16 within one unit of the format plus the FP32 bar.  Consumed counts
are 3 ceil(n/2) by definition (checked on the batched path)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import NAME, TDT, assert_close, case, dev, host, run, u64
from helpers import stat_bounds
from paper_1004_3105_amd import binding as nb

pytestmark = pytest.mark.gpu

FLOAT_DTYPES = [nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_BF16, nb.NRNG_F16]


def test_b3_f64_stream():
    n = (1 << 22) + 1
    ref, _ = O.b3(1, 0, n)
    z = host(run("b3", 1, 0, n, nb.NRNG_F64))
    assert_close(z, ref, nb.NRNG_F64, what="b3 f64", poly=True)


@pytest.mark.parametrize("seed,offset,mu,sigma", [(1, 0, 0.0, 1.0), (0xDEADBEEF, 12345, 3.5, 2.25),
                                                   ((1 << 64) - 7, 3, -10.0, 0.1)])
def test_b3_f32_stream(seed, offset, mu, sigma):
    n = (1 << 22) + 3
    ref, _ = O.b3(seed, offset, n, mu, sigma)
    z = host(run("b3", seed, offset, n, nb.NRNG_F32, mu, sigma))
    assert_close(z, ref, nb.NRNG_F32, mu, sigma, what="b3 f32")


@pytest.mark.parametrize("dtype", [nb.NRNG_BF16, nb.NRNG_F16])
def test_b3_half_stream(dtype):
    n = (1 << 18) + 5
    ref, _ = O.b3(11, 0, n, 0.5, 1.5)
    zt = run("b3", 11, 0, n, dtype, 0.5, 1.5)
    assert_close(host(zt), ref, dtype, 0.5, 1.5, what="b3 half")
    z32 = run("b3", 11, 0, n, nb.NRNG_F32, 0.5, 1.5)
    assert torch.equal(zt, z32.to(TDT[dtype]))


@pytest.mark.parametrize("dtype", FLOAT_DTYPES)
def test_b3_words_edge_cases(dtype):
    """Hand-value uniforms, m within four units of the split u = 8/9 on both
    sides (as u1 and as u2), m = 0 and 1 - 2^-53, angles at every sixteenth
    of a turn, random words."""
    w = synth.b3_edge_words()
    npairs = w.size // 3
    ref = O.b3_words(w)
    d = dev()
    out = torch.empty(2 * npairs, dtype=TDT[dtype], device=d)
    case("b3 words", NAME[dtype], npairs)
    nb.nrng_test_b3_words(torch.from_numpy(w.view(np.int64)).to(d), npairs, 0.0, 1.0, out, dtype)
    torch.cuda.synchronize()
    assert_close(host(out), ref, dtype, what="b3 words", poly=True)


def test_b3_hand_values_through_gpu():
    """The closed-form rows of the oracle's B3 fixture, computed by the FP64
    kernel from words holding exactly those uniforms: the same budgets as
    the oracle's pin."""
    from helpers import closed_form, golden_rows, ulp_dist64
    rows = golden_rows("b3_hand_values.txt")
    words = []
    for r in rows:
        for c in range(3):
            u = closed_form(r[c])
            words.append(int(round(u * 2.0**53)) << 11)
    w = np.array(words, dtype=np.uint64)
    d = dev()
    out = torch.empty(2 * len(rows), dtype=torch.float64, device=d)
    case("b3 hand values", len(rows))
    nb.nrng_test_b3_words(torch.from_numpy(w.view(np.int64)).to(d), len(rows), 0.0, 1.0, out, nb.NRNG_F64)
    torch.cuda.synchronize()
    vals = host(out).reshape(-1, 2)
    for k, r in enumerate(rows):
        kind, amt = r[5].split(":")
        for c in range(2):
            want, got = closed_form(r[3 + c]), vals[k, c]
            if kind == "abs" or want == 0.0:
                assert abs(got - want) <= max(float(amt), 1e-15), (r, c, got, want)
            else:
                assert ulp_dist64([got], [want])[0] <= int(amt), (r, c, got, want)


def test_b3_offsets_alignment_small_n():
    d = dev()
    for dtype in FLOAT_DTYPES:
        full = run("b3", 5, 100, 4099, dtype)
        # the stream from offset + 3k continues the same values (pair k)
        part = run("b3", 5, 100 + 3 * 37, 4099 - 74, dtype)
        assert torch.equal(part, full[74:])
        buf = torch.zeros(4099 + 3, dtype=TDT[dtype], device=d)
        for sh in (1, 2, 3):
            o = buf[sh:sh + 4099]
            run("b3", 5, 100, 4099, dtype, out=o)
            assert torch.equal(o, full)
        for n in (1, 2, 3, 5, 31):
            z = run("b3", 5, 100, n, dtype)
            assert torch.equal(z, full[:n])
    z = run("b3", 5, 0, 1001, nb.NRNG_F32, 2.5, 0.0)
    assert torch.all(z == 2.5)


def test_b3_batched_matches_oracle():
    d = dev()
    cfg = synth.batched_streams(96, n_lo=1.0, n_hi=2e4)
    ns, total = 96, cfg["total"]
    D = {k: torch.from_numpy(cfg[k].view(np.int64) if cfg[k].dtype == np.uint64 else cfg[k]).to(d)
         for k in ("seed", "offset", "n", "mu", "sigma")}
    for dtype in (nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_BF16):
        out = torch.empty(total, dtype=TDT[dtype], device=d)
        cons = torch.zeros(ns, dtype=torch.int64, device=d)
        case("b3 batched", NAME[dtype], ns, total)
        nb.nrng_batched(nb.NRNG_METHOD_B3, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out,
                        total, dtype, None, cons)
        torch.cuda.synchronize()
        c = u64(cons)
        z = host(out)
        for j in range(ns):
            n, o0 = int(cfg["n"][j]), int(cfg["out_off"][j])
            mu, sg = float(cfg["mu"][j]), float(cfg["sigma"][j])
            ref, used = O.b3(int(cfg["seed"][j]), int(cfg["offset"][j]), n, mu, sg)
            assert int(c[j]) == used == 3 * ((n + 1) // 2), j
            assert_close(z[o0:o0 + n], ref, dtype, mu, sg, what="b3 batched stream %d" % j, poly=True)
        # each stream alone through nrng_b3: the same bits
        for j in (0, ns // 2, ns - 1):
            n, o0 = int(cfg["n"][j]), int(cfg["out_off"][j])
            zs = run("b3", int(cfg["seed"][j]), 0, n, dtype, float(cfg["mu"][j]), float(cfg["sigma"][j]))
            assert torch.equal(zs, out[o0:o0 + n])


def test_b3_results_do_not_depend_on_launch_variant():
    for kernel in (nb.KERNEL_B1, nb.KERNEL_B1_BATCHED):
        for dtype in (nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_F16):
            saved = nb.nrng_tune_get(kernel, dtype)
            outs = []
            try:
                for wg, un in nb.nrng_tune_variants(kernel):
                    for gpc in (0, 1):
                        nb.nrng_tune_set(kernel, dtype, wg, un, gpc)
                        if kernel == nb.KERNEL_B1:
                            outs.append(run("b3", 21, 8, 300007, dtype))
                        else:
                            d = dev()
                            nn = torch.tensor([300007, 5, 77777], dtype=torch.int64, device=d)
                            sd = torch.tensor([21, 22, 23], dtype=torch.int64, device=d)
                            zo = torch.zeros(3, dtype=torch.int64, device=d)
                            mu = torch.tensor([0.0, 1.0, -2.0], dtype=torch.float64, device=d)
                            sg = torch.tensor([1.0, 0.5, 3.0], dtype=torch.float64, device=d)
                            o = torch.empty(300007 + 5 + 77777, dtype=TDT[dtype], device=d)
                            case("b3 batched variant", wg, un, gpc)
                            nb.nrng_batched(nb.NRNG_METHOD_B3, 3, sd, zo, nn, None, mu, sg, o, o.numel(), dtype)
                            torch.cuda.synchronize()
                            outs.append(o)
            finally:
                nb.nrng_tune_set(kernel, dtype, *saved)
            for o in outs[1:]:
                assert torch.equal(o, outs[0])


def test_b3_gpu_output_distribution():
    from scipy import stats
    n = 1 << 22
    z = host(run("b3", 12345, 0, n, nb.NRNG_F32))
    bd = stat_bounds(n)
    assert abs(z.mean()) < bd["mean"]
    assert abs(z.var() - 1) < bd["var"]
    assert abs(stats.skew(z)) < bd["skew"]
    assert abs(stats.kurtosis(z, fisher=False) - 3) < bd["kurt"]
    assert stats.kstest(z, "norm").statistic < bd["ks"]
    e = 0.5 * (z[0::2] ** 2 + z[1::2] ** 2)          # -ln(1 - u), u = max(u1, u2)^2 uniform
    assert stats.kstest(e, "expon").statistic < 1.95 / np.sqrt(e.size)


def test_b3_error_report(capsys):
    """Largest error against the oracle per dtype on the first 2^22 normals of
    the seed-1 stream (printed; asserted within the bars)."""
    n = 1 << 22
    ref, _ = O.b3(1, 0, n)
    rows = []
    for dtype in FLOAT_DTYPES:
        z = host(run("b3", 1, 0, n, dtype))
        frac = assert_close(z, ref, dtype, what="b3 %s" % NAME[dtype], poly=True)
        rel = float(np.max(np.abs(z - ref) / np.maximum(1.0, np.abs(ref))))
        rows.append("b3 %-4s max|dz|/max(1,|z|) %.3e  %s" % (
            NAME[dtype], rel, ("max ulp %d" % frac) if dtype == nb.NRNG_F64 else ("max err/bar %.3f" % frac)))
    with capsys.disabled():
        print("\n[B3 error report, n = 2^22]\n" + "\n".join(rows), flush=True)
