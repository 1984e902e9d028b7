"""GPU parity of Algorithm R (Section 5 of the paper: the ratio method in its
basic form; x = sqrt(8/e)(v - 1/2)/(1 - u), accepted iff
x^2 <= -4 ln(1 - u), one value sigma x + mu per accepted candidate) against
the FP64 oracle, through the C ABI.

Bars: accept masks, word prefixes, output indices and consumed counts
bit-exact (the test is decided in FP64 on both sides, in the same order of
operations); FP64 values within 4 ulp (D2 when mu != 0); FP32 within
2e-6 max(1, |z|) (widened by |mu| and sigma |n|); BF16/FP16 within one unit
of the format plus the FP32 bar."""
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


def test_ratio_f64_stream():
    n = (1 << 22) + 3
    ref, used = O.ratio(21, 0, n)
    zt, cons = run("ratio", 21, 0, n, nb.NRNG_F64, with_consumed=True)
    assert cons == used
    assert_close(host(zt), ref, nb.NRNG_F64, what="ratio f64")


@pytest.mark.parametrize("seed,offset,mu,sigma", [(21, 0, 0.0, 1.0), (0xBEEF, 77, 6.0, 0.5)])
def test_ratio_f32_stream(seed, offset, mu, sigma):
    n = (1 << 23) + 1
    ref, used = O.ratio(seed, offset, n, mu, sigma)
    zt, cons = run("ratio", seed, offset, n, nb.NRNG_F32, mu, sigma, with_consumed=True)
    assert cons == used
    assert_close(host(zt), ref, nb.NRNG_F32, mu, sigma, what="ratio f32")


@pytest.mark.parametrize("dtype", [nb.NRNG_BF16, nb.NRNG_F16])
def test_ratio_half_stream(dtype):
    n = (1 << 18) + 7
    ref, used = O.ratio(17, 4, n, -1.0, 0.75)
    zt, cons = run("ratio", 17, 4, n, dtype, -1.0, 0.75, with_consumed=True)
    assert cons == used
    assert_close(host(zt), ref, dtype, -1.0, 0.75, what="ratio half")
    z32 = run("ratio", 17, 4, n, nb.NRNG_F32, -1.0, 0.75)
    assert torch.equal(zt, z32.to(TDT[dtype]))


def test_ratio_trace_bit_exact():
    """Masks and word prefixes over about 1.4e7 candidates (the stream of
    2^23 values of seed 21) against the oracle's FP64 decisions."""
    n = 1 << 23
    _, used = O.ratio(21, 0, n)
    ncand = used // 2 + 777
    masks, pref, _ = O.ratio_trace(21, 0, ncand)
    d = dev()
    nw = (ncand + 63) // 64
    gm = torch.zeros(nw, dtype=torch.int64, device=d)
    gp = torch.zeros(nw, dtype=torch.int64, device=d)
    case("ratio trace", ncand)
    nb.nrng_ratio_trace(21, 0, ncand, gm, gp)
    torch.cuda.synchronize()
    assert np.array_equal(u64(gm), masks)
    assert np.array_equal(u64(gp), pref)


@pytest.mark.parametrize("dtype", FLOAT_DTYPES)
def test_ratio_words_edge_cases(dtype):
    """u = 0; u = 1 - 2^-53 with v = 1/2 + k 2^-53, |k| <= 9 (accepted iff
    |k| <= 7); points 1, 2 and 1024 units of v from the curve on both sides;
    random words.  Masks and count bit-exact."""
    w = synth.ratio_edge_words()
    ncand = w.size // 2
    ref, masks, a = O.ratio_words(w)
    d = dev()
    out = torch.empty(ncand, dtype=TDT[dtype], device=d)
    gm = torch.zeros((ncand + 63) // 64, dtype=torch.int64, device=d)
    cnt = torch.zeros(1, dtype=torch.int64, device=d)
    case("ratio words", NAME[dtype], ncand)
    nb.nrng_test_ratio_words(torch.from_numpy(w.view(np.int64)).to(d), ncand, 0.0, 1.0, out, dtype, gm, cnt)
    torch.cuda.synchronize()
    assert np.array_equal(u64(gm), masks)
    assert int(cnt.item()) == a
    assert_close(host(out[:a]), ref, dtype, what="ratio words")


def test_ratio_hand_values_through_gpu():
    from helpers import closed_form, golden_rows, ulp_dist64
    rows = golden_rows("ratio_hand_values.txt")
    w = np.array([int(round(closed_form(r[c]) * 2.0**53)) << 11 for r in rows for c in range(2)], dtype=np.uint64)
    d = dev()
    n = len(rows)
    out = torch.empty(n, dtype=torch.float64, device=d)
    gm = torch.zeros((n + 63) // 64, dtype=torch.int64, device=d)
    cnt = torch.zeros(1, dtype=torch.int64, device=d)
    case("ratio hand values", n)
    nb.nrng_test_ratio_words(torch.from_numpy(w.view(np.int64)).to(d), n, 0.0, 1.0, out, nb.NRNG_F64, gm, cnt)
    torch.cuda.synchronize()
    acc = [int(r[2]) for r in rows]
    assert int(cnt.item()) == sum(acc)
    bits = [(int(u64(gm)[j // 64]) >> (j % 64)) & 1 for j in range(n)]
    assert bits == acc
    vals = host(out[:sum(acc)])
    k = 0
    for r in rows:
        if r[2] == "0":
            continue
        kind, amt = r[4].split(":")
        want, got = closed_form(r[3]), vals[k]
        if kind == "abs" or want == 0.0:
            assert abs(got - want) <= float(amt), (r, got, want)
        else:
            assert ulp_dist64([got], [want])[0] <= int(amt), (r, got, want)
        k += 1


def test_ratio_budget_continuation():
    """A stream that outgrows its candidate budget continues serially past
    it in its last tile; the result is the same stream."""
    d = dev()
    n = 100001
    ref, cons = run("ratio", 3, 1, n, nb.NRNG_F32, with_consumed=True)
    for words in (1, 2, 33, 1000, 2100, 2140, 2200):
        out = torch.empty(n, dtype=torch.float32, device=d)
        c = torch.zeros(1, dtype=torch.int64, device=d)
        case("ratio budget", words)
        nb.nrng_test_ratio_budget(3, 1, n, 0.0, 1.0, out, nb.NRNG_F32, words, None, c)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), words
        assert int(c.item()) == cons


def test_ratio_offsets_alignment_small_n():
    d = dev()
    for dtype in FLOAT_DTYPES:
        full, used = run("ratio", 9, 50, 5001, dtype, with_consumed=True)
        head, u1 = run("ratio", 9, 50, 1000, dtype, with_consumed=True)
        tail, u2 = run("ratio", 9, 50 + u1, 4001, dtype, with_consumed=True)
        assert torch.equal(torch.cat([head, tail]), full) and u1 + u2 == used
        buf = torch.zeros(5001 + 7, dtype=TDT[dtype], device=d)
        for sh in range(1, 8):
            o = buf[sh:sh + 5001]
            run("ratio", 9, 50, 5001, dtype, out=o)
            assert torch.equal(o, full)
        for n in (1, 2, 3, 7):
            z, c = run("ratio", 9, 50, n, dtype, with_consumed=True)
            assert c == O.ratio(9, 50, n)[1]
            assert torch.equal(z, full[:n])
    z = run("ratio", 9, 0, 999, nb.NRNG_F32, -2.0, 0.0)
    assert torch.all(z == -2.0)


def test_ratio_batched_matches_oracle():
    d = dev()
    cfg = synth.batched_streams(96, n_lo=1.0, n_hi=2e4)
    ns, total = 96, cfg["total"]
    D = {k: torch.from_numpy(cfg[k].view(np.int64) if cfg[k].dtype == np.uint64 else cfg[k]).to(d)
         for k in ("seed", "offset", "n", "mu", "sigma")}
    for dtype in (nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_BF16):
        out = torch.empty(total, dtype=TDT[dtype], device=d)
        cons = torch.zeros(ns, dtype=torch.int64, device=d)
        case("ratio batched", NAME[dtype], ns, total)
        nb.nrng_batched(nb.NRNG_METHOD_R, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out,
                        total, dtype, None, cons)
        torch.cuda.synchronize()
        c = u64(cons)
        z = host(out)
        for j in range(ns):
            n, o0 = int(cfg["n"][j]), int(cfg["out_off"][j])
            mu, sg = float(cfg["mu"][j]), float(cfg["sigma"][j])
            ref, used = O.ratio(int(cfg["seed"][j]), int(cfg["offset"][j]), n, mu, sg)
            assert int(c[j]) == used, j
            assert_close(z[o0:o0 + n], ref, dtype, mu, sg, what="ratio batched stream %d" % j)
        for j in (0, ns // 2, ns - 1):
            n, o0 = int(cfg["n"][j]), int(cfg["out_off"][j])
            zs = run("ratio", int(cfg["seed"][j]), 0, n, dtype, float(cfg["mu"][j]), float(cfg["sigma"][j]))
            assert torch.equal(zs, out[o0:o0 + n])


def test_ratio_results_do_not_depend_on_launch_variant():
    for dtype in (nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_F16):
        saved = nb.nrng_tune_get(nb.KERNEL_POLAR, dtype)
        outs = []
        try:
            for wg, un in nb.nrng_tune_variants(nb.KERNEL_POLAR):
                for gpc in (0, 1):
                    nb.nrng_tune_set(nb.KERNEL_POLAR, dtype, wg, un, gpc)
                    outs.append(run("ratio", 21, 8, 300007, dtype, with_consumed=True))
        finally:
            nb.nrng_tune_set(nb.KERNEL_POLAR, dtype, *saved)
        assert len({c for _, c in outs}) == 1
        for o, _ in outs[1:]:
            assert torch.equal(o, outs[0][0])


def test_ratio_gpu_output_distribution():
    from scipy import stats
    n = 1 << 22
    z = host(run("ratio", 12345, 0, n, nb.NRNG_F32))
    bd = stat_bounds(n)
    assert abs(z.mean()) < bd["mean"]
    assert abs(z.var() - 1) < bd["var"]
    assert abs(stats.skew(z)) < bd["skew"]
    assert abs(stats.kurtosis(z, fisher=False) - 3) < bd["kurt"]
    assert stats.kstest(z, "norm").statistic < bd["ks"]


def test_ratio_error_report(capsys):
    n = 1 << 22
    ref, _ = O.ratio(21, 0, n)
    rows = []
    for dtype in FLOAT_DTYPES:
        z = host(run("ratio", 21, 0, n, dtype))
        frac = assert_close(z, ref, dtype, what="ratio %s" % NAME[dtype])
        rel = float(np.max(np.abs(z - ref) / np.maximum(1.0, np.abs(ref))))
        rows.append("ratio %-4s max|dz|/max(1,|z|) %.3e  %s" % (
            NAME[dtype], rel, ("max ulp %d" % frac) if dtype == nb.NRNG_F64 else ("max err/bar %.3f" % frac)))
    with capsys.disabled():
        print("\n[Algorithm R error report, n = 2^22]\n" + "\n".join(rows), flush=True)
