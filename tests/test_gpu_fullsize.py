"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (the library's tuned defaults), on outputs
the oracle computes independently:

* single streams of 2^30 normals (B1 seed 1, Polar seed 7): FP32 B1 at
  sampled output indices, each pair from its own counters; FP32 Polar on
  whole candidate chunks, placed by the oracle's own prefix of accepted
  counts, plus the consumed count; and both in full in FP32, BF16 and FP16,
  every value against the oracle's whole stream;
* single streams of 2^30 FP32 normals of P2 (seed 7) and Algorithm R (seed
  21) on whole candidate chunks placed by the oracle's prefix, with the
  consumed count, and of B2 and B3 (seed 1) at sampled output indices;
* the batched workload of 4096 streams (about 4.4e8 normals per method, B1,
  Polar, P2, B3, Algorithm R and B2) in full: every value and every
  consumed count of every stream; and its BF16 and FP16 outputs equal to the
  FP32 output rounded to nearest even, bit for bit;
* 64 graph-replayed fills of 2^28 FP32 Polar normals from one device cursor
  (2^34 normals of one stream): the final cursor against the oracle's count,
  and sampled slices of sampled fills, placed by the oracle's prefix, with
  moments and a KS statistic over all the sampled values.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import NAME, TDT, assert_close, case, dev, host, u64
from helpers import b2_f32_extra, stat_bounds
from paper_1004_3105_amd import binding as nb

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
CHUNK = 1 << 22          # candidate pairs per oracle count / window call


class PolarIndex:
    """The oracle's placement of a Polar stream: accepted counts of
    consecutive candidate chunks and their exclusive prefix."""

    def __init__(self, seed, offset, npairs):
        self.seed, self.offset = seed, offset
        ncand = int(npairs * 4 / np.pi * 1.0005) + (1 << 16)
        while True:
            counts = O.polar_chunk_counts(seed, offset, ncand, CHUNK, THREADS)
            if counts.sum() >= npairs:
                break
            ncand += ncand // 8
        self.ncand = ncand
        self.pref = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)

    def chunk_of_pair(self, a):
        return int(np.searchsorted(self.pref, a, side="right")) - 1

    def window(self, c, mu=0.0, sigma=1.0):
        """Values of the accepted pairs of chunk c, and the first output
        pair index they occupy."""
        c0 = c * CHUNK
        vals = O.polar_window(self.seed, self.offset, c0, min(CHUNK, self.ncand - c0), mu, sigma)
        return vals, int(self.pref[c])

    def consumed(self, npairs):
        """Uniforms consumed by a stream of npairs pairs: 2 (j + 1) for the
        candidate j that supplies pair npairs - 1."""
        c = self.chunk_of_pair(npairs - 1)
        c0 = c * CHUNK
        masks, _, _ = O.polar_trace(self.seed, self.offset + 2 * c0, min(CHUNK, self.ncand - c0))
        bits = np.unpackbits(masks.view(np.uint8), bitorder="little")
        j = c0 + int(np.flatnonzero(bits)[npairs - 1 - int(self.pref[c])])
        return 2 * (j + 1)


class RejIndex:
    """The oracle's placement of a stream of method P2 or Algorithm R:
    accepted counts of consecutive candidate chunks, their exclusive prefix,
    and each chunk's values.  P2 yields a pair per accepted candidate, R one
    value."""

    RATE = {"polar2": np.pi / 4, "ratio": np.sqrt(np.pi * np.e) / 4}

    def __init__(self, kind, seed, offset, n):
        self.kind, self.seed, self.offset = kind, seed, offset
        self.epc = 1 if kind == "ratio" else 2
        need = (n + self.epc - 1) // self.epc
        ncand = int(need / self.RATE[kind] * 1.0005) + (1 << 16)
        while True:
            counts = O.polar_chunk_counts(seed, offset, ncand, CHUNK, THREADS, kind)
            if counts.sum() >= need:
                break
            ncand += ncand // 8
        self.ncand, self.need = ncand, need
        self.pref = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        self.count = O.ratio_count if kind == "ratio" else O.polar2_count
        self.win = O.ratio_window if kind == "ratio" else O.polar2_window

    def chunk_of(self, a):
        return int(np.searchsorted(self.pref, a, side="right")) - 1

    def window(self, c):
        """Values of chunk c's accepted candidates and the output element
        index of the first."""
        c0 = c * CHUNK
        return self.win(self.seed, self.offset, c0, min(CHUNK, self.ncand - c0)), self.epc * int(self.pref[c])

    def consumed(self):
        """2 (j + 1) for the candidate j that supplies the last needed
        accepted candidate, found by bisection on the oracle's counts."""
        k = self.need - 1
        c = self.chunk_of(k)
        c0 = c * CHUNK
        want = k - int(self.pref[c]) + 1          # accepted candidates needed inside the chunk
        lo, hi = 1, min(CHUNK, self.ncand - c0)   # count(c0, hi) >= want
        while lo < hi:
            mid = (lo + hi) // 2
            if self.count(self.seed, self.offset + 2 * c0, mid) >= want:
                hi = mid
            else:
                lo = mid + 1
        return 2 * (c0 + lo)


@pytest.mark.parametrize("method,seed", [("b1", 1), ("polar", 7)])
def test_full_stream_error_2e30(method, seed, capsys):
    """Every one of the 2^30 values of the B1 (seed 1) and Polar (seed 7)
    streams, in FP32, BF16 and FP16 output, against the oracle's whole
    stream (computed once, in chunks on the host threads), compared chunk by
    chunk at each type's bar; the worst error per type is printed.  The
    three outputs come from three calls with the same arguments, so the
    Polar consumed count is checked for each."""
    d = dev()
    n = 1 << 30
    outs = {}
    for dtype in (nb.NRNG_F32, nb.NRNG_BF16, nb.NRNG_F16):
        out = torch.empty(n, dtype=TDT[dtype], device=d)
        cons = torch.zeros(1, dtype=torch.int64, device=d)
        case(method, NAME[dtype], "single stream, full comparison", n)
        if method == "b1":
            nb.nrng_boxmuller(seed, 0, n, 0.0, 1.0, out, dtype)
        else:
            nb.nrng_polar(seed, 0, n, 0.0, 1.0, out, dtype, None, cons)
        torch.cuda.synchronize()
        outs[dtype] = (out, cons)
    if method == "b1":
        ref, used = O.b1_parallel(seed, 0, n, threads=THREADS), 2 * (n // 2)
    else:
        ref, used = O.polar_parallel(seed, 0, n, threads=THREADS)
        for dtype, (_, cons) in outs.items():
            assert int(u64(cons)[0]) == used, NAME[dtype]
    step = 1 << 26
    report = []
    for dtype, (out, _) in outs.items():
        worst, rel = 0.0, 0.0
        for c0 in range(0, n, step):
            z = host(out[c0:c0 + step])
            r = ref[c0:c0 + step]
            worst = max(worst, assert_close(z, r, dtype, what="%s %s 2^30 full, chunk at %d" % (method, NAME[dtype], c0)))
            rel = max(rel, float(np.max(np.abs(z - r) / np.maximum(1.0, np.abs(r)))))
        report.append("%s max|dz|/max(1,|z|) %.3e, max err/bar %.3f" % (NAME[dtype], rel, worst))
    del ref
    with capsys.disabled():
        print("\n[%s, all 2^30 values] %s" % (method, "; ".join(report)), flush=True)


@pytest.mark.parametrize("kind,seed", [("polar2", 7), ("ratio", 21)])
def test_rejection_single_stream_2e30_sampled(kind, seed):
    """2^30 FP32 normals of method P2 (seed 7) and Algorithm R (seed 21), the
    single streams the benchmark times: whole candidate chunks placed by the
    oracle's own prefix counts (the first, the last and random ones), and the
    consumed count."""
    d = dev()
    n = 1 << 30
    out = torch.empty(n, dtype=torch.float32, device=d)
    cons = torch.zeros(1, dtype=torch.int64, device=d)
    case(kind, "f32 single stream", n)
    f = nb.nrng_polar2 if kind == "polar2" else nb.nrng_ratio
    f(seed, 0, n, 0.0, 1.0, out, nb.NRNG_F32, None, cons)
    torch.cuda.synchronize()
    ix = RejIndex(kind, seed, 0, n)
    assert int(u64(cons)[0]) == ix.consumed()
    last = ix.chunk_of(ix.need - 1)
    chunks = sorted({0, last} | set(synth.rng(35).integers(0, last, 8).tolist()))
    for c in chunks:
        vals, e0 = ix.window(c)
        m = min(vals.size, n - e0)
        got = host(out[e0:e0 + m])
        assert_close(got, vals[:m], nb.NRNG_F32, what="%s 2^30 chunk %d" % (kind, c))


@pytest.mark.parametrize("method", ["b2", "b3"])
def test_box_muller_family_single_stream_2e30_sampled(method):
    """2^30 FP32 normals of methods B2 and B3 (seed 1, as the benchmark),
    at sampled output indices, each from its own pair's counters."""
    d = dev()
    n = 1 << 30
    out = torch.empty(n, dtype=torch.float32, device=d)
    case(method, "f32 single stream", n)
    (nb.nrng_b2 if method == "b2" else nb.nrng_b3)(1, 0, n, 0.0, 1.0, out, nb.NRNG_F32)
    torch.cuda.synchronize()
    idx = np.concatenate([np.arange(64), n - 64 + np.arange(64),
                          synth.rng(36).integers(0, n, 4096)]).astype(np.int64)
    got = host(out[torch.from_numpy(idx).to(d)])
    ref = O.pairs_at(method, 1, 0, idx)
    extra = None
    if method == "b2":
        other = O.pairs_at(method, 1, 0, idx ^ 1)          # the same pair's other value
        extra = 2.0**-19 * np.hypot(ref, other)
    assert_close(got, ref, nb.NRNG_F32, what="%s 2^30 sampled" % method, extra=extra)


def test_b1_single_stream_2e30_sampled():
    d = dev()
    n = 1 << 30
    out = torch.empty(n, dtype=torch.float32, device=d)
    case("b1 f32 single stream", n)
    nb.nrng_boxmuller(1, 0, n, 0.0, 1.0, out, nb.NRNG_F32)
    torch.cuda.synchronize()
    idx = np.concatenate([np.arange(64), n - 64 + np.arange(64),
                          synth.rng(31).integers(0, n, 8192)]).astype(np.int64)
    got = host(out[torch.from_numpy(idx).to(d)])
    assert_close(got, O.b1_at(1, 0, idx), nb.NRNG_F32, what="b1 2^30 sampled")


def test_polar_single_stream_2e30_sampled():
    d = dev()
    n = 1 << 30
    P = n // 2
    out = torch.empty(n, dtype=torch.float32, device=d)
    cons = torch.zeros(1, dtype=torch.int64, device=d)
    case("polar f32 single stream", n)
    nb.nrng_polar(7, 0, n, 0.0, 1.0, out, nb.NRNG_F32, None, cons)
    torch.cuda.synchronize()
    ix = PolarIndex(7, 0, P)
    assert int(u64(cons)[0]) == ix.consumed(P)
    last = ix.chunk_of_pair(P - 1)
    chunks = sorted({0, last} | set(synth.rng(32).integers(0, last, 10).tolist()))
    for c in chunks:
        vals, a0 = ix.window(c)
        m = min(vals.size, n - 2 * a0)
        got = host(out[2 * a0:2 * a0 + m])
        assert_close(got, vals[:m], nb.NRNG_F32, what="polar 2^30 chunk %d" % c)


ORACLE_OF = {nb.NRNG_METHOD_B1: O.b1, nb.NRNG_METHOD_POLAR: O.polar, nb.NRNG_METHOD_P2: O.polar2,
             nb.NRNG_METHOD_B3: O.b3, nb.NRNG_METHOD_R: O.ratio, nb.NRNG_METHOD_B2: O.b2}


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR, nb.NRNG_METHOD_P2, nb.NRNG_METHOD_B3,
                                    nb.NRNG_METHOD_R, nb.NRNG_METHOD_B2])
def test_batched_full_workload(method, capsys):
    """The batched workload the benchmark times (4096 streams, about 4.4e8
    FP32 normals), in full: every value of every stream against the oracle's
    own call for that stream (run on the host threads), and every consumed
    count equal to the oracle's -- for the rejection methods this is the
    exact position of the last accepted candidate in Section 2's stable
    order."""
    d = dev()
    cfg = synth.batched_streams()
    ns, total = len(cfg["n"]), cfg["total"]
    D = {k: torch.from_numpy(cfg[k].view(np.int64) if cfg[k].dtype == np.uint64 else cfg[k]).to(d)
         for k in ("seed", "offset", "n", "mu", "sigma")}
    out = torch.empty(total, dtype=torch.float32, device=d)
    cons = torch.zeros(ns, dtype=torch.int64, device=d)
    nb.nrng_reserve(total, ns)
    case("batched full workload", method, ns, total)
    nb.nrng_batched(method, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out, total,
                    nb.NRNG_F32, None, cons)
    torch.cuda.synchronize()
    c = u64(cons)
    z_all = out.cpu().numpy()
    del out
    n = cfg["n"].astype(np.int64)
    fn = ORACLE_OF[method]

    def one(j):
        o0, nj = int(cfg["out_off"][j]), int(n[j])
        mu, sg, seed = float(cfg["mu"][j]), float(cfg["sigma"][j]), int(cfg["seed"][j])
        ref, used = fn(seed, 0, nj, mu, sg)
        assert int(c[j]) == used, ("consumed", j, int(c[j]), used)
        extra = None
        if method == nb.NRNG_METHOD_B2:
            pairs, _ = O.b2(seed, 0, 2 * ((nj + 1) // 2), mu, sg)
            extra = b2_f32_extra(pairs, mu, nj)
        return assert_close(z_all[o0:o0 + nj].astype(np.float64), ref, nb.NRNG_F32, mu, sg,
                            what="batched stream %d" % j, extra=extra)

    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        worst = max(ex.map(one, range(ns)))
    with capsys.disabled():
        print("\n[batched method %d, all %d streams, %d values] worst error / bar %.3f" % (method, ns, total, worst),
              flush=True)


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR, nb.NRNG_METHOD_P2, nb.NRNG_METHOD_B3,
                                    nb.NRNG_METHOD_R, nb.NRNG_METHOD_B2])
def test_batched_full_workload_half_is_rounded_f32(method):
    """BF16 and FP16 output of the whole batched workload equals the FP32
    output of the same call rounded to nearest even, bit for bit (C15: the
    value is computed in FP32 and rounded once more).  A conversion fused
    with the final FMA into one mixed-precision instruction would round once
    and differ in rare near-tie cases; about 4.4e8 values per method reach
    such cases.  The consumed counts do not depend on the output type."""
    d = dev()
    cfg = synth.batched_streams()
    ns, total = len(cfg["n"]), cfg["total"]
    D = {k: torch.from_numpy(cfg[k].view(np.int64) if cfg[k].dtype == np.uint64 else cfg[k]).to(d)
         for k in ("seed", "offset", "n", "mu", "sigma")}
    nb.nrng_reserve(total, ns)
    out32 = torch.empty(total, dtype=torch.float32, device=d)
    c32 = torch.zeros(ns, dtype=torch.int64, device=d)
    case("batched full workload f32", method, ns, total)
    nb.nrng_batched(method, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out32, total,
                    nb.NRNG_F32, None, c32)
    for dtype in (nb.NRNG_BF16, nb.NRNG_F16):
        out = torch.empty(total, dtype=TDT[dtype], device=d)
        cons = torch.zeros(ns, dtype=torch.int64, device=d)
        case("batched full workload", method, dtype, ns, total)
        nb.nrng_batched(method, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out, total,
                        dtype, None, cons)
        torch.cuda.synchronize()
        want = out32.to(TDT[dtype])
        bad = int((out.view(torch.int16) != want.view(torch.int16)).sum().item())
        assert bad == 0, (NAME[dtype], bad)
        assert torch.equal(cons, c32)
        del out, want


def test_graph_fill_64_x_2e28_sampled():
    d = dev()
    nf, fills = 1 << 28, 64
    slen, per_fill, sampled_fills = 1 << 16, 4, 16
    s = torch.cuda.Stream()
    cursor = torch.zeros(1, dtype=torch.int64, device=d)
    out = torch.empty(nf, dtype=torch.float32, device=d)
    nb.nrng_reserve(nf, 0)
    fsel = set(synth.rng(34).choice(fills, sampled_fills, replace=False).tolist()) | {0, fills - 1}
    starts = {f: synth.slice_starts(per_fill, slen, nf, seed=0x51CE + f) for f in fsel}
    samples = {}
    case("graph fill create", nf)
    g = nb.nrng_fillgraph_create(7, cursor, nf, 0.0, 1.0, out, nb.NRNG_F32, s)
    try:
        for f in range(fills):
            nb.nrng_fillgraph_launch(g, s)
            if f in fsel:
                s.synchronize()
                samples[f] = [host(out[st:st + slen]) for st in starts[f]]
        s.synchronize()
    finally:
        nb.nrng_fillgraph_destroy(g)
    ix = PolarIndex(7, 0, fills * nf // 2)
    assert int(u64(cursor)[0]) == ix.consumed(fills * nf // 2)

    def reference(f, st):
        a = (f * nf + int(st)) // 2            # first output pair of the slice
        b = a + slen // 2
        ref = []
        c = ix.chunk_of_pair(a)
        while True:
            vals, a0 = ix.window(c)
            lo, hi = max(a, a0), min(b, a0 + vals.size // 2)
            if hi > lo:
                ref.append(vals[2 * (lo - a0):2 * (hi - a0)])
            if a0 + vals.size // 2 >= b:
                return np.concatenate(ref)
            c += 1

    jobs = [(f, st, got) for f in sorted(samples) for st, got in zip(starts[f], samples[f])]
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        refs = list(ex.map(lambda j: reference(j[0], j[1]), jobs))
    allv = []
    for (f, st, got), ref in zip(jobs, refs):
        assert_close(got, ref, nb.NRNG_F32, what="fill %d slice at %d" % (f, st))
        allv.append(got)
    z = np.concatenate(allv)
    bd = stat_bounds(z.size)
    m = O.moments(z)
    assert abs(m[0]) < bd["mean"] and abs(m[1] - 1) < bd["var"]
    assert abs(m[2]) < bd["skew"] and abs(m[3] - 3) < bd["kurt"]
    assert O.ks_normal(z) < bd["ks"]
