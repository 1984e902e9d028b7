"""Batched streams in one persistent launch, and repeated fills through a
HIP graph with a device-resident counter offset, against single-stream
calls (bit-exact) and the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_util import NAME, TDT, assert_close, case, dev, host, run, u64
from paper_1004_3105_amd import binding as nb

pytestmark = pytest.mark.gpu

U64MAX = (1 << 64) - 1


def to_dev(cfg, d):
    return {
        "seed": torch.from_numpy(cfg["seed"].view(np.int64)).to(d),
        "offset": torch.from_numpy(cfg["offset"].view(np.int64)).to(d),
        "n": torch.from_numpy(cfg["n"].view(np.int64)).to(d),
        "mu": torch.from_numpy(cfg["mu"]).to(d),
        "sigma": torch.from_numpy(cfg["sigma"]).to(d),
    }


def small_config(nstreams=97):
    cfg = synth.batched_streams(nstreams=nstreams, seed=0x5EED, n_lo=1, n_hi=2e4)
    cfg["n"][3] = 0          # an empty stream
    cfg["n"][5] = 1          # a single value
    cfg["offset"] = synth.rng(3).integers(0, 1 << 40, nstreams, dtype=np.uint64)
    cfg["out_off"] = np.concatenate([[0], np.cumsum(cfg["n"][:-1])]).astype(np.uint64)
    cfg["total"] = int(cfg["n"].sum())
    return cfg


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR])
@pytest.mark.parametrize("dtype", [nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_BF16, nb.NRNG_F16])
def test_batched_packed_matches_single_streams(method, dtype):
    d = dev()
    cfg = small_config()
    D = to_dev(cfg, d)
    out = torch.full((cfg["total"],), float("nan"), dtype=TDT[dtype], device=d)
    cons = torch.zeros(len(cfg["n"]), dtype=torch.int64, device=d)
    case("batched packed", method, dtype, len(cfg["n"]), cfg["total"])
    nb.nrng_batched(method, len(cfg["n"]), D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out,
                    cfg["total"], dtype, None, cons)
    torch.cuda.synchronize()
    c = u64(cons)
    name = "b1" if method == nb.NRNG_METHOD_B1 else "polar"
    for j in range(len(cfg["n"])):
        n = int(cfg["n"][j])
        o0 = int(cfg["out_off"][j])
        seg = out[o0:o0 + n]
        single, used = run(name, int(cfg["seed"][j]), int(cfg["offset"][j]), n, dtype, float(cfg["mu"][j]),
                           float(cfg["sigma"][j]), with_consumed=True)
        assert torch.equal(seg, single), j
        if name == "b1":
            assert c[j] == 2 * ((n + 1) // 2)
        elif n > 0:
            assert c[j] == used, j
        else:
            assert c[j] == 0
        if j % 8 == 0 and n > 0:
            fn = O.b1 if name == "b1" else O.polar
            ref, uref = fn(int(cfg["seed"][j]), int(cfg["offset"][j]), n, float(cfg["mu"][j]),
                           float(cfg["sigma"][j]))
            assert c[j] == uref
            assert_close(host(seg), ref, dtype, float(cfg["mu"][j]), float(cfg["sigma"][j]),
                         what="batched stream %d" % j)


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR, nb.NRNG_METHOD_R])
def test_batched_many_streams_across_setup_chunks(method):
    """8315 streams: the set-up kernel takes streams in chunks of 4096 and
    carries both prefixes (packed output offsets and the tile table) from
    chunk to chunk.  The packed call equals the same call with explicit
    offsets element for element, and the streams at the chunk boundaries,
    plus a random sample, equal single-stream calls bit for bit, consumed
    counts included."""
    d = dev()
    ns = 2 * 4096 + 123
    cfg = synth.batched_streams(nstreams=ns, seed=0xC4A1, n_lo=1, n_hi=600)
    cfg["n"][[4095, 8192]] = 0          # empty streams on both sides of a chunk boundary
    cfg["out_off"] = np.concatenate([[0], np.cumsum(cfg["n"][:-1])]).astype(np.uint64)
    total = int(cfg["n"].sum())
    D = to_dev(cfg, d)
    res = []
    for packed in (True, False):
        out = torch.full((total,), float("nan"), dtype=torch.float32, device=d)
        cons = torch.zeros(ns, dtype=torch.int64, device=d)
        off = None if packed else torch.from_numpy(cfg["out_off"].view(np.int64)).to(d)
        case("batched across set-up chunks", method, "packed", packed, ns, total)
        nb.nrng_batched(method, ns, D["seed"], D["offset"], D["n"], off, D["mu"], D["sigma"], out, total,
                        nb.NRNG_F32, None, cons)
        torch.cuda.synchronize()
        res.append((out, u64(cons)))
    (out, c), (out_x, c_x) = res
    assert not torch.isnan(out).any()
    assert torch.equal(out, out_x)
    assert np.array_equal(c, c_x)
    name = {nb.NRNG_METHOD_B1: "b1", nb.NRNG_METHOD_POLAR: "polar", nb.NRNG_METHOD_R: "ratio"}[method]
    edges = [0, 1, 4094, 4095, 4096, 4097, 8191, 8192, 8193, ns - 1]
    sample = sorted(set(edges) | set(int(j) for j in synth.rng(17).integers(0, ns, 24)))
    for j in sample:
        n = int(cfg["n"][j])
        o0 = int(cfg["out_off"][j])
        single, used = run(name, int(cfg["seed"][j]), int(cfg["offset"][j]), n, nb.NRNG_F32,
                           float(cfg["mu"][j]), float(cfg["sigma"][j]), with_consumed=True)
        assert torch.equal(out[o0:o0 + n], single), j
        if name == "b1":
            assert c[j] == 2 * ((n + 1) // 2), j
        else:
            assert c[j] == (used if n > 0 else 0), j


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR])
def test_batched_explicit_offsets_and_invalid_streams(method):
    d = dev()
    cfg = small_config(33)
    n = cfg["n"]
    # gaps of 0..3 elements between streams, so starts have every alignment
    gaps = synth.rng(9).integers(0, 4, len(n)).astype(np.uint64)
    off = np.zeros(len(n), dtype=np.uint64)
    pos = 0
    for j in range(len(n)):
        pos += int(gaps[j])
        off[j] = pos
        pos += int(n[j])
    out_len = pos
    # stream 7 now points past the end of the buffer: it must be skipped
    off[7] = out_len - int(n[7]) + 1 if n[7] > 0 else out_len + 1
    D = to_dev(cfg, d)
    doff = torch.from_numpy(off.view(np.int64)).to(d)
    out = torch.full((out_len,), -777.0, dtype=torch.float32, device=d)
    cons = torch.zeros(len(n), dtype=torch.int64, device=d)
    case("batched explicit offsets", method)
    nb.nrng_batched(method, len(n), D["seed"], D["offset"], D["n"], doff, D["mu"], D["sigma"], out, out_len,
                    nb.NRNG_F32, None, cons)
    torch.cuda.synchronize()
    c = u64(cons)
    assert c[7] == U64MAX
    name = "b1" if method == nb.NRNG_METHOD_B1 else "polar"
    written = torch.zeros(out_len, dtype=torch.bool, device=d)
    for j in range(len(n)):
        if j == 7:
            continue
        o0, nj = int(off[j]), int(n[j])
        single = run(name, int(cfg["seed"][j]), int(cfg["offset"][j]), nj, nb.NRNG_F32, float(cfg["mu"][j]),
                     float(cfg["sigma"][j]))
        assert torch.equal(out[o0:o0 + nj], single), j
        written[o0:o0 + nj] = True
    # gaps and the skipped stream's range are untouched (except where a
    # valid stream overlaps them)
    assert torch.all(out[~written] == -777.0)


def test_batched_overflowing_total_is_rejected_on_device():
    d = dev()
    cfg = small_config(16)
    D = to_dev(cfg, d)
    total = cfg["total"]
    out_len = total - 1 - int(cfg["n"][-1]) // 2
    out = torch.zeros(max(out_len, 1), dtype=torch.float32, device=d)
    cons = torch.zeros(16, dtype=torch.int64, device=d)
    case("batched packed overflow")
    nb.nrng_batched(nb.NRNG_METHOD_POLAR, 16, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out,
                    out_len, nb.NRNG_F32, None, cons)
    torch.cuda.synchronize()
    c = u64(cons)
    # packed layout: the streams that fit are produced, the last one is skipped
    assert c[-1] == U64MAX
    assert all(x != U64MAX for x in c[:-1])


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR])
def test_batched_huge_length_inside_a_setup_group(method):
    """A packed batch whose sixth stream has n = 2^64 - 1: the set-up kernel
    sums the lengths of four consecutive streams per thread, so the packed
    prefix saturates inside the group of streams 4..7.  Streams 0..4 keep
    their exact offsets (0, 10, 30, 35, 42) and equal single-stream calls bit
    for bit; the huge stream and every stream after it (whose packed offsets
    saturate) are skipped, and nothing beyond the valid ranges is written."""
    d = dev()
    lens = np.array([10, 20, 5, 7, 3, U64MAX, 4, 6, 9, 1], dtype=np.uint64)
    ns = len(lens)
    cfg = {"n": lens, "seed": (np.arange(ns, dtype=np.uint64) * 7919 + 5).astype(np.uint64),
           "offset": np.zeros(ns, dtype=np.uint64), "mu": np.linspace(-1.0, 1.0, ns),
           "sigma": np.linspace(0.5, 2.0, ns)}
    D = to_dev(cfg, d)
    out_len = 64
    out = torch.full((out_len,), -777.0, dtype=torch.float32, device=d)
    cons = torch.zeros(ns, dtype=torch.int64, device=d)
    case("batched huge length", method)
    nb.nrng_batched(method, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out, out_len,
                    nb.NRNG_F32, None, cons)
    torch.cuda.synchronize()
    c = u64(cons)
    name = "b1" if method == nb.NRNG_METHOD_B1 else "polar"
    starts = [0, 10, 30, 35, 42]
    for j, o0 in enumerate(starts):
        nj = int(lens[j])
        single, used = run(name, int(cfg["seed"][j]), 0, nj, nb.NRNG_F32, float(cfg["mu"][j]),
                           float(cfg["sigma"][j]), with_consumed=True)
        assert torch.equal(out[o0:o0 + nj], single), j
        assert c[j] == (2 * ((nj + 1) // 2) if name == "b1" else used), j
    assert all(c[j] == U64MAX for j in range(5, ns))
    assert torch.all(out[45:] == -777.0)


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR])
def test_batched_overlapping_total_is_rejected_on_device(method):
    """Explicit offsets that place four valid streams of 100 over one buffer
    of 150: each range fits, but their lengths total 400 > out_len, so the
    set-up kernel fails the whole call (every consumed count UINT64_MAX,
    nothing written)."""
    d = dev()
    ns = 4
    cfg = {"n": np.full(ns, 100, dtype=np.uint64), "seed": np.arange(1, ns + 1, dtype=np.uint64),
           "offset": np.zeros(ns, dtype=np.uint64), "mu": np.zeros(ns), "sigma": np.ones(ns)}
    D = to_dev(cfg, d)
    off = torch.from_numpy(np.array([0, 50, 25, 0], dtype=np.int64)).to(d)
    out = torch.full((150,), -777.0, dtype=torch.float32, device=d)
    cons = torch.zeros(ns, dtype=torch.int64, device=d)
    case("batched overlapping total", method)
    nb.nrng_batched(method, ns, D["seed"], D["offset"], D["n"], off, D["mu"], D["sigma"], out, 150,
                    nb.NRNG_F32, None, cons)
    torch.cuda.synchronize()
    assert all(x == U64MAX for x in u64(cons))
    assert torch.all(out == -777.0)


def test_fillgraph_repeated_fills_continue_one_stream():
    d = dev()
    n = (1 << 20) + 5
    s = torch.cuda.Stream()
    cursor = torch.zeros(1, dtype=torch.int64, device=d)
    out = torch.empty(n, dtype=torch.float32, device=d)
    nb.nrng_reserve(n, 0)
    case("fillgraph create", n)
    g = nb.nrng_fillgraph_create(7, cursor, n, 0.0, 1.0, out, nb.NRNG_F32, s)
    try:
        off = 0
        for f in range(6):
            case("fillgraph replay", f)
            nb.nrng_fillgraph_launch(g, s)
            s.synchronize()
            ref, used = O.polar(7, off, n)
            off += used
            assert int(cursor.item()) == off, f
            assert_close(host(out), ref, nb.NRNG_F32, what="fill %d" % f)
            # eager work between replays
            torch.cuda.synchronize()
            x = torch.randn(1000, device=d).sum()
            torch.cuda.synchronize()
            del x
    finally:
        nb.nrng_fillgraph_destroy(g)


def test_polar_dev_under_torch_graph_capture():
    d = dev()
    n = 50001
    cursor = torch.zeros(1, dtype=torch.int64, device=d)
    out = torch.empty(n, dtype=torch.float64, device=d)
    nb.nrng_reserve(n, 0)
    # warm-up call outside capture (library state initialised)
    nb.nrng_polar_dev(3, cursor, n, 0.0, 1.0, out, nb.NRNG_F64)
    torch.cuda.synchronize()
    off = int(cursor.item())
    g = torch.cuda.CUDAGraph()
    case("torch graph capture nrng_polar_dev")
    with torch.cuda.graph(g):
        nb.nrng_polar_dev(3, cursor, n, 0.0, 1.0, out, nb.NRNG_F64)
    for r in range(4):
        case("torch graph replay", r)
        g.replay()
        torch.cuda.synchronize()
        ref, used = O.polar(3, off, n)
        off += used
        assert int(cursor.item()) == off
        assert_close(host(out), ref, nb.NRNG_F64, what="replay %d" % r)
        y = torch.ones(10, device=d) * r
        torch.cuda.synchronize()
        del y


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR, nb.NRNG_METHOD_P2,
                                    nb.NRNG_METHOD_B3, nb.NRNG_METHOD_R, nb.NRNG_METHOD_B2])
def test_exec_parts_equal_exec(method):
    """The count half then the generate half of the exec sequence, and the
    exec whose main kernel is timed by two events (the timing hooks, whole
    or as the generate half after the count half), give exactly what exec
    gives; the events bracket a positive time no longer than the whole
    exec's; a part outside 0..2 is an argument error."""
    d = dev()
    cfg = small_config(61)
    D = to_dev(cfg, d)
    ns = len(cfg["n"])
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    for e in evs:
        e.record(stream)   # torch creates its events on their first record
    outs = []
    for parts in ((0,), (1, 2), (1, "timed2"), ("timed",)):
        out = torch.full((cfg["total"],), float("nan"), dtype=torch.float32, device=d)
        cons = torch.zeros(ns, dtype=torch.int64, device=d)
        case("exec parts", method, parts)
        nb.nrng_batched_plan(method, ns, D["n"], None, cfg["total"], nb.NRNG_F32, None, cons)
        for p in parts:
            if p == "timed":
                evs[0].record(stream)
                nb.nrng_batched_exec_timed(0, method, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"],
                                           out, nb.NRNG_F32, stream, cons, evs[1], evs[2])
                evs[3].record(stream)
            elif p == "timed2":
                nb.nrng_batched_exec_timed(2, method, ns, D["seed"], D["offset"], D["n"], None, D["mu"],
                                           D["sigma"], out, nb.NRNG_F32, stream, cons, evs[4], evs[5])
            else:
                nb.nrng_batched_exec_part(p, method, ns, D["seed"], D["offset"], D["n"], None, D["mu"],
                                          D["sigma"], out, nb.NRNG_F32, None, cons)
        torch.cuda.synchronize()
        outs.append((out, u64(cons)))
    for o in outs[1:]:
        assert torch.equal(outs[0][0], o[0])
        assert np.array_equal(outs[0][1], o[1])
    kernel_ms, exec_ms = evs[1].elapsed_time(evs[2]), evs[0].elapsed_time(evs[3])
    assert 0.0 < kernel_ms <= exec_ms, (kernel_ms, exec_ms)
    assert evs[4].elapsed_time(evs[5]) > 0.0
    with pytest.raises(nb.NrngError):
        nb.nrng_batched_exec_part(3, method, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"],
                                  outs[0][0], nb.NRNG_F32, None, None)


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR, nb.NRNG_METHOD_P2,
                                    nb.NRNG_METHOD_B3, nb.NRNG_METHOD_R, nb.NRNG_METHOD_B2])
def test_batched_plan_and_exec_under_torch_graph_capture(method):
    """A whole batched call (plan + exec) captured once in a HIP graph (torch's
    graph API) and replayed three times, with eager work between the replays
    and the outputs cleared before each: every replay equals the eager call
    bit for bit, consumed counts included."""
    d = dev()
    cfg = small_config(97)
    D = to_dev(cfg, d)
    ns, total = len(cfg["n"]), cfg["total"]
    nb.nrng_reserve(total, ns)
    out = torch.empty(total, dtype=torch.float32, device=d)
    cons = torch.zeros(ns, dtype=torch.int64, device=d)
    case("batched eager before capture", method)
    nb.nrng_batched(method, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out, total,
                    nb.NRNG_F32, None, cons)
    torch.cuda.synchronize()
    ref, ref_cons = out.clone(), cons.clone()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    case("batched capture", method)
    with torch.cuda.graph(g, stream=s):
        nb.nrng_batched(method, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out, total,
                        nb.NRNG_F32, s, cons)
    for r in range(3):
        out.fill_(float("nan"))
        cons.zero_()
        torch.cuda.synchronize()
        case("batched replay", method, r)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), r
        assert torch.equal(cons, ref_cons), r
        y = torch.ones(1 << 16, device=d).sum()           # eager work between replays
        torch.cuda.synchronize()
        del y


@pytest.mark.parametrize("method", [nb.NRNG_METHOD_B1, nb.NRNG_METHOD_B3, nb.NRNG_METHOD_B2])
@pytest.mark.parametrize("dtype", [nb.NRNG_F64, nb.NRNG_F32, nb.NRNG_BF16, nb.NRNG_F16])
def test_batched_box_muller_every_place_in_a_line(method, dtype):
    """The batched Box-Muller family starts each stream's passes on a
    128-byte line of the output (its first segment begins up to a line
    before the stream and stores nothing there).  Streams whose first
    element takes every place in a line, with lengths around the pass and
    segment sizes, equal the single-stream calls bit for bit, and nothing
    outside the streams is written (gaps of 1 to 3 elements stay as they
    were)."""
    d = dev()
    esize = {nb.NRNG_F64: 8, nb.NRNG_F32: 4, nb.NRNG_BF16: 2, nb.NRNG_F16: 2}[dtype]
    line = 128 // esize
    lens = [1, 2, 3, 5, 31, 33, 64, 255, 257, 1023, 1025, 2049, 4095, 4097, 9001]
    ns = 2 * line
    r = synth.rng(31)
    n = np.array([lens[j % len(lens)] for j in range(ns)], dtype=np.uint64)
    off = np.zeros(ns, dtype=np.uint64)
    pos = 0
    for j in range(ns):
        # stream j starts at place j mod line of a line (the buffer is line-aligned)
        pos += (j % line - pos) % line or line
        off[j] = pos
        pos += int(n[j]) + int(r.integers(1, 4))
    out_len = pos
    seeds = r.integers(0, 1 << 63, ns, dtype=np.uint64)
    offs = r.integers(0, 1 << 40, ns, dtype=np.uint64)
    mus = r.uniform(-3.0, 3.0, ns)
    sigmas = r.uniform(0.5, 2.0, ns)
    D = {"seed": torch.from_numpy(seeds.view(np.int64)).to(d), "offset": torch.from_numpy(offs.view(np.int64)).to(d),
         "n": torch.from_numpy(n.view(np.int64)).to(d), "mu": torch.from_numpy(mus).to(d),
         "sigma": torch.from_numpy(sigmas).to(d), "off": torch.from_numpy(off.view(np.int64)).to(d)}
    out = torch.full((out_len,), -512.0, dtype=TDT[dtype], device=d)
    assert out.data_ptr() % 128 == 0
    cons = torch.zeros(ns, dtype=torch.int64, device=d)
    case("batched Box-Muller line places", method, NAME[dtype])
    nb.nrng_batched(method, ns, D["seed"], D["offset"], D["n"], D["off"], D["mu"], D["sigma"], out, out_len, dtype,
                    None, cons)
    torch.cuda.synchronize()
    name = {nb.NRNG_METHOD_B1: "b1", nb.NRNG_METHOD_B3: "b3", nb.NRNG_METHOD_B2: "b2"}[method]
    written = torch.zeros(out_len, dtype=torch.bool, device=d)
    for j in range(ns):
        o0, nj = int(off[j]), int(n[j])
        single = run(name, int(seeds[j]), int(offs[j]), nj, dtype, float(mus[j]), float(sigmas[j]))
        assert torch.equal(out[o0:o0 + nj], single), (j, o0 % line, nj)
        written[o0:o0 + nj] = True
    assert torch.all(out[~written] == -512.0)


@pytest.mark.parametrize("pair", [(nb.NRNG_METHOD_B1, nb.NRNG_METHOD_POLAR), (nb.NRNG_METHOD_B3, nb.NRNG_METHOD_R),
                                  (nb.NRNG_METHOD_B2, nb.NRNG_METHOD_P2)])
def test_two_families_planned_together_and_run_side_by_side(pair):
    """The Box-Muller family and the rejection family keep separate batched
    tables: both plans are made first, then the two execs run at the same
    time on two streams (the rejection exec split in its two parts around a
    join, as the benchmark does); every output and consumed count equals the
    calls made one after the other on one stream."""
    d = dev()
    cfg = small_config(211)
    D = to_dev(cfg, d)
    ns, total = len(cfg["n"]), cfg["total"]
    nb.nrng_reserve(total, ns)
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    ref = {}
    for m in pair:
        out = torch.full((total,), float("nan"), dtype=torch.float32, device=d)
        cons = torch.zeros(ns, dtype=torch.int64, device=d)
        case("family reference", m)
        nb.nrng_batched(m, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], out, total, nb.NRNG_F32,
                        main, cons)
        torch.cuda.synchronize()
        ref[m] = (out, u64(cons))
    bm, rj = pair
    got = {m: (torch.full((total,), float("nan"), dtype=torch.float32, device=d),
               torch.zeros(ns, dtype=torch.int64, device=d)) for m in pair}
    for rep in range(3):
        case("families side by side", pair, rep)
        fork, join = torch.cuda.Event(), torch.cuda.Event()
        fork.record(main)
        side.wait_event(fork)
        nb.nrng_batched_plan(bm, ns, D["n"], None, total, nb.NRNG_F32, main, got[bm][1])
        nb.nrng_batched_plan(rj, ns, D["n"], None, total, nb.NRNG_F32, side, got[rj][1])
        nb.nrng_batched_exec(bm, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], got[bm][0],
                             nb.NRNG_F32, main, got[bm][1])
        nb.nrng_batched_exec_part(1, rj, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], got[rj][0],
                                  nb.NRNG_F32, side, got[rj][1])
        join.record(side)
        main.wait_event(join)
        nb.nrng_batched_exec_part(2, rj, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], got[rj][0],
                                  nb.NRNG_F32, main, got[rj][1])
        torch.cuda.synchronize()
        for m in pair:
            assert torch.equal(got[m][0], ref[m][0]), (m, rep)
            assert np.array_equal(u64(got[m][1]), ref[m][1]), (m, rep)
    # a plan of one family leaves the other family's plan in place
    nb.nrng_batched_plan(rj, ns, D["n"], None, total, nb.NRNG_F32, main, got[rj][1])
    nb.nrng_batched_plan(bm, ns, D["n"], None, total, nb.NRNG_F32, main, got[bm][1])
    nb.nrng_batched_exec(rj, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], got[rj][0],
                         nb.NRNG_F32, main, got[rj][1])
    torch.cuda.synchronize()
    assert torch.equal(got[rj][0], ref[rj][0])


def test_exec_needs_the_matching_plan_of_its_family():
    """exec runs over the latest plan of its method's family and returns
    NRNG_EINVAL, before any launch, unless that plan was made for the same
    method, stream count, dtype and layout; a plan of the other family
    leaves it in place."""
    d = dev()
    cfg = small_config(37)
    D = to_dev(cfg, d)
    ns, total = len(cfg["n"]), cfg["total"]
    off = torch.from_numpy(cfg["out_off"].view(np.int64)).to(d)
    out = torch.full((total,), float("nan"), dtype=torch.float32, device=d)
    out64 = torch.full((total,), float("nan"), dtype=torch.float64, device=d)
    cons = torch.zeros(ns, dtype=torch.int64, device=d)

    def exec_status(method, nstreams=ns, d_out_off=None, o=out, dtype=nb.NRNG_F32):
        try:
            nb.nrng_batched_exec(method, nstreams, D["seed"], D["offset"], D["n"], d_out_off, D["mu"], D["sigma"],
                                 o, dtype, None, cons)
        except nb.NrngError as e:
            return e.status
        return nb.NRNG_OK

    case("plan of the family", "B1 then B3")
    nb.nrng_batched_plan(nb.NRNG_METHOD_B1, ns, D["n"], None, total, nb.NRNG_F32, None, cons)
    nb.nrng_batched_plan(nb.NRNG_METHOD_B3, ns, D["n"], None, total, nb.NRNG_F32, None, cons)
    assert exec_status(nb.NRNG_METHOD_B1) == nb.NRNG_EINVAL
    assert exec_status(nb.NRNG_METHOD_B3) == nb.NRNG_OK
    case("plan of the family", "Polar: stream count, dtype, layout")
    nb.nrng_batched_plan(nb.NRNG_METHOD_POLAR, ns, D["n"], None, total, nb.NRNG_F32, None, cons)
    assert exec_status(nb.NRNG_METHOD_P2) == nb.NRNG_EINVAL
    assert exec_status(nb.NRNG_METHOD_POLAR, nstreams=ns - 1) == nb.NRNG_EINVAL
    assert exec_status(nb.NRNG_METHOD_POLAR, o=out64, dtype=nb.NRNG_F64) == nb.NRNG_EINVAL
    assert exec_status(nb.NRNG_METHOD_POLAR, d_out_off=off) == nb.NRNG_EINVAL
    case("plan of the family", "B2 plan leaves the Polar plan")
    nb.nrng_batched_plan(nb.NRNG_METHOD_B2, ns, D["n"], None, total, nb.NRNG_F32, None, cons)
    assert exec_status(nb.NRNG_METHOD_POLAR) == nb.NRNG_OK
    torch.cuda.synchronize()
    ref = torch.full((total,), float("nan"), dtype=torch.float32, device=d)
    ref_cons = torch.zeros(ns, dtype=torch.int64, device=d)
    nb.nrng_batched(nb.NRNG_METHOD_POLAR, ns, D["seed"], D["offset"], D["n"], None, D["mu"], D["sigma"], ref, total,
                    nb.NRNG_F32, None, ref_cons)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert np.array_equal(u64(cons), u64(ref_cons))
