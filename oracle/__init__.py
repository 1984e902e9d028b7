"""FP64 CPU oracle for the normal-deviate path (TEST INFRASTRUCTURE ONLY).

This package wraps ``nrng_oracle.c`` -- a plain single-threaded C99
implementation, in IEEE double precision without fused multiply-add, of
Box-Muller Algorithm B1 and the Polar method (Algorithm P) from Section 2 of
Brent's "Fast Normal Random Number Generators for Vector Processors" (1993),
methods B2 and B3 of its Section 3, method P2 of its Section 4 and Algorithm R of
its Section 5, fed by a counter-based SplitMix64 uniform stream.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  The product library (``paper_1004_3105_amd``)
never imports, links or calls it, and this package imports nothing from the
product.  The helpers below only marshal arguments and split long ranges into
independent chunks (each chunk is one call of the C reference); they do no
arithmetic of the method themselves.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nrng_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libnrng_oracle.so")
_lock = threading.Lock()
_lib = None

u64 = ctypes.c_uint64
i32 = ctypes.c_int32
f64 = ctypes.c_double
vp = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no contraction into FMA)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB_PATH)
            sig = {
                "orc_splitmix64": (u64, [u64]),
                "orc_uniform": (f64, [u64, u64]),
                "orc_int32": (i32, [u64, u64]),
                "orc_hash_block": (None, [u64, u64, u64, vp]),
                "orc_uniform_block": (None, [u64, u64, u64, vp]),
                "orc_int32_block": (None, [u64, u64, u64, vp]),
                "orc_b1_uv": (None, [vp, vp, u64, f64, f64, vp]),
                "orc_b1_words": (None, [vp, u64, f64, f64, vp]),
                "orc_b1": (u64, [u64, u64, u64, f64, f64, vp]),
                "orc_polar_accept": (ctypes.c_int, [i32, i32]),
                "orc_polar_xy": (u64, [vp, u64, f64, f64, vp, vp]),
                "orc_polar": (u64, [u64, u64, u64, f64, f64, vp]),
                "orc_polar_count": (u64, [u64, u64, u64]),
                "orc_polar_trace": (u64, [u64, u64, u64, vp, vp]),
                "orc_polar_window": (u64, [u64, u64, u64, u64, f64, f64, vp]),
                "orc_p2_cheb": (None, [ctypes.c_int, vp]),
                "orc_p2_h": (f64, [ctypes.c_int, f64]),
                "orc_polar2_accept": (ctypes.c_int, [i32, i32]),
                "orc_polar2_xy": (u64, [vp, u64, f64, f64, vp, vp]),
                "orc_polar2": (u64, [u64, u64, u64, f64, f64, vp]),
                "orc_polar2_count": (u64, [u64, u64, u64]),
                "orc_polar2_window": (u64, [u64, u64, u64, u64, f64, f64, vp]),
                "orc_b2_coef": (None, [vp, vp]),
                "orc_b2_sincos": (None, [f64, vp, vp]),
                "orc_b2_uv": (None, [vp, vp, u64, f64, f64, vp]),
                "orc_b2_words": (None, [vp, u64, f64, f64, vp]),
                "orc_b2": (u64, [u64, u64, u64, f64, f64, vp]),
                "orc_b3_u": (None, [vp, vp, vp, u64, f64, f64, vp]),
                "orc_b3_words": (None, [vp, u64, f64, f64, vp]),
                "orc_b3": (u64, [u64, u64, u64, f64, f64, vp]),
                "orc_ratio_accept": (ctypes.c_int, [f64, f64]),
                "orc_ratio_words": (u64, [vp, u64, f64, f64, vp, vp]),
                "orc_ratio": (u64, [u64, u64, u64, f64, f64, vp]),
                "orc_ratio_count": (u64, [u64, u64, u64]),
                "orc_ratio_trace": (u64, [u64, u64, u64, vp, vp]),
                "orc_ratio_window": (u64, [u64, u64, u64, u64, f64, f64, vp]),
                "orc_moments": (None, [vp, u64, vp]),
                "orc_normal_cdf": (f64, [f64]),
                "orc_ks": (f64, [vp, u64, ctypes.c_int, f64, f64]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(vp)


M64 = (1 << 64) - 1


# ---------------------------------------------------------------- uniforms
def splitmix64(x: int) -> int:
    return int(lib().orc_splitmix64(x & M64))


def hashes(seed: int, offset: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    lib().orc_hash_block(seed & M64, offset & M64, count, _p(out))
    return out


def uniforms(seed: int, offset: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    lib().orc_uniform_block(seed & M64, offset & M64, count, _p(out))
    return out


def int32s(seed: int, offset: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.int32)
    lib().orc_int32_block(seed & M64, offset & M64, count, _p(out))
    return out


# ---------------------------------------------------------------- B1
def b1(seed: int, offset: int, n: int, mu: float = 0.0, sigma: float = 1.0):
    """n normals by Algorithm B1; returns (values, uniforms consumed)."""
    out = np.empty(max(n, 1), dtype=np.float64)
    used = lib().orc_b1(seed & M64, offset & M64, n, mu, sigma, _p(out))
    return out[:n], int(used)


def b1_uv(u, v, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert u.shape == v.shape
    out = np.empty(2 * u.size, dtype=np.float64)
    lib().orc_b1_uv(_p(u), _p(v), u.size, mu, sigma, _p(out))
    return out


def b1_words(words, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint64)
    assert w.size % 2 == 0
    out = np.empty(w.size, dtype=np.float64)
    lib().orc_b1_words(_p(w), w.size // 2, mu, sigma, _p(out))
    return out


def b1_at(seed: int, offset: int, index: np.ndarray, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    """Values at the given output indices of a B1 stream (each index k is
    computed on its own from pair k // 2)."""
    index = np.asarray(index, dtype=np.int64)
    out = np.empty(index.size, dtype=np.float64)
    pair = np.empty(2, dtype=np.float64)
    L = lib()
    for t, k in enumerate(index.tolist()):
        L.orc_b1((seed) & M64, (offset + 2 * (k // 2)) & M64, 2, mu, sigma, _p(pair))
        out[t] = pair[k % 2]
    return out


def pairs_at(method: str, seed: int, offset: int, index: np.ndarray, mu: float = 0.0,
             sigma: float = 1.0) -> np.ndarray:
    """Values at the given output indices of a stream of a Box-Muller-family
    method ("b1", "b2" or "b3"; pair k uses uniforms upp k .. upp k + upp - 1,
    upp = 2, 2, 3), each index computed on its own from its pair."""
    index = np.asarray(index, dtype=np.int64)
    out = np.empty(index.size, dtype=np.float64)
    pair = np.empty(2, dtype=np.float64)
    L = lib()
    fn, upp = {"b1": (L.orc_b1, 2), "b2": (L.orc_b2, 2), "b3": (L.orc_b3, 3)}[method]
    for t, k in enumerate(index.tolist()):
        fn(seed & M64, (offset + upp * (k // 2)) & M64, 2, mu, sigma, _p(pair))
        out[t] = pair[k % 2]
    return out


def b1_parallel(seed: int, offset: int, n: int, mu: float = 0.0, sigma: float = 1.0,
                threads: int | None = None, chunk_pairs: int = 1 << 20) -> np.ndarray:
    """Algorithm B1 over a long stream, split into independent chunks of whole
    pairs, each computed by one call of the reference."""
    out = np.empty(n, dtype=np.float64)
    npairs = (n + 1) // 2
    L = lib()

    def work(c0):
        c1 = min(npairs, c0 + chunk_pairs)
        m = min(n, 2 * c1) - 2 * c0
        buf = out[2 * c0: 2 * c0 + m]
        L.orc_b1(seed & M64, (offset + 2 * c0) & M64, m, mu, sigma, _p(buf))

    with ThreadPoolExecutor(max_workers=threads or os.cpu_count()) as ex:
        list(ex.map(work, range(0, npairs, chunk_pairs)))
    return out


# ---------------------------------------------------------------- Polar
def polar(seed: int, offset: int, n: int, mu: float = 0.0, sigma: float = 1.0):
    """n normals by Algorithm P; returns (values, uniforms consumed)."""
    out = np.empty(max(n, 1), dtype=np.float64)
    used = lib().orc_polar(seed & M64, offset & M64, n, mu, sigma, _p(out))
    return out[:n], int(used)


def polar_xy(xy, mu: float = 0.0, sigma: float = 1.0):
    """Algorithm P on explicit integer candidates xy[j] = (X_j, Y_j).
    Returns (compacted values, mask words, number accepted)."""
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1)
    ncand = xy.size // 2
    out = np.empty(max(2 * ncand, 1), dtype=np.float64)
    masks = np.empty(max((ncand + 63) // 64, 1), dtype=np.uint64)
    a = int(lib().orc_polar_xy(_p(xy), ncand, mu, sigma, _p(out), _p(masks)))
    return out[:2 * a], masks[:(ncand + 63) // 64], a


def polar_accept(X: int, Y: int) -> bool:
    return bool(lib().orc_polar_accept(int(X), int(Y)))


def polar_count(seed: int, offset: int, ncand: int) -> int:
    return int(lib().orc_polar_count(seed & M64, offset & M64, ncand))


def polar_trace(seed: int, offset: int, ncand: int):
    nw = (ncand + 63) // 64
    masks = np.empty(max(nw, 1), dtype=np.uint64)
    pref = np.empty(max(nw, 1), dtype=np.uint64)
    a = int(lib().orc_polar_trace(seed & M64, offset & M64, ncand, _p(masks), _p(pref)))
    return masks[:nw], pref[:nw], a


def polar_window(seed: int, offset: int, j0: int, ncand: int, mu: float = 0.0, sigma: float = 1.0):
    out = np.empty(max(2 * ncand, 1), dtype=np.float64)
    a = int(lib().orc_polar_window(seed & M64, offset & M64, j0, ncand, mu, sigma, _p(out)))
    return out[:2 * a]


def polar_chunk_counts(seed: int, offset: int, ncand: int, chunk: int, threads: int | None = None,
                       kind: str = "polar") -> np.ndarray:
    """Accepted counts of consecutive candidate chunks [c, c + chunk) of the
    stream, each from one call of the reference count of the rejection
    method `kind` ("polar", "polar2" or "ratio"; two uniforms per candidate
    in each)."""
    starts = list(range(0, ncand, chunk))
    L = lib()
    count = {"polar": L.orc_polar_count, "polar2": L.orc_polar2_count, "ratio": L.orc_ratio_count}[kind]

    def work(c0):
        return int(count(seed & M64, (offset + 2 * c0) & M64, min(chunk, ncand - c0)))

    with ThreadPoolExecutor(max_workers=threads or os.cpu_count()) as ex:
        return np.array(list(ex.map(work, starts)), dtype=np.int64)


def polar_parallel(seed: int, offset: int, n: int, mu: float = 0.0, sigma: float = 1.0,
                   threads: int | None = None, chunk: int = 1 << 20):
    """Algorithm P over a long stream on several host threads: a count pass
    over candidate chunks, an exclusive prefix of the counts, then each chunk
    writes its accepted values at its prefix.  Same result as polar()."""
    npairs = (n + 1) // 2
    if n == 0:
        return np.empty(0), 0
    # Enough candidates: grow until the accepted count reaches npairs.
    ncand = int(npairs * 4 / np.pi * 1.01) + 4096
    while True:
        counts = polar_chunk_counts(seed, offset, ncand, chunk, threads)
        if counts.sum() >= npairs:
            break
        ncand *= 2
    pref = np.concatenate([[0], np.cumsum(counts)])
    last = int(np.searchsorted(pref, npairs, side="left")) - 1  # chunk holding pair npairs-1
    out = np.empty(2 * int(pref[last + 1]), dtype=np.float64)
    L = lib()

    def work(ci):
        c0 = ci * chunk
        m = min(chunk, ncand - c0)
        buf = out[2 * int(pref[ci]): 2 * int(pref[ci + 1])]
        L.orc_polar_window(seed & M64, offset & M64, c0, m, mu, sigma, _p(buf))

    with ThreadPoolExecutor(max_workers=threads or os.cpu_count()) as ex:
        list(ex.map(work, range(last + 1)))
    # candidate index of the npairs-th accepted pair -> consumed uniforms
    c0 = last * chunk
    masks, _, _ = polar_trace(seed, (offset + 2 * c0) & M64, min(chunk, ncand - c0))
    need = npairs - int(pref[last])
    bits = np.unpackbits(masks.view(np.uint8), bitorder="little")
    jlast = c0 + int(np.flatnonzero(bits)[need - 1])
    return out[:n], 2 * (jlast + 1)


# ---------------------------------------------------------------- P2
def p2_cheb(degree: int = 15) -> np.ndarray:
    """Chebyshev coefficients c_0..c_degree of h(v) on [-1, 1]."""
    c = np.empty(degree + 1, dtype=np.float64)
    lib().orc_p2_cheb(degree, _p(c))
    return c


def p2_h(v: float, degree: int = 15) -> float:
    """h(v) by the Chebyshev series truncated after T_degree."""
    return float(lib().orc_p2_h(degree, v))


def polar2(seed: int, offset: int, n: int, mu: float = 0.0, sigma: float = 1.0):
    """n normals by method P2; returns (values, uniforms consumed)."""
    out = np.empty(max(n, 1), dtype=np.float64)
    used = lib().orc_polar2(seed & M64, offset & M64, n, mu, sigma, _p(out))
    return out[:n], int(used)


def polar2_xy(xy, mu: float = 0.0, sigma: float = 1.0):
    """Method P2 on explicit integer candidates; as polar_xy."""
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1)
    ncand = xy.size // 2
    out = np.empty(max(2 * ncand, 1), dtype=np.float64)
    masks = np.empty(max((ncand + 63) // 64, 1), dtype=np.uint64)
    a = int(lib().orc_polar2_xy(_p(xy), ncand, mu, sigma, _p(out), _p(masks)))
    return out[:2 * a], masks[:(ncand + 63) // 64], a


def polar2_accept(X: int, Y: int) -> bool:
    return bool(lib().orc_polar2_accept(int(X), int(Y)))


def polar2_count(seed: int, offset: int, ncand: int) -> int:
    return int(lib().orc_polar2_count(seed & M64, offset & M64, ncand))


def polar2_window(seed: int, offset: int, j0: int, ncand: int, mu: float = 0.0, sigma: float = 1.0):
    out = np.empty(max(2 * ncand, 1), dtype=np.float64)
    a = int(lib().orc_polar2_window(seed & M64, offset & M64, j0, ncand, mu, sigma, _p(out)))
    return out[:2 * a]


# ---------------------------------------------------------------- B2
def b2_coef():
    """(s1, s3, s5, s7) and (c0, c2, c4, c6) of method B2's sine and cosine."""
    s = np.empty(4, dtype=np.float64)
    c = np.empty(4, dtype=np.float64)
    lib().orc_b2_coef(_p(s), _p(c))
    return s, c


def b2_sincos(v: float):
    """B2's approximations to sin(2 pi v - pi) and cos(2 pi v - pi)."""
    sn = np.empty(1, dtype=np.float64)
    cs = np.empty(1, dtype=np.float64)
    lib().orc_b2_sincos(float(v), _p(sn), _p(cs))
    return float(sn[0]), float(cs[0])


def b2(seed: int, offset: int, n: int, mu: float = 0.0, sigma: float = 1.0):
    """n normals by method B2; returns (values, uniforms consumed)."""
    out = np.empty(max(n, 1), dtype=np.float64)
    used = lib().orc_b2(seed & M64, offset & M64, n, mu, sigma, _p(out))
    return out[:n], int(used)


def b2_uv(u, v, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert u.shape == v.shape
    out = np.empty(2 * u.size, dtype=np.float64)
    lib().orc_b2_uv(_p(u), _p(v), u.size, mu, sigma, _p(out))
    return out


def b2_words(words, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint64)
    assert w.size % 2 == 0
    out = np.empty(w.size, dtype=np.float64)
    lib().orc_b2_words(_p(w), w.size // 2, mu, sigma, _p(out))
    return out


# ---------------------------------------------------------------- B3
def b3(seed: int, offset: int, n: int, mu: float = 0.0, sigma: float = 1.0):
    """n normals by method B3; returns (values, uniforms consumed)."""
    out = np.empty(max(n, 1), dtype=np.float64)
    used = lib().orc_b3(seed & M64, offset & M64, n, mu, sigma, _p(out))
    return out[:n], int(used)


def b3_u(u1, u2, u3, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    u1 = np.ascontiguousarray(u1, dtype=np.float64)
    u2 = np.ascontiguousarray(u2, dtype=np.float64)
    u3 = np.ascontiguousarray(u3, dtype=np.float64)
    assert u1.shape == u2.shape == u3.shape
    out = np.empty(2 * u1.size, dtype=np.float64)
    lib().orc_b3_u(_p(u1), _p(u2), _p(u3), u1.size, mu, sigma, _p(out))
    return out


def b3_words(words, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint64)
    assert w.size % 3 == 0
    out = np.empty(2 * (w.size // 3), dtype=np.float64)
    lib().orc_b3_words(_p(w), w.size // 3, mu, sigma, _p(out))
    return out


# ---------------------------------------------------------------- Algorithm R
def ratio(seed: int, offset: int, n: int, mu: float = 0.0, sigma: float = 1.0):
    """n normals by Algorithm R; returns (values, uniforms consumed)."""
    out = np.empty(max(n, 1), dtype=np.float64)
    used = lib().orc_ratio(seed & M64, offset & M64, n, mu, sigma, _p(out))
    return out[:n], int(used)


def ratio_accept(u: float, v: float) -> bool:
    return bool(lib().orc_ratio_accept(u, v))


def ratio_words(words, mu: float = 0.0, sigma: float = 1.0):
    """Algorithm R on explicit hash words (u-word, v-word per candidate).
    Returns (compacted values, mask words, number accepted)."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    ncand = w.size // 2
    out = np.empty(max(ncand, 1), dtype=np.float64)
    masks = np.empty(max((ncand + 63) // 64, 1), dtype=np.uint64)
    a = int(lib().orc_ratio_words(_p(w), ncand, mu, sigma, _p(out), _p(masks)))
    return out[:a], masks[:(ncand + 63) // 64], a


def ratio_count(seed: int, offset: int, ncand: int) -> int:
    return int(lib().orc_ratio_count(seed & M64, offset & M64, ncand))


def ratio_trace(seed: int, offset: int, ncand: int):
    nw = (ncand + 63) // 64
    masks = np.empty(max(nw, 1), dtype=np.uint64)
    pref = np.empty(max(nw, 1), dtype=np.uint64)
    a = int(lib().orc_ratio_trace(seed & M64, offset & M64, ncand, _p(masks), _p(pref)))
    return masks[:nw], pref[:nw], a


def ratio_window(seed: int, offset: int, j0: int, ncand: int, mu: float = 0.0, sigma: float = 1.0):
    out = np.empty(max(ncand, 1), dtype=np.float64)
    a = int(lib().orc_ratio_window(seed & M64, offset & M64, j0, ncand, mu, sigma, _p(out)))
    return out[:a]


# ---------------------------------------------------------------- statistics
def moments(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(4, dtype=np.float64)
    lib().orc_moments(_p(x), x.size, _p(out))
    return out


def normal_cdf(z: float) -> float:
    return float(lib().orc_normal_cdf(z))


def ks_normal(x, mu: float = 0.0, sigma: float = 1.0) -> float:
    x = np.array(x, dtype=np.float64, copy=True)
    return float(lib().orc_ks(_p(x), x.size, 0, mu, sigma))


def ks_uniform(x) -> float:
    x = np.array(x, dtype=np.float64, copy=True)
    return float(lib().orc_ks(_p(x), x.size, 1, 0.0, 1.0))


class use_library:
    """Context manager that points this wrapper at another build of the
    reference (the mutation tests compile deliberately broken copies of the
    C source on the CPU and check that the pins reject them)."""

    def __init__(self, path: str):
        self.path = path
        self.saved = None

    def __enter__(self):
        global _lib
        lib()
        self.saved = _lib
        L = ctypes.CDLL(self.path)
        for name in dir(self.saved):
            if name.startswith("orc_"):
                fn, ref = getattr(L, name), getattr(self.saved, name)
                fn.restype, fn.argtypes = ref.restype, ref.argtypes
        with _lock:
            _lib = L
        return L

    def __exit__(self, *exc):
        global _lib
        with _lock:
            _lib = self.saved
        return False


def build_variant(src_text: str, out_path: str) -> str:
    """Compile a (modified) copy of the reference source to out_path."""
    src_path = out_path + ".c"
    with open(src_path, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fPIC", "-shared",
                    "-I", _HERE, "-o", out_path, src_path, "-lm"], check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()
