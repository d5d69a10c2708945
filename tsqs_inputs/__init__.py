"""Seeded synthetic inputs shaped like the paper's workloads.

This module generates inputs only; it holds no part of any sort.  The tests,
the benchmark and the smoke check use it for both the GPU library and the CPU
oracle, so that both sort the same data.

Random numbers come from the counter-based SplitMix64 generator (Steele, Lea,
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
``x_i = mix(seed + (i + 1) * 0x9E3779B97F4A7C15)`` so that any element can be
generated on its own.

Families (the seven of the large single-sort workload, in the spirit of the
paper's SVI/SIX inputs, whose exact definitions in its reference [3] are not
available):

``uniform``        low 32 bits of ``x_i`` (int32/uint32), all 64 bits (int64/uint64),
                   N(0,1) by Box-Muller for float32 (with the special values below)
``sorted``         ``k_i = i``
``reversed``       ``k_i = n - 1 - i``
``nearly_sorted``  ``k_i = i``, then ``n // 200`` sequential swaps of positions
                   ``(x_{2j} mod n, x_{2j+1} mod n)`` (about 1% of positions moved)
``many_equals``    ``x_i mod 100``
``stair_steps``    ``i // 1000`` (ascending runs of 1000 equal values)
``organ_pipe``     ``1..n/2`` then ``n/2..1`` (``i + 1`` for ``i < n/2``, ``n - i`` after)

float32 families other than ``uniform`` are the float value of the integer family
(exact below 2^24).  ``special_float32`` salts N(0,1) with 0.1% each of -0.0,
+0.0, +inf, -inf and a quiet NaN.  ``distinct10_u64`` draws uint64 keys from a
pool of n/10 random values.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
FAMILIES = ["uniform", "sorted", "reversed", "nearly_sorted", "many_equals",
            "stair_steps", "organ_pipe"]
DTYPES = {"int32": np.int32, "uint32": np.uint32, "int64": np.int64,
          "uint64": np.uint64, "float32": np.float32}
BASE_SEED = 0x75C50000
CHUNK = 1 << 23


def seed_for(config: int, family: str | int) -> int:
    """Seed of a (workload number, family) pair: 0x75C50000 + 16*config + family."""
    f = FAMILIES.index(family) if isinstance(family, str) else int(family)
    return BASE_SEED + 16 * int(config) + f


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """x_i for i in [start, start + count) as uint64."""
    out = np.empty(count, dtype=np.uint64)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for c0 in range(0, count, CHUNK):
            c1 = min(count, c0 + CHUNK)
            i = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.uint64)
            out[c0:c1] = _mix(s + i * GOLDEN)
    return out


def _index_family(family: str, n: int, seed: int) -> np.ndarray:
    """Integer-valued families as int64 values (before the cast to a dtype)."""
    i = np.arange(n, dtype=np.int64)
    if family == "sorted":
        return i
    if family == "reversed":
        return n - 1 - i
    if family == "nearly_sorted":
        k = i.copy()
        nsw = n // 200
        if nsw and n > 1:
            x = splitmix64(seed, 2 * nsw)
            a = (x[0::2] % np.uint64(n)).astype(np.int64)
            b = (x[1::2] % np.uint64(n)).astype(np.int64)
            for p, q in zip(a.tolist(), b.tolist()):
                k[p], k[q] = k[q], k[p]
        return k
    if family == "many_equals":
        return (splitmix64(seed, n) % np.uint64(100)).astype(np.int64)
    if family == "stair_steps":
        return i // 1000
    if family == "organ_pipe":
        h = n // 2
        return np.where(i < h, i + 1, n - i)
    raise KeyError(family)


def normal_float32(seed: int, n: int) -> np.ndarray:
    """N(0,1) by Box-Muller from one 64-bit draw per element."""
    x = splitmix64(seed, n)
    u1 = ((x >> np.uint64(40)).astype(np.float64) + 1.0) * 2.0 ** -24
    u2 = (x & np.uint64(0xFFFFFF)).astype(np.float64) * 2.0 ** -24
    return (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).astype(np.float32)


SPECIAL_F32_BITS = [0x80000000, 0x00000000, 0x7F800000, 0xFF800000, 0x7FC00000]


def special_float32(seed: int, n: int) -> np.ndarray:
    """N(0,1) salted with 0.1% each of -0.0, +0.0, +inf, -inf, NaN (0x7FC00000)."""
    v = normal_float32(seed, n).view(np.uint32)
    sel = splitmix64(seed + 1, n) % np.uint64(1000)
    for j, bits in enumerate(SPECIAL_F32_BITS):
        v[sel == np.uint64(j)] = np.uint32(bits)
    return v.view(np.float32)


def distinct10_u64(seed: int, n: int) -> np.ndarray:
    """uint64 keys drawn from a pool of max(1, n // 10) random values."""
    pool_n = max(1, n // 10)
    pool = splitmix64(seed + 1, pool_n)
    idx = splitmix64(seed, n) % np.uint64(pool_n)
    return pool[idx.astype(np.int64)]


def family(name: str, n: int, dtype="int32", seed: int | None = None,
           config: int = 2) -> np.ndarray:
    """Keys of one family at size n and dtype (a numpy array on the host)."""
    dt = np.dtype(DTYPES[dtype] if isinstance(dtype, str) else dtype)
    if seed is None:
        seed = seed_for(config, name)
    if name == "uniform":
        if dt == np.float32:
            return special_float32(seed, n)
        x = splitmix64(seed, n)
        if dt.itemsize == 4:
            return (x & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(dt)
        return x.view(dt)
    v = _index_family(name, n, seed)
    if dt == np.float32:
        return v.astype(np.float32)
    return v.astype(dt)


def batch_sizes(seed: int, count: int, lo_log2: int = 4, hi_log2: int = 20) -> np.ndarray:
    """Sizes floor(2^lo * 2^((hi-lo)*u)), u uniform in [0,1): log-uniform on [2^lo, 2^hi]."""
    x = splitmix64(seed, count)
    u = (x >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.floor(2.0 ** lo_log2 * 2.0 ** ((hi_log2 - lo_log2) * u)).astype(np.int64)


def batch_families(seed: int, count: int) -> list:
    x = splitmix64(seed + 7, count)
    return [FAMILIES[int(v % np.uint64(len(FAMILIES)))] for v in x]


def batch(seed: int, count: int, lo_log2: int = 4, hi_log2: int = 20, dtype="int32",
          max_total: int | None = None):
    """Concatenated keys of ``count`` independent arrays with log-uniform sizes,
    each of a family drawn uniformly from the seven; array j uses sub-seed
    ``seed + 0x100000 + j`` so it can be regenerated alone.

    Returns (keys, offsets[count+1] uint64, families).  With ``max_total`` the
    arrays are drawn until the total would exceed it."""
    sizes = batch_sizes(seed, count, lo_log2, hi_log2)
    fams = batch_families(seed, count)
    if max_total is not None:
        cs = np.cumsum(sizes)
        keep = int(np.searchsorted(cs, max_total, side="right"))
        sizes, fams = sizes[:keep], fams[:keep]
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    dt = np.dtype(DTYPES[dtype] if isinstance(dtype, str) else dtype)
    keys = np.empty(int(offs[-1]), dtype=dt)
    for j, (s, f) in enumerate(zip(sizes.tolist(), fams)):
        keys[int(offs[j]):int(offs[j + 1])] = family(f, s, dt, seed=seed + 0x100000 + j)
    return keys, offs, fams


# ---- device-side generation (same arrays, generated by tsqs_inputs/gen.hip) ----

FAMILY_CODE = {f: i for i, f in enumerate(FAMILIES)}
DTYPE_CODE = {"int32": 0, "uint32": 1, "int64": 2, "uint64": 3, "float32": 4}
# device tensors hold unsigned keys in the signed type of the same width
TORCH_DTYPE = {"int32": "int32", "uint32": "int32", "int64": "int64", "uint64": "int64",
               "float32": "float32"}
_gen_lib = None


def _load_gen():
    global _gen_lib
    if _gen_lib is None:
        import ctypes
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtsqs_inputs.so")
        if not os.path.exists(path):
            raise ImportError("libtsqs_inputs.so is not built (python tsqs_inputs/build.py)")
        lib = ctypes.CDLL(path)
        lib.tsqs_inputs_generate.restype = ctypes.c_int
        lib.tsqs_inputs_generate.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                             ctypes.c_void_p]
        _gen_lib = lib
    return _gen_lib


def device_generate(out, dtype: str, offsets, fams, seeds) -> None:
    """Fill the device tensor ``out`` with arrays [offsets[j], offsets[j+1]) of
    family fams[j] (names) from seeds[j], exactly as ``family`` would on the host."""
    import torch
    lib = _load_gen()
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    fc = np.ascontiguousarray([FAMILY_CODE[f] for f in fams], dtype=np.int32)
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    count = len(fc)
    assert offs.size == count + 1 and sd.size == count
    assert out.is_cuda and out.numel() >= int(offs[-1])
    stream = torch.cuda.current_stream(out.device).cuda_stream
    rc = lib.tsqs_inputs_generate(out.data_ptr(), DTYPE_CODE[dtype], offs.ctypes.data,
                                  fc.ctypes.data, sd.ctypes.data, count, stream)
    if rc != 0:
        raise RuntimeError("tsqs_inputs_generate failed (%d)" % rc)


def device_family(name: str, n: int, dtype="int32", seed: int | None = None, config: int = 2,
                  device="cuda:0"):
    """``family(name, n, dtype, seed)`` generated directly in device memory."""
    import torch
    if seed is None:
        seed = seed_for(config, name)
    t = torch.empty(n, dtype=getattr(torch, TORCH_DTYPE[dtype]), device=device)
    device_generate(t, dtype, np.array([0, n], dtype=np.uint64), [name], [seed])
    return t


def batch_plan(seed: int, count: int, lo_log2: int = 4, hi_log2: int = 20,
               max_total: int | None = None):
    """Sizes, offsets, families and per-array seeds of ``batch`` (no keys)."""
    sizes = batch_sizes(seed, count, lo_log2, hi_log2)
    fams = batch_families(seed, count)
    if max_total is not None:
        cs = np.cumsum(sizes)
        keep = int(np.searchsorted(cs, max_total, side="right"))
        sizes, fams = sizes[:keep], fams[:keep]
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    seeds = np.uint64(seed + 0x100000) + np.arange(len(sizes), dtype=np.uint64)
    return sizes, offs, fams, seeds


def device_batch(seed: int, count: int, lo_log2: int = 4, hi_log2: int = 20, dtype="int32",
                 max_total: int | None = None, device="cuda:0"):
    """``batch(...)`` generated directly in device memory: (tensor, offsets, families)."""
    import torch
    sizes, offs, fams, seeds = batch_plan(seed, count, lo_log2, hi_log2, max_total)
    t = torch.empty(int(offs[-1]), dtype=getattr(torch, TORCH_DTYPE[dtype]), device=device)
    device_generate(t, dtype, offs, fams, seeds)
    return t, offs, fams


# ---- the input types and reorderings of the paper's comparison tests (SVI) -------------
#
# Input types (values before the cast to a dtype), with m the value range / period:
#   random    uniform in [0, m)                     sawtooth  i mod m
#   stagger   (i*m + i) mod n                      plateau   min(i, m)
#   shuffle   two interleaved increasing runs, the run chosen at random (one in m
#             picks the odd run)
#   hill      rises from 0 by 1 to the middle and falls back, clipped at m (SVI)
#   organ_pipes  straight ramps between random levels in [1, m] (plus op_add), each over a
#             random length of 1..op_max_distance keys (SVI)
# Reorderings: as generated, sorted, reversed, front half reversed, back half reversed,
# dither (key + i mod 5), and fort: the sorted keys, reversed as a whole, then each half
# again, recursively, while a range is longer than fort_min (SVI).
PAPER_TYPES = ["random", "sawtooth", "stagger", "plateau", "shuffle", "hill", "organ_pipes"]
PAPER_ORDERS = ["as_is", "sorted", "reversed", "front_half_reversed", "back_half_reversed",
                "dither", "fort"]


def _uniform_int(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    """Integers uniform in [lo, hi] (64-bit draws reduced modulo the range)."""
    return lo + (splitmix64(seed, n) % np.uint64(hi - lo + 1)).astype(np.int64)


def paper_type(kind: str, n: int, m: int, seed: int = 1, op_max_distance: int = 1000,
               op_add: int = 0) -> np.ndarray:
    """One of the SVI input types as int64 values."""
    i = np.arange(n, dtype=np.int64)
    m = max(1, int(m))
    if kind == "random":
        return _uniform_int(seed, n, 0, m - 1)
    if kind == "sawtooth":
        return i % m
    if kind == "stagger":
        return (i * m + i) % max(n, 1)
    if kind == "plateau":
        return np.minimum(i, m)
    if kind == "shuffle":
        odd = (splitmix64(seed, n) % np.uint64(m)) == 0      # one in m: the odd run
        out = np.empty(n, dtype=np.int64)
        ko = np.cumsum(odd) - 1                               # index within each run
        ke = np.cumsum(~odd) - 1
        out[odd] = 2 * ko[odd] + 1
        out[~odd] = 2 * ke[~odd]
        return out
    if kind == "hill":
        return np.minimum(np.where(i < (n >> 1), i, n - i), m)
    if kind == "organ_pipes":
        out = np.empty(n, dtype=np.float64)
        pos, k = 0, 0
        lv = _uniform_int(seed, 1, 1, m)[0]
        while pos < n:
            # the levels and lengths of the next 4096 ramps at once
            draws = splitmix64(seed + 1, 2 * 4096, start=2 * 4096 * k)
            lvl = 1 + (draws[0::2] % np.uint64(m)).astype(np.int64) + op_add
            dist = 1 + (draws[1::2] % np.uint64(max(1, op_max_distance))).astype(np.int64)
            for v, d in zip(lvl.tolist(), dist.tolist()):
                e = min(n, pos + d)
                step = (v - lv) / d
                out[pos:e] = lv + step * np.arange(e - pos)
                pos = e
                lv = v
                if pos >= n:
                    break
            k += 1
        return np.floor(out).astype(np.int64)
    raise KeyError(kind)


def fort(a: np.ndarray, fort_min: int) -> np.ndarray:
    """The ranges of a recursive halving, each reversed in turn from the whole array
    down: a range [lo, hi] is reversed, then, if it holds more than fort_min keys,
    [lo, mid] and [mid+1, hi] (mid = floor((lo+hi)/2)) are treated the same way."""
    out = np.array(a, copy=True)
    n = out.size
    lo = np.zeros(1, dtype=np.int64)
    hi = np.full(1, n - 1, dtype=np.int64)
    fort_min = max(1, int(fort_min))
    while lo.size and n:
        ln = hi - lo + 1
        idx = np.arange(n, dtype=np.int64)
        # every range of this depth reversed at once: position p -> lo + hi - p
        starts = np.repeat(lo, ln)
        ends = np.repeat(hi, ln)
        pos = starts + (np.arange(int(ln.sum()), dtype=np.int64) - np.repeat(np.cumsum(ln) - ln, ln))
        idx[pos] = starts + ends - pos
        out = out[idx]
        go = ln > fort_min
        mid = (lo + hi) >> 1
        lo, hi = np.concatenate([lo[go], mid[go] + 1]), np.concatenate([mid[go], hi[go]])
    return out


def paper_input(kind: str, order: str, n: int, m: int, dtype="int32", seed: int = 1,
                fort_min: int = 16) -> np.ndarray:
    """An SVI input type under one of the SVI reorderings, cast to dtype."""
    v = paper_type(kind, n, m, seed)
    h = n // 2
    if order == "sorted":
        v = np.sort(v)
    elif order == "reversed":
        v = v[::-1]
    elif order == "front_half_reversed":
        v = np.concatenate([v[:h][::-1], v[h:]])
    elif order == "back_half_reversed":
        v = np.concatenate([v[:h], v[h:][::-1]])
    elif order == "dither":
        v = v + np.arange(n, dtype=np.int64) % 5
    elif order == "fort":
        v = fort(np.sort(v), fort_min)
    elif order != "as_is":
        raise KeyError(order)
    dt = np.dtype(DTYPES[dtype] if isinstance(dtype, str) else dtype)
    return np.ascontiguousarray(v).astype(dt)
