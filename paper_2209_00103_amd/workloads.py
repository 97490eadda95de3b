"""Seeded synthetic workloads for the GGArray hot path.

This module only produces inputs: which logical thread inserts, what payload it
inserts, how many elements a thread inserts, and the per-array sizes of the batched
workload.  It holds none of the data structure's arithmetic (no bucket law, no
index mapping, no scan), so both the HIP library and the CPU oracle may consume it.

Every random quantity is drawn from one counter-based generator,

    K(seed, a, b) = splitmix64((seed << 56) ^ (a << 8) ^ b),   seed < 2^8, a < 2^48, b < 2^8,

where splitmix64(x) is the output of the SplitMix64 generator of Steele, Lea and
Flood ("Fast splittable pseudorandom number generators", OOPSLA 2014) whose state
equals x before the step: add the golden-ratio increment 0x9E3779B97F4A7C15, then
apply the two xor-shift-multiply rounds and a final xor-shift.  The HIP kernels and
the oracle each carry their own implementation of the same published definition;
this numpy one is the third, used to build buffer-mode inputs.

The paper evaluates on synthetic doubling/insertion loops only (Sec. VI-A, VI-C,
VI-D); the workloads below keep those shapes and add the irregular, batched and
served shapes of the project's configurations.
"""
from __future__ import annotations

from decimal import Decimal, getcontext

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)
_U64 = np.uint64


def splitmix64(x) -> np.ndarray:
    """SplitMix64 output for state ``x`` (uint64 array), wrapping mod 2^64."""
    z = np.asarray(x, dtype=np.uint64) + GOLDEN_GAMMA
    z = (z ^ (z >> _U64(30))) * _MIX1
    z = (z ^ (z >> _U64(27))) * _MIX2
    return z ^ (z >> _U64(31))


def K(seed: int, a, b) -> np.ndarray:
    """The counter-based generator K(seed, a, b) over uint64 arrays."""
    if not 0 <= int(seed) < 256:
        raise ValueError("seed must be < 2^8")
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    x = (_U64(seed) << _U64(56)) ^ (a << _U64(8)) ^ b
    return splitmix64(x)


# ---------------------------------------------------------------------------
# Configuration 1: Bernoulli(1/2) insertions, hashed payload.
# ---------------------------------------------------------------------------
CFG1 = dict(V=256, F=1024, block=1024, n_threads=1 << 18, rounds=4, elem_bytes=4)


def bernoulli_round(seed: int, r: int, n_threads: int, elem_bytes: int = 4):
    """Thread ``gid`` of round ``r`` draws h = K(seed, gid, r); it inserts iff the top
    bit of h is set, and its payload is h truncated to the element width.
    Returns (values, flags)."""
    h = K(seed, np.arange(n_threads, dtype=np.uint64), r)
    flags = (h >> _U64(63)).astype(np.uint8)
    values = h.astype(np.uint32) if elem_bytes == 4 else h.copy()
    return values, flags


# ---------------------------------------------------------------------------
# Configuration 2: 2^28 insertions over 12 growth rounds, shrink 1/10 per round.
# ---------------------------------------------------------------------------
CFG2 = dict(F=1024, block=1024, V_sweep=(32, 256, 512), V=512, rounds=12,
            shrink=(1, 10), tag_shift=27, elem_bytes=4)


def cfg2_round_threads(rounds: int = 12) -> list[int]:
    """n_0 = 2^17 and n_r = 2^(16+r) for r >= 1, so that 12 rounds insert 2^28."""
    return [1 << 17] + [1 << (16 + r) for r in range(1, rounds)]


def round_tag_values(r: int, n_threads: int, tag_shift: int = 27, elem_bytes: int = 4):
    """Every thread inserts (r << tag_shift) | gid, truncated to the element width."""
    g = np.arange(n_threads, dtype=np.uint64)
    v = (_U64(r) << _U64(tag_shift)) | g
    return v.astype(np.uint32) if elem_bytes == 4 else v


# ---------------------------------------------------------------------------
# Configuration 3: per-thread counts Poisson(3) capped at 16, uint64 payloads.
# ---------------------------------------------------------------------------
CFG3 = dict(F=1024, block=1024, V=65536, n_threads=1 << 26, phases=4, lam=3,
            max_count=16, elem_bytes=8)


def poisson_thresholds(lam: int = 3, kmax: int = 16) -> np.ndarray:
    """T[k] = floor(2^64 * P(X <= k)) for X ~ Poisson(lam), k = 0..kmax-1.

    A thread drawing a uniform 64-bit u then inserts c = #{k : u >= T[k]}
    elements, so P(c > k) = 1 - P(X <= k): c is Poisson(lam) capped at kmax.
    Computed once on the host in 60-digit decimal arithmetic."""
    getcontext().prec = 60
    lam_d = Decimal(lam)
    term = (-lam_d).exp()
    cdf = Decimal(0)
    out = []
    two64 = Decimal(2) ** 64
    for k in range(kmax):
        if k > 0:
            term = term * lam_d / Decimal(k)
        cdf += term
        t = int((cdf * two64).to_integral_value(rounding="ROUND_FLOOR"))
        out.append(min(t, (1 << 64) - 1))
    return np.array(out, dtype=np.uint64)


def poisson_counts(seed: int, phase: int, n_threads: int, thresholds: np.ndarray,
                   gid0: int = 0) -> np.ndarray:
    """c[gid] = #{k : K(seed, gid, 0x80 | phase) >= T[k]} (uint8)."""
    u = K(seed, np.arange(gid0, gid0 + n_threads, dtype=np.uint64), 0x80 | phase)
    c = np.zeros(n_threads, dtype=np.uint8)
    for t in thresholds:
        c += (u >= t).astype(np.uint8)
    return c


def poisson_payload(seed: int, phase: int, gid, j) -> np.ndarray:
    """Payload j of thread gid in insert phase ``phase``: K(seed, gid, 16*phase + j)."""
    return K(seed, gid, 16 * phase + np.asarray(j, dtype=np.uint64))


# ---------------------------------------------------------------------------
# Configuration 4: 512 arrays of log-uniform target size.
# ---------------------------------------------------------------------------
CFG4 = dict(n_arrays=512, lo_log2=10, span_log2=14, rounds=4, elem_bytes=4,
            block_sweep=(256, 512, 1024), F_sweep=tuple(1 << k for k in range(6, 15)))


def cfg4_sizes(seed: int, n_arrays: int = 512) -> np.ndarray:
    """n_a = floor(2^(10 + 14 * u_a / 2^53)) with u_a = K(seed, a, 0xF0) >> 11."""
    u = K(seed, np.arange(n_arrays, dtype=np.uint64), 0xF0) >> _U64(11)
    expo = 10.0 + 14.0 * (u.astype(np.float64) / float(1 << 53))
    return np.floor(np.exp2(expo)).astype(np.int64)


def cfg4_vectors(n_a: int) -> int:
    """LFVector count of a batched array: the smallest power of two >= n_a / 2^14,
    clamped to [1, 1024].  A fixed rule, never tuned."""
    need = -(-int(n_a) // (1 << 14))
    v = 1
    while v < need:
        v <<= 1
    return max(1, min(1024, v))


def cfg4_round_threads(n_a: int, rounds: int = 4) -> list[int]:
    """ceil(n_a / rounds) threads per round, the remainder in the last round."""
    per = -(-int(n_a) // rounds)
    out = [per] * (rounds - 1)
    out.append(int(n_a) - per * (rounds - 1))
    return out


def cfg4_values(seed: int, a: int, r: int, n_threads: int) -> np.ndarray:
    """Thread t of round r of array a inserts (u32) K(seed, (a << 32) | t, r)."""
    t = np.arange(n_threads, dtype=np.uint64)
    return K(seed, (_U64(a) << _U64(32)) | t, r).astype(np.uint32)


# ---------------------------------------------------------------------------
# Configuration 5: served requests over resident arrays.
# ---------------------------------------------------------------------------
CFG5 = dict(n_arrays=4096, median_log2=16, sigma=1.0, size_cap_log2=24, n_requests=1 << 20,
            append_median_log2=10, append_cap_log2=20, mix=(0.6, 0.3, 0.1), cap_bytes=64 << 30,
            elem_bytes=4, fill_round=0xA1, append_round=0xA0, append_shift=20,
            loads=(0.25, 0.5, 0.75, 0.9, 1.1))

REQ_APPEND, REQ_RW, REQ_FLATTEN = 0, 1, 2


def _unit(seed: int, a, b: int) -> np.ndarray:
    """Uniform doubles in (0, 1): (top 53 bits of K + 1/2) / 2^53."""
    return ((K(seed, a, b) >> _U64(11)).astype(np.float64) + 0.5) / float(1 << 53)


def _normal(seed: int, a, b1: int, b2: int) -> np.ndarray:
    """Standard normal by Box-Muller: sqrt(-2 ln u1) cos(2 pi u2)."""
    u1, u2 = _unit(seed, a, b1), _unit(seed, a, b2)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def cfg5_sizes(seed: int, n_arrays: int = 4096, median_log2: int = 16, sigma: float = 1.0,
               cap_log2: int = 24) -> np.ndarray:
    """Initial sizes s_a = round(2^median_log2 * e^(sigma z_a)), clipped to [1, 2^cap_log2]."""
    z = _normal(seed, np.arange(n_arrays, dtype=np.uint64), 0xB0, 0xB1)
    s = np.rint(float(1 << median_log2) * np.exp(sigma * z))
    return np.clip(s, 1, 1 << cap_log2).astype(np.int64)


def cfg5_first_bucket(n_a: int, V: int) -> int:
    """First bucket of a served array: the largest power of two <= n_a / (8 V),
    clamped to [64, 4096].  A fixed rule, never tuned."""
    f = 64
    while f * 2 <= min(4096, int(n_a) // (8 * V)):
        f *= 2
    return f


def cfg5_fill_values(seed: int, a: int, n: int) -> np.ndarray:
    """Initial contents of array a: one round where thread t inserts (u32) K(seed, (a << 32) | t, 0xA1)."""
    return cfg4_values(seed, a, CFG5["fill_round"], n)


def cfg5_trace(seed: int, n_requests: int, n_arrays: int, append_median_log2: int = 10,
               append_cap_log2: int = 20, mix=(0.6, 0.3, 0.1)) -> dict:
    """Request r: gap g_r ~ Exp(1) (in units of the mean inter-arrival time), type
    append / r/w / flatten with probabilities mix, target uniform over the arrays,
    append length round(2^append_median_log2 * e^z) clipped to [1, 2^append_cap_log2]."""
    r = np.arange(n_requests, dtype=np.uint64)
    gap = -np.log(_unit(seed, r, 0xC0))
    u = _unit(seed, r, 0xC1)
    kind = np.where(u < mix[0], REQ_APPEND, np.where(u < mix[0] + mix[1], REQ_RW, REQ_FLATTEN)).astype(np.uint8)
    target = ((K(seed, r, 0xC2) >> _U64(11)) % _U64(n_arrays)).astype(np.uint32)
    z = _normal(seed, r, 0xC3, 0xC4)
    length = np.clip(np.rint(float(1 << append_median_log2) * np.exp(z)), 1, 1 << append_cap_log2)
    length = np.where(kind == REQ_APPEND, length, 0).astype(np.uint32)
    return dict(gap=gap, kind=kind, target=target, length=length)


def cfg5_arrivals_ns(gap: np.ndarray, rate_per_s: float) -> np.ndarray:
    """Arrival times in ns of a trace offered at rate_per_s requests per second
    (rate 0 or inf: everything arrives at once)."""
    if not rate_per_s or not np.isfinite(rate_per_s):
        return np.zeros(gap.size, dtype=np.uint64)
    return np.floor(np.cumsum(gap) * (1e9 / rate_per_s)).astype(np.uint64)


def cfg5_append_values(seed: int, req: int, n: int) -> np.ndarray:
    """Payload of append request req: element j is (u32) K(seed, (req << 20) | j, 0xA0)."""
    j = np.arange(n, dtype=np.uint64)
    return K(seed, (_U64(req) << _U64(CFG5["append_shift"])) | j, CFG5["append_round"]).astype(np.uint32)


# ---------------------------------------------------------------------------
# Generic random cases for property tests.
# ---------------------------------------------------------------------------
def random_round(rng: np.random.Generator, n_threads: int, p: float, elem_bytes: int):
    """Uniform payloads with Bernoulli(p) insert flags from a numpy Generator."""
    if elem_bytes == 4:
        values = rng.integers(0, 1 << 32, size=n_threads, dtype=np.uint64).astype(np.uint32)
    else:
        values = rng.integers(0, np.iinfo(np.uint64).max, size=n_threads,
                              dtype=np.uint64, endpoint=True)
    flags = (rng.random(n_threads) < p).astype(np.uint8)
    return values, flags
