"""Seeded synthetic tables shared by the oracle side and the GPU side of the tests.

Holds no arithmetic of the method: only a counter-based random generator
(SplitMix64; Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), the relabelling of symbols used to make a table
invariant under c -> c xor m, and the exchange of strings 1 and 2 used to
make it invariant under that too.  Everything is torch integer arithmetic, so the
same call gives identical bits on the CPU and on a GPU.
"""
from __future__ import annotations

import torch

_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _s64(x: int) -> int:
    """Python int -> the int64 with the same 64 bits."""
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= 1 << 63 else x


def _lsr(z: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def splitmix64(seed: int, idx: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output number idx+1 from the state seed * 2^32 * golden, i.e.
    the mix of the state (seed * 2^32 + idx + 1) * golden (mod 2^64)."""
    z = (idx.to(torch.int64) + 1) * _s64(_GOLDEN) + _s64((seed << 32) * _GOLDEN)
    z = (z ^ _lsr(z, 30)) * _s64(_M1)
    z = (z ^ _lsr(z, 27)) * _s64(_M2)
    return z ^ _lsr(z, 31)


def uniform(seed: int, idx: torch.Tensor, scale: float = 8.0) -> torch.Tensor:
    """float64 values in [0, scale) from the top 53 bits of SplitMix64."""
    return _lsr(splitmix64(seed, idx), 11).to(torch.float64) * (scale * 2.0 ** -53)


def representative(idx: torch.Tensor, sigma: int, d: int, h: int) -> torch.Tensor:
    """Index with every symbol xor-ed by the string-1 head symbol, so the
    string-1 head becomes 0 (layout: beta-bit symbols, position-major, string
    1 first, heads in the top d*beta bits)."""
    beta = {2: 1, 4: 2}[sigma]
    n = sigma ** (d * h)
    head_shift = beta * d * (h - 1) + beta * (d - 1)
    rep_bits = (n - 1) // (sigma - 1)
    m = (idx >> head_shift) & (sigma - 1)
    return idx ^ (m * _s64(rep_bits))


def exchanged(idx: torch.Tensor, sigma: int, d: int, h: int) -> torch.Tensor:
    """Index of the tuple with strings 1 and 2 exchanged (their symbol fields
    swapped at every position); sigma = 2 or 4."""
    beta = {2: 1, 4: 2}[sigma]
    slot = beta * d
    r = ((1 << (slot * h)) - 1) // ((1 << slot) - 1)   # the lowest bit of every position
    f = (1 << beta) - 1
    a = _s64(r * (f << (slot - beta)))                  # string 1's field
    b = _s64(r * (f << (slot - 2 * beta)))              # string 2's field
    rest = _s64(((1 << (slot * h)) - 1) & ~(r * (f << (slot - beta)) | r * (f << (slot - 2 * beta))))
    return _lsr(idx & a, beta) | ((idx & b) << beta) | (idx & rest)


def table(sigma: int, d: int, h: int, seed: int, dtype=torch.float64, device="cpu",
          symmetric: bool = True, scale: float = 8.0, chunk: int = 1 << 26,
          exchange: bool = False) -> torch.Tensor:
    """A seeded table of sigma^(d h) values; symmetric under c -> c xor m if
    asked, and also under exchanging strings 1 and 2 if
    `exchange`: each value is then drawn at the lower of the two
    representatives."""
    n = sigma ** (d * h)
    out = torch.empty(n, dtype=dtype, device=device)
    for lo in range(0, n, chunk):
        idx = torch.arange(lo, min(n, lo + chunk), dtype=torch.int64, device=device)
        if symmetric:
            idx = representative(idx, sigma, d, h)
        if exchange:
            assert symmetric
            idx = torch.minimum(idx, representative(exchanged(idx, sigma, d, h), sigma, d, h))
        out[lo:lo + idx.numel()] = uniform(seed, idx, scale).to(dtype)
    return out


def sample_indices(n: int, count: int, seed: int) -> torch.Tensor:
    """Sorted distinct-ish sample of [0, n) plus both ends and the quarter
    boundaries (where the head symbols change)."""
    base = (_lsr(splitmix64(seed, torch.arange(count, dtype=torch.int64)), 1) % n)
    cand = {0, 1, n - 2, n - 1, n // 4 - 1, n // 4, n // 2 - 1, n // 2, 3 * n // 4 - 1, 3 * n // 4}
    edges = torch.tensor(sorted(e for e in cand if 0 <= e < n), dtype=torch.int64)
    return torch.unique(torch.cat([base, edges]))


def orbit(idx: int, sigma: int, d: int, h: int) -> list:
    """Every index of the orbit of idx under the relabellings c -> c xor m and
    the exchange of strings 1 and 2 (sorted); a table symmetric under both is
    constant on it."""
    n = sigma ** (d * h)
    rep_bits = (n - 1) // (sigma - 1)
    e = int(exchanged(torch.tensor([idx], dtype=torch.int64), sigma, d, h)[0])
    return sorted({j ^ (m * rep_bits) for j in (idx, e) for m in range(sigma)})


def stored_table(sigma: int, d: int, h: int, seed: int, dtype=torch.float64, device="cpu",
                 scale: float = 8.0, chunk: int = 1 << 26) -> torch.Tensor:
    """The first n / sigma values (string-1 head 0) of table(..., exchange=True)."""
    n = sigma ** (d * h)
    ns = n // sigma
    out = torch.empty(ns, dtype=dtype, device=device)
    for lo in range(0, ns, chunk):
        idx = torch.arange(lo, min(ns, lo + chunk), dtype=torch.int64, device=device)
        idx = torch.minimum(idx, representative(exchanged(idx, sigma, d, h), sigma, d, h))
        out[lo:lo + idx.numel()] = uniform(seed, idx, scale).to(dtype)
    return out
