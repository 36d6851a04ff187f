"""Seeded synthetic inputs shaped like the workloads the benchmarks and tests use.

This module only draws random bytes; it holds none of the coding arithmetic and
is shared by the oracle-side tests and the GPU-side tests/benchmark, which both
consume the very same bytes.  Generation runs with numpy on the host, or with
torch on a device (for the multi-GiB inputs); the two backends are not expected
to produce equal bytes, and nothing relies on that: parity always compares both
implementations on one buffer.

Distributions
-------------
* ``zipf``    -- finite Zipf(s) over 256 ranks, p_k proportional to k**-s
                 (k = 1..256); rank k is mapped to byte perm[k-1] with perm a
                 seeded permutation of 0..255.
* ``uniform`` -- i.i.d. uniform bytes (incompressible).
* ``skewed``  -- one dominant byte perm[0] with probability 0.9, each of the
                 other 255 values with probability 0.1/255.
* ``fp32``    -- the little-endian bytes of float32 values drawn from N(0, 1).

Workloads
---------
* single 1 MiB Zipf(1.2) stream, block size 4 KiB;
* single 256 MiB Zipf(1.1) stream, block size 64 KiB;
* 4 GiB mixed buffer: 64 segments of 64 MiB, segment t of kind
  (uniform, skewed, fp32)[t % 3], one codebook per segment.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 1107
MASK64 = (1 << 64) - 1

KIB = 1024
MIB = 1024 * 1024
GIB = 1024 * MIB

SEGMENT_KINDS = ("uniform", "skewed", "fp32")


def splitmix64(x: int) -> int:
    """SplitMix64 output function (Steele, Lea, Flood 2014): seed mixer."""
    x = (x + 0x9E3779B97F4A7C15) & MASK64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def derive_seed(config_id: int, index: int, base: int = BASE_SEED) -> int:
    """Seed of segment/buffer ``index`` of workload ``config_id``."""
    return splitmix64((base ^ (config_id << 32) ^ index) & MASK64) & ((1 << 63) - 1)


def zipf_cdf(s: float) -> np.ndarray:
    k = np.arange(1, 257, dtype=np.float64)
    p = k ** (-float(s))
    p /= p.sum()
    return np.cumsum(p)


def permutation(seed: int) -> np.ndarray:
    return np.random.default_rng(seed ^ 0x5EED).permutation(256).astype(np.uint8)


# ---------------------------------------------------------------- numpy (host)
def zipf_bytes(n: int, s: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    perm = permutation(seed)
    cdf = zipf_cdf(s)
    out = np.empty(n, dtype=np.uint8)
    step = 16 * MIB
    for a in range(0, n, step):
        u = rng.random(min(step, n - a))
        k = np.minimum(np.searchsorted(cdf, u, side="right"), 255)
        out[a:a + u.size] = perm[k]
    return out


def uniform_bytes(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 256, size=n, dtype=np.uint8)


def skewed_bytes(n: int, seed: int, p_major: float = 0.9) -> np.ndarray:
    rng = np.random.default_rng(seed)
    perm = permutation(seed)
    major = rng.random(n) < p_major
    others = perm[1 + rng.integers(0, 255, size=n)]
    return np.where(major, perm[0], others).astype(np.uint8)


def fp32_bytes(n: int, seed: int) -> np.ndarray:
    assert n % 4 == 0
    v = np.random.default_rng(seed).standard_normal(n // 4).astype("<f4")
    return v.view(np.uint8).copy()


def segment_bytes(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "uniform":
        return uniform_bytes(n, seed)
    if kind == "skewed":
        return skewed_bytes(n, seed)
    if kind == "fp32":
        return fp32_bytes(n, seed)
    raise ValueError(kind)


def mixed_kind(t: int) -> str:
    return SEGMENT_KINDS[t % 3]


# ---------------------------------------------------------------- torch (device)
def _torch_gen(seed: int, device):
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def zipf_bytes_torch(n: int, s: float, seed: int, device="cuda", out=None):
    import torch

    g = _torch_gen(seed, device)
    perm = torch.from_numpy(permutation(seed)).to(device)
    cdf = torch.from_numpy(zipf_cdf(s)).to(device)
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=device)
    step = 32 * MIB
    for a in range(0, n, step):
        m = min(step, n - a)
        u = torch.rand(m, dtype=torch.float64, device=device, generator=g)
        k = torch.clamp(torch.searchsorted(cdf, u, right=True), max=255)
        out[a:a + m] = perm[k]
    return out


def segment_bytes_torch(kind: str, n: int, seed: int, device="cuda", out=None):
    import torch

    g = _torch_gen(seed, device)
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=device)
    if kind == "uniform":
        out.copy_(torch.randint(0, 256, (n,), dtype=torch.uint8, device=device, generator=g))
    elif kind == "skewed":
        perm = torch.from_numpy(permutation(seed)).to(device)
        step = 32 * MIB
        for a in range(0, n, step):
            m = min(step, n - a)
            major = torch.rand(m, device=device, generator=g) < 0.9
            others = perm[1 + torch.randint(0, 255, (m,), device=device, generator=g)]
            out[a:a + m] = torch.where(major, perm[0], others)
    elif kind == "fp32":
        assert n % 4 == 0
        v = torch.randn(n // 4, dtype=torch.float32, device=device, generator=g)
        out.copy_(v.view(torch.uint8))
    else:
        raise ValueError(kind)
    return out


# ---------------------------------------------------------------- workloads
WORKLOADS = {
    "zipf1.2-1MiB-B4KiB": dict(config_id=1, n=1 * MIB, dist="zipf", s=1.2, block=4 * KIB),
    "zipf1.1-256MiB-B64KiB": dict(config_id=2, n=256 * MIB, dist="zipf", s=1.1, block=64 * KIB),
    "mixed-4GiB-64x64MiB": dict(config_id=3, n=4 * GIB, dist="mixed", segment=64 * MIB,
                                 blocks=(4 * KIB, 16 * KIB, 64 * KIB, 256 * KIB)),
}
