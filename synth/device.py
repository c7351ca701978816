"""Seeded generators that build large synthetic operands directly in device
memory with torch (for benchmark-sized inputs that would take minutes to
build on the host).  Patterns and values only: none of the product's
arithmetic.  The results are ordinary CSR tensors; copying one back gives the
oracle the same operand."""
from __future__ import annotations

import numpy as np


def erdos_renyi_device(m: int, n: int, density: float, seed: int, dtype=None, device="cuda"):
    """Uniform-random pattern: row i draws Binomial(n, density) column indices
    uniformly *with* replacement and keeps the distinct ones (sorted), so a
    row's expected length is n*(1 - (1 - 1/n)^L) for L drawn indices -- below
    the Binomial mean by about L/(2n) relative (under 0.5 % for density <=
    1e-2).  Values uniform in [-1, 1).  Returns (row_ptr int32, col int32,
    val) torch tensors on `device`."""
    import torch
    dtype = dtype or torch.float64
    rng = np.random.default_rng(seed)
    lengths = rng.binomial(n, density, size=m).astype(np.int64)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    total = int(lengths.sum())
    if total == 0:
        return (torch.zeros(m + 1, dtype=torch.int32, device=device),
                torch.zeros(0, dtype=torch.int32, device=device), torch.zeros(0, dtype=dtype, device=device))
    rows = torch.repeat_interleave(torch.arange(m, device=device, dtype=torch.int64),
                                   torch.from_numpy(lengths).to(device))
    cols = torch.randint(0, n, (total,), device=device, generator=gen, dtype=torch.int64)
    keys = torch.unique(rows * n + cols)  # sorted by (row, column), duplicates removed
    r = keys // n
    c = (keys - r * n).to(torch.int32)
    counts = torch.bincount(r, minlength=m)
    rp = torch.zeros(m + 1, dtype=torch.int64, device=device)
    rp[1:] = torch.cumsum(counts, 0)
    val = torch.rand(c.numel(), device=device, generator=gen, dtype=torch.float64) * 2.0 - 1.0
    return rp.to(torch.int32), c, val.to(dtype)
