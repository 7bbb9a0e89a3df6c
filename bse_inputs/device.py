"""Seeded generator of Bethe-Salpeter problems made directly in device memory.

The same distribution as generators.gen_bse (A = diag(u) + s_a/sqrt(n)
(G1 + G1^H)/sqrt(2) with u ~ U[1, 10], B = s_b/sqrt(n) (G2 + G2^T)/sqrt(2), G
complex Gaussian of unit variance, a unit complex dipole), drawn with torch's
device generator (Philox) instead of numpy's PCG64, so that a stream of
thousands of requests can be made on the device at submission time without
holding them all in host or device memory.  A seed always gives the same
matrices on the same device type; the values differ from gen_bse's.  No
definiteness check is made (with the default scales it never fails, see the
rejection note in generators.py).

Returned buffers are column-major (the layout the solver reads): a tensor
holding M^T row-major.
"""

from __future__ import annotations

import math

import torch


def gen_bse_device(n: int, seed: int, device, s_a: float = 0.1, s_b: float = 0.05):
    """Returns (A_colmajor, B_colmajor, d) complex128 on `device`."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    u = 1.0 + 9.0 * torch.rand(n, generator=g, device=device, dtype=torch.float64)

    def cgauss():
        re = torch.randn((n, n), generator=g, device=device, dtype=torch.float64)
        im = torch.randn((n, n), generator=g, device=device, dtype=torch.float64)
        return torch.complex(re, im) / math.sqrt(2.0)

    g1 = cgauss()
    A = (s_a / math.sqrt(n)) * (g1 + g1.conj().transpose(0, 1)) / math.sqrt(2.0)
    A.diagonal().add_(u.to(torch.complex128))
    del g1
    g2 = cgauss()
    B = (s_b / math.sqrt(n)) * (g2 + g2.transpose(0, 1)) / math.sqrt(2.0)
    del g2
    dr = torch.randn(2 * n, generator=g, device=device, dtype=torch.float64)
    di = torch.randn(2 * n, generator=g, device=device, dtype=torch.float64)
    d = torch.complex(dr, di)
    d = d / torch.linalg.vector_norm(d)
    return A.transpose(0, 1).contiguous(), B.transpose(0, 1).contiguous(), d

