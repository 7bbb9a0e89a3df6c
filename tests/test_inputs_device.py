"""The device-side request generator (bse_inputs.device), run on the CPU:
structure of the problems it makes (A Hermitian with its diagonal in
[1, 10], B complex symmetric, a unit dipole), the column-major layout the
solver reads, determinism by seed, and the off-diagonal scales of the
stated distribution."""

import math

import numpy as np
import torch

from bse_inputs.device import gen_bse_device


def test_structure_layout_and_seed():
    n = 96
    Ac, Bc, d = gen_bse_device(n, 7, "cpu", s_a=0.3, s_b=0.05)
    A, B = Ac.transpose(0, 1), Bc.transpose(0, 1)   # column-major buffers hold M^T row-major
    assert Ac.dtype == torch.complex128 and Ac.shape == (n, n) and d.shape == (2 * n,)
    assert torch.equal(A, A.conj().transpose(0, 1))
    assert torch.equal(B, B.transpose(0, 1))
    dg = A.diagonal().real
    # u ~ U[1, 10] plus the kernel's real diagonal term (standard deviation s_a / sqrt(n) ~ 0.03 here)
    assert float(dg.min()) >= 0.5 and float(dg.max()) <= 10.5
    assert abs(float(torch.linalg.vector_norm(d)) - 1.0) < 1e-14
    Ac2, Bc2, d2 = gen_bse_device(n, 7, "cpu", s_a=0.3, s_b=0.05)
    assert torch.equal(Ac, Ac2) and torch.equal(Bc, Bc2) and torch.equal(d, d2)
    Ac3, _, _ = gen_bse_device(n, 8, "cpu", s_a=0.3, s_b=0.05)
    assert not torch.equal(Ac, Ac3)


def test_off_diagonal_scales():
    # off-diagonal entries of A and B are complex Gaussian with E|x|^2 = s^2 / n
    n, s_a, s_b = 400, 0.3, 0.05
    Ac, Bc, _ = gen_bse_device(n, 3, "cpu", s_a=s_a, s_b=s_b)
    off = ~torch.eye(n, dtype=torch.bool)
    va = float((Ac.abs() ** 2)[off].mean())
    vb = float((Bc.abs() ** 2)[off].mean())
    assert math.isclose(va, s_a ** 2 / n, rel_tol=0.02)
    assert math.isclose(vb, s_b ** 2 / n, rel_tol=0.02)
    # the diagonal of A is u ~ U[1, 10] plus a real kernel term of variance s_a^2 / n
    u = Ac.diagonal().real.numpy()
    assert abs(float(np.mean(u)) - 5.5) < 0.5
