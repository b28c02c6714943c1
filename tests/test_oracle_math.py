"""Pins of the oracle's math against libraries and closed forms (CPU only).

- exp: error bound against the correctly rounded exponential;
- SH basis: orthonormality by exact quadrature and the addition theorem;
- fp16 / bf16 rounding: numpy's and torch's independent conversions.
"""
import math

import numpy as np
import pytest

import oracle


def _ulp(x):
    return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)


def test_vm_exp_error_bound():
    """The decision exp stays within 2 ulp of exp over the splat's domain [-87, 0]."""
    rng = np.random.default_rng(1)
    x = np.concatenate([np.linspace(-87.0, 0.0, 400001), rng.uniform(-87.0, 0.0, 200000),
                        -np.logspace(-8, 0, 2000), [-0.0, 0.0, -87.0, -1e-30]]).astype(np.float32)
    y = oracle.vm_exp_n(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    err = np.abs(y - ref) / _ulp(ref.astype(np.float32))
    assert err.max() <= 2.0, err.max()
    assert oracle.vm_exp(0.0) == 1.0
    # below -87 the definition returns exactly zero
    assert oracle.vm_exp(-87.5) == 0.0 and oracle.vm_exp(-1000.0) == 0.0


def test_vm_exp_monotone():
    """exp must not decrease: alpha thresholds rely on it."""
    x = np.linspace(-20.0, 0.0, 300001).astype(np.float32)
    y = oracle.vm_exp_n(x)
    assert np.all(np.diff(y) >= 0.0)


def _sphere_quadrature(n_theta=24, n_phi=48):
    # Gauss-Legendre in cos(theta) and a uniform grid in phi: exact for the
    # degree <= 6 products of two degree-3 harmonics
    xg, wg = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1.0 - ct ** 2)
    x, y, z = st * np.cos(ph), st * np.sin(ph), ct
    w = np.repeat(wg[:, None], n_phi, 1) * (2.0 * np.pi / n_phi)
    return x.ravel(), y.ravel(), z.ravel(), w.ravel()


def test_sh_orthonormal():
    x, y, z, w = _sphere_quadrature()
    B = np.array([[oracle.sh_basis(k, a, b, c) for a, b, c in zip(x, y, z)] for k in range(16)])
    gram = (B * w) @ B.T
    assert np.abs(gram - np.eye(16)).max() < 1e-10


def test_sh_addition_theorem():
    rng = np.random.default_rng(2)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        for l in range(4):
            s = sum(oracle.sh_basis(k, *d) ** 2 for k in range(l * l, (l + 1) * (l + 1)))
            assert abs(s - (2 * l + 1) / (4 * math.pi)) < 1e-12


def test_sh_degree0_constant():
    assert abs(oracle.sh_basis(0, 0.3, 0.4, math.sqrt(0.75)) - 0.5 / math.sqrt(math.pi)) < 1e-15


def test_round_f16_matches_numpy():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 100000), rng.normal(0, 1e-5, 20000),
                        rng.uniform(-7e4, 7e4, 20000), np.array([0.0, -0.0, 65504.0, 65519.9, 65520.0,
                                                                 6.1e-5, 5.96e-8, 2.98e-8, 1.0 + 2 ** -11])]).astype(np.float32)
    # exact ties: halfway between neighbouring fp16 values
    h = np.float16(rng.normal(0, 10, 5000)).astype(np.float32)
    x = np.concatenate([x, h + np.spacing(np.float16(h)).astype(np.float32) / 2])
    got = oracle.round_f16_n(x)
    ref = x.astype(np.float16).astype(np.float32)
    same = (got == ref) | (np.isnan(got) & np.isnan(ref))
    assert same.all(), x[~same][:5]


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(0, 1, 100000), rng.normal(0, 1e-30, 1000), rng.normal(0, 1e30, 1000)]).astype(np.float32)
    b = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    ties = b + np.spacing(b) * 0  # bf16 values
    mid = (ties.view(np.uint32) + np.uint32(0x8000)).view(np.float32)  # exact halfway points
    x = np.concatenate([x, mid])
    got = oracle.round_bf16_n(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(got, ref)
