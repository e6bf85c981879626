"""Pins of the oracle's integral code against mathematics it does not use.

* Boys function vs mpmath's incomplete gamma (F_m(T) = gamma(m+1/2, T) / (2 T^(m+1/2))).
* s-s primitive integral vs its closed form S_ab erf(sqrt(a) R)/R, a = p z^2/(p+z^2),
  including the R -> 0 limit (Appendix-style derivation from Eq. 6).
* zeta -> infinity gives the textbook point-charge nuclear attraction; zeta -> 0 gives
  (2 zeta/sqrt(pi)) times the overlap.
* Any angular momentum vs an independent quadrature: erf(z r)/r = 2/sqrt(pi) int_0^z exp(-s^2 r^2) ds,
  Gauss-Legendre in s and exact Gauss-Hermite three-centre overlaps in x, y, z.
* p-type = (1/2 alpha) d/dA_x of the s-type closed form (complex-step derivative).
* Derivative block vs central differences of the value block.
* Contracted normalisation: unit self-overlap by Gauss-Hermite quadrature.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import erf, roots_hermite, roots_legendre

from oracle import oracle as O


def cart_list(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


@pytest.mark.parametrize("m", [0, 1, 2, 3, 5, 7])
@pytest.mark.parametrize("T", [0.0, 1e-6, 0.3, 2.5, 11.0, 29.9, 30.1, 45.0, 120.0])
def test_boys_vs_mpmath(m, T):
    F = O.boys(m, T)
    mpmath.mp.dps = 40
    for mm in range(m + 1):
        if T == 0.0:
            ref = 1.0 / (2 * mm + 1)
        else:
            ref = float(mpmath.gammainc(mm + 0.5, 0, T) / (2 * mpmath.mpf(T) ** (mm + 0.5)))
        assert abs(F[mm] - ref) <= 2e-15 * ref + 1e-300


def ss_closed(A, ea, B, eb, C, z):
    p = ea + eb
    P = (ea * A + eb * B) / p
    K = np.exp(-ea * eb / p * np.sum((A - B) ** 2))
    S = (np.pi / p) ** 1.5 * K
    a = p * z * z / (p + z * z)
    R = np.sqrt(np.sum((P - C) ** 2))
    if abs(R) < 1e-300:
        return S * 2.0 * np.sqrt(a / np.pi)
    return S * erf(np.sqrt(a) * R) / R


def test_ss_closed_form():
    rng = np.random.default_rng(11)
    for _ in range(200):
        A, B, C = rng.normal(size=(3, 3)) * 2.0
        ea, eb = np.exp(rng.uniform(np.log(0.05), np.log(500.0), 2))
        z = np.exp(rng.uniform(np.log(0.5), np.log(20.0)))
        v = O.prim_block(0, 0, A, ea, B, eb, C, z)[0, 0]
        ref = ss_closed(A, ea, B, eb, C, z)
        assert abs(v - ref) <= 1e-13 * abs(ref) + 1e-300


def test_ss_coincident_limit():
    A = np.array([0.3, -0.2, 0.1])
    v = O.prim_block(0, 0, A, 1.3, A, 0.7, A, 3.0)[0, 0]
    ref = ss_closed(A, 1.3, A, 0.7, A, 3.0)
    assert abs(v - ref) <= 1e-14 * ref


def test_zeta_infinite_is_nuclear_attraction():
    A, B, C = np.array([0.1, 0.2, -0.3]), np.array([-0.5, 0.4, 0.2]), np.array([0.9, -0.7, 0.5])
    ea, eb = 0.8, 1.7
    p = ea + eb
    P = (ea * A + eb * B) / p
    K = math.exp(-ea * eb / p * np.sum((A - B) ** 2))
    T = p * np.sum((P - C) ** 2)
    F0 = float(mpmath.gammainc(0.5, 0, T) / (2 * mpmath.mpf(T) ** 0.5))
    ref = 2 * math.pi / p * K * F0
    v = O.prim_block(0, 0, A, ea, B, eb, C, 1e7)[0, 0]
    assert abs(v - ref) <= 1e-12 * ref


def three_centre_overlap(a, A, ea, b, B, eb, C, s2, nh=12):
    """prod_d int (x-A)^a (x-B)^b exp(-ea(x-A)^2 - eb(x-B)^2 - s2 (x-C)^2) dx, exact Gauss-Hermite."""
    t, w = roots_hermite(nh)
    q = ea + eb + s2
    out = 1.0
    for d in range(3):
        Q = (ea * A[d] + eb * B[d] + s2 * C[d]) / q
        E = (ea * eb * (A[d] - B[d]) ** 2 + ea * s2 * (A[d] - C[d]) ** 2 + eb * s2 * (B[d] - C[d]) ** 2) / q
        x = Q + t / math.sqrt(q)
        out *= math.exp(-E) * np.sum(w * (x - A[d]) ** a[d] * (x - B[d]) ** b[d]) / math.sqrt(q)
    return out


def quad_block(la, lb, A, ea, B, eb, C, z, ns=200):
    s, ws = roots_legendre(ns)
    s = 0.5 * z * (s + 1.0)
    ws = 0.5 * z * ws
    out = np.zeros((len(cart_list(la)), len(cart_list(lb))))
    for i, a in enumerate(cart_list(la)):
        for j, b in enumerate(cart_list(lb)):
            out[i, j] = 2.0 / math.sqrt(math.pi) * sum(
                wk * three_centre_overlap(a, A, ea, b, B, eb, C, sk * sk) for sk, wk in zip(s, ws))
    return out


@pytest.mark.parametrize("la,lb", [(0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (1, 2), (2, 1), (2, 2), (3, 2)])
def test_block_vs_quadrature(la, lb):
    rng = np.random.default_rng(100 + 10 * la + lb)
    for _ in range(3):
        A, B, C = rng.normal(size=(3, 3)) * 1.2
        ea, eb = np.exp(rng.uniform(np.log(0.2), np.log(4.0), 2))
        z = rng.uniform(1.0, 5.0)
        v = O.prim_block(la, lb, A, ea, B, eb, C, z)
        ref = quad_block(la, lb, A, ea, B, eb, C, z)
        scale = np.abs(ref).max()
        assert np.abs(v - ref).max() <= 1e-12 * scale


def test_zeta_to_zero_is_scaled_overlap():
    A, B, C = np.array([0.1, 0.2, -0.3]), np.array([-0.5, 0.4, 0.2]), np.array([3.0, -2.0, 1.5])
    z = 1e-5
    for la, lb in [(0, 0), (1, 1), (2, 1), (2, 2)]:
        v = O.prim_block(la, lb, A, 0.9, B, 1.4, C, z)
        ov = np.array([[three_centre_overlap(a, A, 0.9, b, B, 1.4, C, 0.0) for b in cart_list(lb)]
                       for a in cart_list(la)])
        ref = 2 * z / math.sqrt(math.pi) * ov
        assert np.abs(v - ref).max() <= 1e-8 * np.abs(ref).max()


def test_p_type_is_derivative_of_closed_form():
    A, B, C = np.array([0.3, -0.1, 0.4]), np.array([-0.6, 0.5, 0.1]), np.array([1.1, 0.7, -0.9])
    ea, eb, z = 1.1, 0.6, 3.2
    h = 1e-20
    v = O.prim_block(1, 0, A, ea, B, eb, C, z)[:, 0]
    for d in range(3):
        Ac = A.astype(complex)
        Ac[d] += 1j * h
        p = ea + eb
        P = (ea * Ac + eb * B) / p
        K = np.exp(-ea * eb / p * np.sum((Ac - B) ** 2))
        a = p * z * z / (p + z * z)
        R = np.sqrt(np.sum((P - C) ** 2))
        f = (np.pi / p) ** 1.5 * K * erf(np.sqrt(a) * R) / R
        ref = f.imag / h / (2 * ea)
        assert abs(v[d] - ref) <= 1e-13 * abs(ref) + 1e-16


def test_derivative_block_vs_central_differences():
    rng = np.random.default_rng(5)
    for la, lb in [(0, 0), (1, 0), (1, 2), (2, 2)]:
        A, B, C = rng.normal(size=(3, 3))
        ea, eb, z = 0.9, 1.6, 2.5
        dA, dB = O.prim_block_deriv(la, lb, A, ea, B, eb, C, z)
        h = 1e-5
        for d in range(3):
            e = np.zeros(3); e[d] = h
            fa = (O.prim_block(la, lb, A + e, ea, B, eb, C, z) - O.prim_block(la, lb, A - e, ea, B, eb, C, z)) / (2 * h)
            fb = (O.prim_block(la, lb, A, ea, B + e, eb, C, z) - O.prim_block(la, lb, A, ea, B - e, eb, C, z)) / (2 * h)
            sc = max(np.abs(fa).max(), np.abs(fb).max())
            assert np.abs(dA[d] - fa).max() <= 1e-8 * sc
            assert np.abs(dB[d] - fb).max() <= 1e-8 * sc


def test_hermitian_block():
    A, B, C = np.array([0.2, 0.1, -0.4]), np.array([-0.3, 0.6, 0.5]), np.array([0.7, -0.2, 0.3])
    for la, lb in [(0, 1), (1, 2), (0, 2)]:
        ab = O.prim_block(la, lb, A, 0.7, B, 1.9, C, 2.0)
        ba = O.prim_block(lb, la, B, 1.9, A, 0.7, C, 2.0)
        assert np.abs(ab - ba.T).max() <= 1e-14 * np.abs(ab).max()


def test_contracted_normalisation(water_oracle):
    om = water_oracle
    t, w = roots_hermite(40)
    for s in range(om.ns):
        l, npr = int(om.sl[s]), int(om.snp[s])
        ex = om.pexp[om.soff[s]:om.soff[s] + npr]
        for c, (ax, ay, az) in enumerate(cart_list(l)):
            cf = om.cn[om.cn_off[s] + c * npr: om.cn_off[s] + (c + 1) * npr]
            tot = 0.0
            for i in range(npr):
                for j in range(npr):
                    q = ex[i] + ex[j]
                    x = t / math.sqrt(q)
                    one = [np.sum(w * x ** (2 * n)) / math.sqrt(q) for n in (ax, ay, az)]
                    tot += cf[i] * cf[j] * one[0] * one[1] * one[2]
            assert abs(tot - 1.0) <= 1e-13
