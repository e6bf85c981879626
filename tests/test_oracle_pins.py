"""Further pins of the oracle, each against a value fixed outside the oracle's own code.

* Eq. 9 in the region where two spheres of unequal radius overlap: the switching value of a
  point is compared with Eq. 9 as printed, 1 - {erf[z(R_J - d)] + erf[z(R_J + d)]}/2,
  evaluated in 40-digit arithmetic (mpmath), with R_J the radius of the *other* atom.
* Gauss's law with an electron density (Sec. 2, Eq. 1 in the conductor limit f = 1): for a
  density held well inside the cavity the induced charge tends to minus the enclosed charge,
  sum q -> -(Z - tr(P S)), as the sphere rule is refined.  This fixes the sign and scale of
  c (Eqs. 5-6) against B z (Eq. 4).
* The Eq. 15 bound for s-type primitives equals [ij|ij]^(1/2): the potential of the product
  density chi_i chi_j (a Gaussian of exponent p at P) is S_ij erf(sqrt(p) r)/r, so
  [ij|ij] = S_ij [chi_i | erf(sqrt(p)|r-P|)/|r-P| | chi_j], the already pinned primitive block
  at C = P, zeta = sqrt(p).
* The far-field form of the auxiliary integrals (the attenuated operator acting as 1/r once
  a r^2 >= T0) differs from the exact Boys form by at most the upper incomplete gamma tail
  Gamma(n+1/2, T) / Gamma(n+1/2); the bound is evaluated here for n <= 5 at T0 = 40 and 30.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from synth import inputs as I

EMPTY = I.Basis(*(np.zeros(0, np.int32) for _ in range(4)), np.zeros(0), np.zeros(0))
ZETA0 = 4.9


def _eq9_printed(zeta, RJ, d):
    mpmath.mp.dps = 40
    z, R, dd = mpmath.mpf(zeta), mpmath.mpf(RJ), mpmath.mpf(d)
    return float(1 - (mpmath.erf(z * (R - dd)) + mpmath.erf(z * (R + dd))) / 2)


@pytest.mark.parametrize("delta", [-0.3, -0.05, 0.0, 0.05, 0.3])
def test_switching_in_overlap_of_unequal_spheres(delta):
    # atom I (radius 2.0) at the origin, atom J (radius 3.1) on the x axis so that I's +x point
    # sits at distance R_J + delta from J, and J's -x point at distance R_I + delta from I
    rI, rJ = 2.0, 3.1
    xJ = rI + rJ + delta
    dirs = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    w = np.array([2.0 * math.pi, 2.0 * math.pi])
    om = O.OracleMol(np.array([[0.0, 0.0, 0.0], [xJ, 0.0, 0.0]]), [1.0, 1.0], [rI, rJ], dirs, w, EMPTY,
                     switch_thresh=0.0)
    assert om.M == 4 and list(om.keep_idx) == [0, 1, 2, 3]
    zI = ZETA0 / (rI * math.sqrt(w[0]))
    zJ = ZETA0 / (rJ * math.sqrt(w[0]))
    cases = [
        (0, zI, rJ, abs(xJ - rI)),          # I's +x point against sphere J
        (1, zI, rJ, xJ + rI),               # I's -x point, far side of I
        (2, zJ, rI, abs(xJ + rJ)),          # J's +x point, far side of J
        (3, zJ, rI, abs(xJ - rJ)),          # J's -x point against sphere I
    ]
    for k, z, R_other, d in cases:
        assert om.zeta[k] == pytest.approx(z, rel=1e-15)
        ref = _eq9_printed(z, R_other, d)
        assert abs(om.S[k] - ref) <= 1e-14 * ref + 1e-300, (k, om.S[k], ref)
        assert om.Akk[k] == pytest.approx(math.sqrt(2.0 / math.pi) * z / ref, rel=1e-14)
    # the overlap points are really in the switching region (not rounded to 0 or 1)
    assert 0.05 < om.S[0] < 0.95 and 0.05 < om.S[3] < 0.95


def _one_atom_s_density(n_sph, Z=4.0, n_el=2.0, radius=3.0):
    basis = I.Basis(shell_atom=np.array([0], np.int32), shell_l=np.array([0], np.int32),
                    shell_nprim=np.array([3], np.int32), shell_off=np.array([0], np.int32),
                    prim_exp=np.array([1.2, 3.0, 8.0]), prim_coef=np.array([0.5, 0.4, 0.3]))
    dirs, w = I.sphere_rule(n_sph)
    om = O.OracleMol(np.zeros((1, 3)), [Z], [radius], dirs, w, basis, eps=1e300)
    assert om.f == 1.0 and om.nbf == 1
    P = np.array([[n_el]])  # one normalised function: tr(P S) = n_el
    bz = om.bz()
    c = om.esp(P)
    q = om.solve_dense(bz + c)
    return om, c, q


def test_gauss_law_with_electron_density():
    Z, n_el = 4.0, 2.0
    errs = []
    for n in (110, 302, 1202):
        om, c, q = _one_atom_s_density(n, Z, n_el)
        # the electrons lower the potential on the surface: c ~ -n_el / R on every point
        assert np.all(c < 0)
        assert abs(c.mean() + n_el / 3.0) < 1e-3 * n_el / 3.0
        errs.append(abs(q.sum() + (Z - n_el)) / (Z - n_el))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3, errs
    # a dropped sign of Eq. 6 would give -(Z + n_el), a doubled c -(Z - 2 n_el): both far off
    assert errs[0] < 0.05


def test_gauss_law_net_zero_charge():
    # a neutral atom (Z equal to the electron count) induces no net surface charge
    om, c, q = _one_atom_s_density(302, Z=2.0, n_el=2.0)
    assert abs(q.sum()) < 1e-3 * np.abs(q).sum() + 1e-9


@pytest.mark.parametrize("seed", range(6))
def test_eq15_bound_is_schwarz_value_for_s_primitives(seed):
    rng = np.random.default_rng(4100 + seed)
    ea, eb = np.exp(rng.uniform(np.log(0.1), np.log(50.0), 2))
    A = np.zeros(3)
    B = rng.normal(size=3) * rng.uniform(0.2, 2.0)
    basis = I.Basis(shell_atom=np.array([0, 1], np.int32), shell_l=np.array([0, 0], np.int32),
                    shell_nprim=np.array([1, 1], np.int32), shell_off=np.array([0, 1], np.int32),
                    prim_exp=np.array([ea, eb]), prim_coef=np.array([0.7, 0.3]))
    dirs, w = I.sphere_rule(50)
    om = O.OracleMol(np.stack([A, B]), [1.0, 1.0], [2.0, 2.0], dirs, w, basis)
    p = ea + eb
    Pc = (ea * A + eb * B) / p
    S_ab = (math.pi / p) ** 1.5 * math.exp(-ea * eb / p * float(((A - B) ** 2).sum()))
    ij_ij = S_ab * O.prim_block(0, 0, A, ea, B, eb, Pc, math.sqrt(p))[0, 0]
    norm = lambda a: (2.0 * a / math.pi) ** 0.75  # unit self-overlap of a one-primitive s shell
    bound = norm(ea) * norm(eb) * math.sqrt(ij_ij)

    def has_pair(thresh):
        pr = om.pairs(thresh=thresh)
        return any(a == 0 and b == 1 for a, b in zip(pr["a"], pr["b"]))

    assert has_pair(bound * (1.0 - 1e-10))
    assert not has_pair(bound * (1.0 + 1e-10))


@pytest.mark.parametrize("T0", [40.0, 30.0])
def test_far_field_tail_bound(T0):
    # relative difference of (2n-1)!!/(2^(n+1)) sqrt(pi/T^(2n+1)) (the far form) from F_n(T),
    # against the bound Gamma(n+1/2, T0)/Gamma(n+1/2), checked with the oracle's Boys function
    mpmath.mp.dps = 40
    for T in (T0, T0 + 0.5, T0 + 3.0, 2.0 * T0):
        F = O.boys(5, T)
        for n in range(6):
            far = math.prod(range(1, 2 * n, 2)) / 2 ** (n + 1) * math.sqrt(math.pi / T ** (2 * n + 1))
            rel = (far - F[n]) / F[n]
            bound = float(mpmath.gammainc(n + 0.5, T0) / mpmath.gamma(n + 0.5))
            assert rel >= -1e-15 and rel <= bound * (1 + 1e-6) + 4e-16, (T, n, rel, bound)
    # the bound itself: at most 1.5e-12 (n = 5) at T0 = 40, 9.3e-9 at T0 = 30
    worst = float(mpmath.gammainc(5.5, T0) / mpmath.gamma(5.5))
    assert worst < (1.5e-12 if T0 == 40.0 else 9.3e-9)
