"""Seeded synthetic inputs for the C-PCM/ISWIG solvation path.

This module only draws inputs: atom positions and elements, Gaussian basis
shapes (exponents and raw contraction coefficients), unit-sphere point rules
and density matrices.  It holds none of the method's arithmetic (no
normalisation, no surface construction, no integrals), so both the oracle and
the HIP library can consume what it returns without sharing method code.

Units: everything returned is in bohr (positions, radii) and atomic units.

Recipes (stand-ins for the paper's protein set, Sec. 3 of the paper: proteins
of 100-500 atoms, 6-31G / 6-31G* basis sets, 110 points per atom, radii of
1.2 x Bondi, water dielectric):

* elements drawn to exact counts from H:C:N:O = 50:31:9:10 (largest remainder);
* positions from a self-avoiding random walk with bond lengths U[1.0, 1.5] A,
  confined to a sphere of protein atom density 0.115 atoms/A^3, no two atoms
  closer than 1.0 A (dead ends backtrack);
* basis shells shaped like 6-31G / 6-31G*: H s(3) s(1); C/N/O s(6), s(3)+p(3)
  with shared exponents, s(1)+p(1) with shared exponents, and d(1) for the
  starred form; exponents log-uniform in per-shell ranges, drawn once per
  element; raw coefficients U[0.1, 1];
* unit-sphere rules: a golden-spiral half set on the x > 0 hemisphere plus its
  x -> -x mirror images, equal weights 4*pi/n (sum of weights = 4*pi);
* density P = 2 C C^T with C the orthonormal columns of a seeded Gaussian
  matrix (thin QR with diag(R) > 0).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ANGSTROM = 1.0 / 0.529177210903  # bohr per angstrom

# Bondi van der Waals radii in angstrom (Bondi 1964); the cavity uses 1.2 x these.
BONDI_A = {"H": 1.20, "C": 1.70, "N": 1.55, "O": 1.52}
ZNUC = {"H": 1.0, "C": 6.0, "N": 7.0, "O": 8.0}
RADIUS_SCALE = 1.2


@dataclass
class Basis:
    """Contracted Cartesian Gaussian shells (raw, un-normalised coefficients)."""
    shell_atom: np.ndarray   # int32 [ns]
    shell_l: np.ndarray      # int32 [ns]  (0, 1, 2)
    shell_nprim: np.ndarray  # int32 [ns]
    shell_off: np.ndarray    # int32 [ns]  offset into prim arrays
    prim_exp: np.ndarray     # float64 [nprim_total]
    prim_coef: np.ndarray    # float64 [nprim_total]

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nbf(self) -> int:
        l = self.shell_l.astype(np.int64)
        return int(((l + 1) * (l + 2) // 2).sum())


@dataclass
class System:
    """One solute: atoms, basis, sphere rule and a density matrix."""
    name: str
    xyz: np.ndarray          # float64 [N,3] bohr
    Z: np.ndarray            # float64 [N]
    radius: np.ndarray       # float64 [N] cavity radius in bohr (1.2 x Bondi)
    elements: list
    basis: Basis
    sph_dirs: np.ndarray     # float64 [n_sph,3] unit vectors
    sph_w: np.ndarray        # float64 [n_sph] weights, sum = 4 pi
    P: np.ndarray            # float64 [nbf,nbf] symmetric
    eps: float = 78.39
    zeta0: float = 4.9
    seeds: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])


# ----------------------------------------------------------------------------
# sphere rules
# ----------------------------------------------------------------------------

def sphere_rule(n: int):
    """Mirror-closed golden-spiral rule with n (even) points and equal weights.

    The first n/2 points cover the x > 0 hemisphere with the polar axis along x;
    the second half are their images under x -> -x, so the rule maps onto
    itself under that mirror.  Weights are 4 pi / n each.
    """
    if n <= 0 or n % 2:
        raise ValueError("sphere rule needs an even, positive point count")
    h = n // 2
    golden = math.pi * (3.0 - math.sqrt(5.0))
    i = np.arange(h, dtype=np.float64)
    cx = 1.0 - (i + 0.5) / h          # cos(theta) in (0, 1)
    st = np.sqrt(np.maximum(0.0, 1.0 - cx * cx))
    ph = i * golden
    half = np.stack([cx, st * np.cos(ph), st * np.sin(ph)], axis=1)
    mirror = half.copy()
    mirror[:, 0] = -mirror[:, 0]
    dirs = np.concatenate([half, mirror], axis=0)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    w = np.full(n, 4.0 * math.pi / n)
    return dirs, w


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def element_counts(n_atoms: int, ratio=(("H", 50), ("C", 31), ("N", 9), ("O", 10))):
    """Exact element counts from a ratio by the largest-remainder rule."""
    tot = sum(r for _, r in ratio)
    quotas = [(e, n_atoms * r / tot) for e, r in ratio]
    base = {e: int(math.floor(q)) for e, q in quotas}
    left = n_atoms - sum(base.values())
    order = sorted(quotas, key=lambda t: (-(t[1] - math.floor(t[1])), [e for e, _ in ratio].index(t[0])))
    for e, _ in order[:left]:
        base[e] += 1
    return base


def confinement_radius_A(n_atoms: int, density=0.115):
    return (3.0 * n_atoms / (4.0 * math.pi * density)) ** (1.0 / 3.0)


def saw_positions(n_atoms: int, rng, conf_radius_A: float, bond=(1.0, 1.5), min_dist=1.0,
                  tries=64):
    """Self-avoiding walk inside a sphere (angstrom); backtracks on dead ends."""
    pos = np.zeros((n_atoms, 3))
    n = 1
    fails = np.zeros(n_atoms, dtype=np.int64)
    md2 = min_dist * min_dist
    r2max = conf_radius_A * conf_radius_A
    while n < n_atoms:
        prev = pos[n - 1]
        placed = False
        for _ in range(tries):
            v = rng.normal(size=3)
            v /= np.linalg.norm(v)
            cand = prev + v * rng.uniform(bond[0], bond[1])
            if cand @ cand > r2max:
                continue
            d = pos[:n] - cand
            if np.min(np.einsum("ij,ij->i", d, d)) < md2:
                continue
            pos[n] = cand
            n += 1
            placed = True
            break
        if not placed:
            fails[n] += 1
            back = 1 + min(int(fails[n]) // 4, 8)
            n = max(1, n - back)
    return pos


def protein_like(n_atoms: int, geom_seed: int, radius_scale: float = 1.0):
    """Element list and positions (bohr) for a protein-shaped synthetic solute."""
    rng = np.random.default_rng(geom_seed)
    counts = element_counts(n_atoms)
    elements = [e for e in ("H", "C", "N", "O") for _ in range(counts[e])]
    perm = rng.permutation(n_atoms)
    elements = [elements[i] for i in perm]
    pos_A = saw_positions(n_atoms, rng, confinement_radius_A(n_atoms) * radius_scale)
    return elements, pos_A * ANGSTROM


# ----------------------------------------------------------------------------
# basis shapes
# ----------------------------------------------------------------------------

def _loguniform(rng, lo, hi, n):
    return np.sort(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n)))[::-1].copy()


def basis_631g_shape(elements, basis_seed: int, polarized: bool = True) -> Basis:
    """6-31G(*)-shaped shells with synthetic exponents drawn once per element."""
    rng = np.random.default_rng(basis_seed)
    per_elem = {}
    for e in ("H", "C", "N", "O"):
        if e == "H":
            shells = [(0, _loguniform(rng, 0.15, 40.0, 3)), (0, _loguniform(rng, 0.08, 0.25, 1))]
        else:
            core = _loguniform(rng, 2.0, 6000.0, 6)
            inner = _loguniform(rng, 0.3, 40.0, 3)
            outer = _loguniform(rng, 0.08, 0.3, 1)
            shells = [(0, core), (0, inner), (1, inner), (0, outer), (1, outer)]
            if polarized:
                shells.append((2, _loguniform(rng, 0.5, 1.0, 1)))
        coefs = [rng.uniform(0.1, 1.0, size=len(ex)) for _, ex in shells]
        per_elem[e] = [(l, ex, c) for (l, ex), c in zip(shells, coefs)]
    return _assemble(elements, per_elem)


def _assemble(elements, per_elem) -> Basis:
    sa, sl, sn, so, pe, pc = [], [], [], [], [], []
    off = 0
    for ia, e in enumerate(elements):
        for l, ex, c in per_elem[e]:
            sa.append(ia); sl.append(l); sn.append(len(ex)); so.append(off)
            pe.extend(ex.tolist()); pc.extend(c.tolist())
            off += len(ex)
    return Basis(np.array(sa, np.int32), np.array(sl, np.int32), np.array(sn, np.int32),
                 np.array(so, np.int32), np.array(pe, np.float64), np.array(pc, np.float64))


# ----------------------------------------------------------------------------
# density matrices
# ----------------------------------------------------------------------------

def orthonormal_columns(n_rows: int, n_cols: int, rng):
    G = rng.normal(size=(n_rows, n_cols))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def density_matrix(nbf: int, n_occ: int, p_seed: int):
    rng = np.random.default_rng(p_seed)
    C = orthonormal_columns(nbf, n_occ, rng)
    P = 2.0 * (C @ C.T)
    return 0.5 * (P + P.T)


def occupied_windows(nbf: int, n_occ: int, p_seed: int, window: int = 1024):
    """Block-diagonal occupied coefficients: windows of `window` consecutive functions, each
    holding its share of the n_occ occupied columns as a seeded orthonormal block.  Returns a
    list of (first function, block) with blocks of shape (window, k)."""
    rng = np.random.default_rng(p_seed)
    out = []
    done = 0
    for s0 in range(0, nbf, window):
        s1 = min(nbf, s0 + window)
        k = round(n_occ * s1 / nbf) - done
        k = max(0, min(k, s1 - s0))
        done += k
        if k:
            out.append((s0, orthonormal_columns(s1 - s0, k, rng)))
    return out


def density_from_windows(nbf: int, windows):
    """P = 2 C C^T for block-diagonal C, symmetrised block by block (P is block-diagonal, so
    this equals symmetrising the whole matrix)."""
    P = np.empty((nbf, nbf))
    P.fill(0.0)  # touched once in order (first-touch page faults of a lazy zero array are slow here)
    for s0, C in windows:
        B = 2.0 * (C @ C.T)
        s1 = s0 + C.shape[0]
        P[s0:s1, s0:s1] = 0.5 * (B + B.T)
    return P


def density_matrix_blocked(nbf: int, n_occ: int, p_seed: int, window: int = 1024):
    """P = 2 C C^T with C block-diagonal over windows of `window` consecutive functions, each
    window holding its share of the n_occ occupied columns as a seeded orthonormal block.
    The columns of C are orthonormal, so P/2 is a projector of rank n_occ, as for the dense
    generator, but the cost is linear in nbf (used where nbf ~ 17k)."""
    return density_from_windows(nbf, occupied_windows(nbf, n_occ, p_seed, window))


def stress_outer_errors(n_out: int = 15):
    """Synthetic DIIS errors of the 2,000-atom stress schedule: e_t = 10 delta_t^1.07 with
    delta_t = 10^(-3 - 4 (t-1)/(n_out-1)), t = 1..n_out, so that Eq. 21 gives back delta_t
    (1e-3 down to 1e-7)."""
    deltas = [10.0 ** (-3.0 - 4.0 * t / (n_out - 1)) for t in range(n_out)]
    return [10.0 * d ** 1.07 for d in deltas], deltas


def perturbed_windows(windows, e_t: float, rng):
    """One outer step of the stress schedule: C_t = orth(C_{t-1} + e_t G_t) window by window,
    G_t seeded Gaussian, orth = QR with diag(R) > 0 (the columns stay orthonormal, so
    P_t = 2 C_t C_t^T is again a rank-n_occ projector times 2)."""
    out = []
    for s0, C in windows:
        Q, R = np.linalg.qr(C + e_t * rng.normal(size=C.shape))
        sg = np.sign(np.diag(R))
        sg[sg == 0] = 1.0
        out.append((s0, Q * sg))
    return out


def stress_density_sequence(s, n_out: int = 15):
    """The occupied windows C_1 .. C_n_out of the stress schedule for system s (2,000 atoms,
    blocked density): C_0 from the system's P seed, G_t from its perturbation seed."""
    nbf = s.basis.nbf
    n_occ = min(int(s.Z.sum()) // 2, nbf)
    C = occupied_windows(nbf, n_occ, s.seeds["P"])
    errs, _ = stress_outer_errors(n_out)
    rng = np.random.default_rng(s.seeds["pert"])
    seq = []
    for e in errs:
        C = perturbed_windows(C, e, rng)
        seq.append(C)
    return seq


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def _radii(elements):
    return np.array([RADIUS_SCALE * BONDI_A[e] * ANGSTROM for e in elements])


def _znuc(elements):
    return np.array([ZNUC[e] for e in elements])


def water_tiny() -> System:
    """3-atom water, 5 shells of 3 primitives, 7 functions, 110-point spheres."""
    c = 1
    elements = ["O", "H", "H"]
    xyz = np.array([[0.0, 0.0, 0.0], [0.757, 0.586, 0.0], [-0.757, 0.586, 0.0]]) * ANGSTROM
    rng = np.random.default_rng(100 * c + 2)
    per_elem = {
        "O": [(0, _loguniform(rng, 0.1, 100.0, 3)), (0, _loguniform(rng, 0.1, 100.0, 3)),
              (1, _loguniform(rng, 0.1, 100.0, 3))],
        "H": [(0, _loguniform(rng, 0.1, 100.0, 3))],
    }
    per_elem = {e: [(l, ex, rng.uniform(0.1, 1.0, size=3)) for l, ex in v] for e, v in per_elem.items()}
    basis = _assemble(elements, per_elem)
    prng = np.random.default_rng(100 * c + 3)
    Q = orthonormal_columns(7, 7, prng)
    C = Q[:, :5]
    P = 2.0 * C @ C.T
    dirs, w = sphere_rule(110)
    return System("water_tiny", xyz, _znuc(elements), _radii(elements), elements, basis, dirs, w,
                  0.5 * (P + P.T), seeds={"geometry": None, "basis": 102, "P": 103, "rbj": 104, "pert": 105})


def protein_system(name: str, n_atoms: int, n_sph: int, cfg: int, polarized: bool = True,
                   radius_scale: float = 1.0, geom_seed=None, p_seed=None, blocked_p: bool = False) -> System:
    gs = 100 * cfg + 1 if geom_seed is None else geom_seed
    ps = 100 * cfg + 3 if p_seed is None else p_seed
    elements, xyz = protein_like(n_atoms, gs, radius_scale)
    basis = basis_631g_shape(elements, 100 * cfg + 2, polarized)
    Z = _znuc(elements)
    n_occ = int(Z.sum()) // 2
    dm = density_matrix_blocked if blocked_p else density_matrix
    P = dm(basis.nbf, min(n_occ, basis.nbf), ps)
    dirs, w = sphere_rule(n_sph)
    return System(name, xyz, Z, _radii(elements), elements, basis, dirs, w, P,
                  seeds={"geometry": gs, "basis": 100 * cfg + 2, "P": ps, "rbj": 100 * cfg + 4,
                         "pert": 100 * cfg + 5})


# Raw unit-sphere rules are sized so that the kept surface has the configured density
# (~50 points per atom, as in the paper's proteins: 26,025 points for 516 atoms).  The
# seeded walk is more compact than those structures and buries ~75% of a 110-point rule.
RAW_SPH_600 = 276    # -> ~30k kept points for 600 atoms
RAW_SPH_2000 = 540   # -> ~150k kept points for 2,000 atoms
RAW_SPH_300 = 270    # -> ~15k kept points for 300 atoms


def protein_single_solve() -> System:
    """600 atoms, 6-31G*-shaped basis, ~30k kept surface points."""
    return protein_system("protein600_631gs", 600, RAW_SPH_600, 2)


def linear_solve_stress() -> System:
    """2,000 atoms, 6-31G*-shaped basis, ~150k kept surface points."""
    return protein_system("protein2000_631gs", 2000, RAW_SPH_2000, 3, blocked_p=True)


def gradient_path() -> System:
    """300 atoms, 6-31G*-shaped basis, ~15k kept surface points."""
    return protein_system("peptide300_631gs", 300, RAW_SPH_300, 4)


CONFORMER_SPH = (96, 116, 136, 162, 194)  # -> 4k-9k kept points per conformer


def conformer(j: int) -> System:
    """Conformer j of a 150-atom peptide, 6-31G-shaped basis, uneven surface sizes."""
    rng = np.random.default_rng(5000 + j)
    scale = float(rng.uniform(1.0, 1.8))
    n_sph = int(CONFORMER_SPH[j % len(CONFORMER_SPH)])
    return protein_system(f"conformer{j}", 150, n_sph, 5, polarized=False, radius_scale=scale,
                          geom_seed=501 + 1000 * j, p_seed=503 + 1000 * j)


def small_protein(n_atoms: int = 8, n_sph: int = 50, seed: int = 7, polarized: bool = True) -> System:
    """Small protein-shaped case for parity tests (several tiles, ragged tails)."""
    return protein_system(f"small{n_atoms}_{seed}", n_atoms, n_sph, 0, polarized=polarized,
                          geom_seed=1000 + seed, p_seed=2000 + seed)


def born_ion(radius: float, n_sph: int, Z: float = 1.0) -> dict:
    """One sphere of cavity radius `radius` (bohr) with a point charge Z at its centre."""
    dirs, w = sphere_rule(n_sph)
    return {"xyz": np.zeros((1, 3)), "Z": np.array([Z]), "radius": np.array([radius]),
            "sph_dirs": dirs, "sph_w": w}
