"""Pins of the oracle's surface, operators, solve, energy and gradient.

Each check uses a fact fixed by the paper or by mathematics, not the oracle's own
formulas: exact switching values far from other atoms, mirror symmetry, symmetry
and positive definiteness of A (Sec. 2, Eqs. 2-3), the Born ion and Gauss's law
(Eq. 1 in the conductor limit), linearity / adjointness of c and the Fock term
(Eqs. 5 and 10), the stationarity identity of the energy (Eq. 13), the
preconditioner limits stated in Sec. 4b-ii, and central finite differences plus
translation invariance of the gradient (Eq. 14).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from synth import inputs as I

EMPTY = I.Basis(*(np.zeros(0, np.int32) for _ in range(4)), np.zeros(0), np.zeros(0))


def test_isolated_points_have_unit_switching():
    # two atoms far apart: every point is > R_J + 6/zeta from the other nucleus
    xyz = np.array([[0.0, 0.0, 0.0], [40.0, 0.0, 0.0]])
    dirs, w = I.sphere_rule(50)
    om = O.OracleMol(xyz, [1.0, 1.0], [2.7, 2.7], dirs, w, EMPTY)
    assert om.M == 100
    assert np.all(om.S == 1.0)
    assert np.allclose(om.Akk, math.sqrt(2 / math.pi) * om.zeta, rtol=0, atol=0)


def test_surface_mirror_symmetry(water_oracle):
    om = water_oracle
    raw = om.N * om.nsph
    keep = np.zeros(raw, bool)
    keep[om.keep_idx] = True
    h = om.nsph // 2
    # x -> -x maps atom 1 <-> 2 (the H atoms), atom 0 onto itself, sphere point j <-> j +- n/2
    def mirror(k):
        I_, j = divmod(k, om.nsph)
        J = {0: 0, 1: 2, 2: 1}[I_]
        return J * om.nsph + (j + h) % om.nsph
    for k in range(raw):
        assert keep[k] == keep[mirror(k)]
    S = dict(zip(om.keep_idx.tolist(), om.S.tolist()))
    for k in om.keep_idx:
        assert abs(S[k] - S[mirror(int(k))]) <= 1e-14 * S[k]


def test_prune_threshold(water):
    om0 = O.mol_from_system(water, switch_thresh=0.0)
    om = O.mol_from_system(water)
    assert om0.M > om.M
    assert np.all(om.S >= 1e-8)


def test_A_symmetric_positive_definite(water_oracle):
    A = water_oracle.amat()
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0


def test_A_offdiagonal_limit_matches_diagonal_reading():
    # Eq. 2 at r -> 0 between two equal Gaussians equals Eq. 3 with S = 1 under the sqrt(2/pi) reading
    xyz = np.zeros((1, 3))
    dirs = np.array([[1.0, 0, 0], [1.0, 1e-9, 0]])
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    w = np.array([2 * math.pi, 2 * math.pi])
    om = O.OracleMol(xyz, [1.0], [3.0], dirs, w, EMPTY)
    A = om.amat()
    assert abs(A[0, 1] - A[0, 0]) <= 1e-12 * A[0, 0]


def born(n, R=3.0, Z=1.0):
    d = I.born_ion(R, n, Z)
    om = O.OracleMol(d["xyz"], d["Z"], d["radius"], d["sph_dirs"], d["sph_w"], EMPTY)
    bz = om.bz()
    A = om.amat()
    q = om.solve_dense(bz, A)
    return om, om.energy(bz, np.zeros(om.M), q, A @ q), q


def test_born_ion_converges_to_born_energy():
    errs = []
    for n in (50, 110, 302, 1202):
        om, E, q = born(n)
        errs.append(abs(E - (-om.f / (2 * 3.0))) / (om.f / 6.0))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-3
    assert errs[1] < 5e-3  # 110 points


def test_gauss_law_total_charge():
    # conductor limit: sum q -> -f Z for a charge inside a closed cavity
    errs = []
    for n in (110, 302, 1202):
        om, E, q = born(n, R=2.5, Z=2.0)
        errs.append(abs(q.sum() + om.f * 2.0) / (2.0 * om.f))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-3


def test_eps_infinite_limit_f_equals_one():
    d = I.born_ion(3.0, 110)
    om = O.OracleMol(d["xyz"], d["Z"], d["radius"], d["sph_dirs"], d["sph_w"], EMPTY, eps=1e300)
    assert om.f == 1.0


def test_c_is_linear_and_adjoint_to_fock(water, water_oracle):
    om = water_oracle
    pr = om.pairs()  # Eq. 15 list, no density weighting: c linear in P exactly
    nbf = om.nbf
    # materialise L[k, mu, nu] by probing c with symmetric unit densities
    L = np.zeros((om.M, nbf, nbf))
    for mu in range(nbf):
        for nu in range(mu, nbf):
            E = np.zeros((nbf, nbf)); E[mu, nu] = 1.0; E[nu, mu] = 1.0
            cvec = om.esp(E, pairs=pr)
            if mu == nu:
                L[:, mu, mu] = cvec
            else:
                L[:, mu, nu] = L[:, nu, mu] = cvec / 2.0
    c = om.esp(water.P, pairs=pr)
    assert np.allclose(c, np.einsum("kmn,mn->k", L, water.P), rtol=1e-13, atol=1e-15)
    rng = np.random.default_rng(3)
    q = rng.normal(size=om.M)
    F = om.fock(q, pairs=pr)
    assert np.allclose(F, np.einsum("k,kmn->mn", q, L), rtol=1e-12, atol=1e-13)
    assert np.array_equal(F, F.T) or np.abs(F - F.T).max() < 1e-14
    lhs, rhs = q @ c, np.sum(water.P * F)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_screening_error_is_negligible(water, water_oracle):
    om = water_oracle
    bz = om.bz()
    A = om.amat()
    c_s = om.esp(water.P)
    c_u = om.esp(water.P, pairs=om.pairs(water.P, thresh=0.0))
    q_s = om.solve_dense(bz + c_s, A)
    q_u = om.solve_dense(bz + c_u, A)
    E_s = om.energy(bz, c_s, q_s, A @ q_s)
    E_u = om.energy(bz, c_u, q_u, A @ q_u)
    assert abs(E_s - E_u) < 1e-10


def test_energy_identities(water, water_oracle):
    om = water_oracle
    sol = O.full_solution(om, water.P)
    v = sol["bz"] + sol["c"]
    assert abs(sol["E"] - 0.5 * v @ sol["q"]) <= 1e-12 * abs(sol["E"])
    assert sol["E"] < 0
    rng = np.random.default_rng(9)
    for _ in range(5):
        dq = rng.normal(size=om.M) * 1e-2
        Eq = om.energy(sol["bz"], sol["c"], sol["q"] + dq, sol["A"] @ (sol["q"] + dq))
        gap = Eq - sol["E"]
        assert gap >= 0
        assert abs(gap - 0.5 / om.f * dq @ (sol["A"] @ dq)) <= 1e-10 * abs(gap) + 1e-15


def test_pcg_matches_cholesky(water, water_oracle):
    om = water_oracle
    sol = O.full_solution(om, water.P)
    b = -om.f * (sol["bz"] + sol["c"])
    for kind in ("none", "jacobi", "rbj"):
        x, it = om.pcg(b, 1e-10, precond=kind, block=32, seed=104, A=sol["A"])
        assert np.linalg.norm(sol["A"] @ x - b) < 1e-10
        assert np.abs(x - sol["q"]).max() <= 1e-7 * np.abs(sol["q"]).max()


def test_rbj_limits(water, water_oracle):
    om = water_oracle
    sol = O.full_solution(om, water.P)
    b = -om.f * (sol["bz"] + sol["c"])
    _, it_j = om.pcg(b, 1e-10, precond="jacobi", A=sol["A"])
    _, it_1 = om.pcg(b, 1e-10, precond="rbj", block=1, seed=5, A=sol["A"])
    assert it_1 == it_j                      # block size 1 is Jacobi
    _, it_M = om.pcg(b, 1e-10, precond="rbj", block=om.M, seed=5, A=sol["A"])
    assert it_M == 1                          # block size M: exact inverse, one step (Sec. 4b-ii)


def test_rbj_partition_is_a_partition(water_oracle):
    om = water_oracle
    for l in (1, 7, 32, 100, om.M):
        perm, off = om.rbj_partition(l, 1234)
        assert sorted(perm.tolist()) == list(range(om.M))
        sizes = np.diff(off)
        assert np.all(sizes[:-1] == min(l, om.M)) and 1 <= sizes[-1] <= l
        for b in range(len(sizes)):
            blk = perm[off[b]:off[b + 1]]
            assert np.all(np.diff(blk) > 0)


def test_rbj_block_holds_strongest_couplings(water_oracle):
    om = water_oracle
    l = 20
    perm, off = om.rbj_partition(l, 77)
    blk = perm[off[0]:off[1]]
    # the first block: some member (the pivot) has its l-1 largest |A_kl| inside the block
    ok = False
    for k in blk:
        row = np.abs(om.arow(int(k)))
        row[k] = -1
        top = np.argsort(-row, kind="stable")[: l - 1]
        if set(top.tolist()) | {int(k)} == set(blk.tolist()):
            ok = True
    assert ok


def test_dynamic_threshold_closed_form():
    assert O.dynamic_threshold(-1.0) == 1.0
    for e in (1e-2, 1e-4, 3.2e-7):
        d = O.dynamic_threshold(e)
        assert abs(0.01 * d ** 1.07 - 1e-3 * e) <= 1e-12 * 1e-3 * e
    assert O.dynamic_threshold(1e3) == 1.0
    assert O.dynamic_threshold(1e-30) == 1e-10


# ------------------------------------------------------------------ gradient

def energy_at(sysobj, pr, keep, xyz=None, r_override=None, P=None):
    om = O.OracleMol(sysobj.xyz if xyz is None else xyz, sysobj.Z, sysobj.radius, sysobj.sph_dirs,
                     sysobj.sph_w, sysobj.basis, keep_idx=keep, r_override=r_override)
    P = sysobj.P if P is None else P
    bz = om.bz()
    c = om.esp(P, pairs=pr)
    A = om.amat()
    q = om.solve_dense(bz + c, A)
    return om.energy(bz, c, q, A @ q)


@pytest.fixture(scope="module")
def water_grad(water, water_oracle):
    om = water_oracle
    pr = om.pairs(water.P)
    sol = O.full_solution(om, water.P)
    g = om.grad_terms(water.P, sol["q"], pairs=pr)
    return om, pr, sol, g


def test_gradient_zero_net_force(water_grad):
    om, pr, sol, g = water_grad
    for t in range(4):
        tot = g["g_nuc_terms"][t].sum(0) + g["g_surf_terms"][t].sum(0)
        scale = np.abs(g["g_nuc_terms"][t]).sum() + np.abs(g["g_surf_terms"][t]).sum()
        assert np.abs(tot).max() <= 1e-12 * max(scale, 1e-300)


def test_gradient_nuclear_fd(water, water_grad):
    om, pr, sol, g = water_grad
    total = om.total_nuclear_gradient(g["g_nuc"], g["g_surf"])
    h = 1e-4
    for I_ in range(om.N):
        for d in range(3):
            xp = om.xyz.copy(); xp[I_, d] += h
            xm = om.xyz.copy(); xm[I_, d] -= h
            fd = (energy_at(water, pr, om.keep_idx, xyz=xp) - energy_at(water, pr, om.keep_idx, xyz=xm)) / (2 * h)
            assert abs(fd - total[I_, d]) <= max(1e-7, 1e-5 * abs(total[I_, d])), (I_, d, fd, total[I_, d])


def test_gradient_surface_fd(water, water_grad):
    om, pr, sol, g = water_grad
    rng = np.random.default_rng(105)
    h = 1e-4
    for k in rng.choice(om.M, 6, replace=False):
        for d in range(3):
            rp = om.r.copy(); rp[k, d] += h
            rm = om.r.copy(); rm[k, d] -= h
            fd = (energy_at(water, pr, om.keep_idx, r_override=rp) -
                  energy_at(water, pr, om.keep_idx, r_override=rm)) / (2 * h)
            assert abs(fd - g["g_surf"][k, d]) <= max(1e-7, 1e-5 * abs(g["g_surf"][k, d])), (k, d)


def test_gradient_mirror_symmetry_without_density(water, water_oracle):
    om = water_oracle
    P0 = np.zeros((om.nbf, om.nbf))
    bz = om.bz()
    A = om.amat()
    q = om.solve_dense(bz, A)
    g = om.grad_terms(P0, q)
    tot = om.total_nuclear_gradient(g["g_nuc"], g["g_surf"])
    # x -> -x swaps the two H atoms: F_x flips sign, F_y, F_z equal; O has F_x = 0
    assert abs(tot[0, 0]) <= 1e-10
    assert abs(tot[1, 0] + tot[2, 0]) <= 1e-10
    assert abs(tot[1, 1] - tot[2, 1]) <= 1e-10


# ------------------------------------------------- d shells (sd, pd, dd classes)

@pytest.fixture(scope="module")
def small():
    s = I.small_protein(6, 50, seed=3)
    om = O.mol_from_system(s)
    return s, om


def test_small_protein_classes_and_adjoint(small):
    s, om = small
    pr = om.pairs()
    counts = np.bincount(pr["cls"], minlength=6)
    assert np.all(counts > 0)  # every class ss..dd present
    rng = np.random.default_rng(1)
    q = rng.normal(size=om.M)
    c = om.esp(s.P, pairs=pr)
    F = om.fock(q, pairs=pr)
    assert abs(q @ c - np.sum(s.P * F)) <= 1e-12 * abs(q @ c)
    assert np.abs(F - F.T).max() <= 1e-12 * np.abs(F).max()


def test_small_protein_gradient(small):
    s, om = small
    pr = om.pairs(s.P)
    sol = O.full_solution(om, s.P)
    g = om.grad_terms(s.P, sol["q"], pairs=pr)
    for t in range(4):
        tot = g["g_nuc_terms"][t].sum(0) + g["g_surf_terms"][t].sum(0)
        scale = np.abs(g["g_nuc_terms"][t]).sum() + np.abs(g["g_surf_terms"][t]).sum()
        assert np.abs(tot).max() <= 1e-11 * max(scale, 1e-300)
    total = om.total_nuclear_gradient(g["g_nuc"], g["g_surf"])
    h = 1e-4
    rng = np.random.default_rng(7)
    for I_ in rng.choice(om.N, 3, replace=False):
        d = int(rng.integers(3))
        xp = om.xyz.copy(); xp[I_, d] += h
        xm = om.xyz.copy(); xm[I_, d] -= h
        fd = (energy_at(s, pr, om.keep_idx, xyz=xp) - energy_at(s, pr, om.keep_idx, xyz=xm)) / (2 * h)
        assert abs(fd - total[I_, d]) <= max(1e-7, 1e-5 * abs(total[I_, d])), (I_, d, fd, total[I_, d])


# ------------------------------------------------------------------ octree partition
def _morton(ix, iy, iz, levels):
    """Z-order code of integer cell coordinates, most significant level first."""
    code = 0
    for lev in range(levels - 1, -1, -1):
        code = (code << 3) | ((ix >> lev) & 1) | (((iy >> lev) & 1) << 1) | (((iz >> lev) & 1) << 2)
    return code


def test_octree_cube_corners_octant_order():
    # octant o holds the corner with x > 0 iff bit 0, y > 0 iff bit 1, z > 0 iff bit 2
    rng = np.random.default_rng(3)
    corners = np.array([[sx, sy, sz] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)], float)
    order = rng.permutation(8)
    r = corners[order]
    perm, off = O.octree_partition(r, 1)
    assert np.array_equal(off, np.arange(9))
    octant = (r[perm, 0] > 0) + 2 * (r[perm, 1] > 0) + 4 * (r[perm, 2] > 0)
    assert np.array_equal(octant, np.arange(8))


def test_octree_regular_grid_is_z_order():
    # a 4x4x4 grid with one point per leaf: depth-first octant order is the Morton order
    g = np.array([[x, y, z] for x in range(4) for y in range(4) for z in range(4)], float)
    rng = np.random.default_rng(8)
    g = g[rng.permutation(len(g))]
    perm, off = O.octree_partition(g, 1)
    assert np.array_equal(off, np.arange(65))
    codes = [_morton(int(x), int(y), int(z), 2) for x, y, z in g]
    assert np.array_equal(perm, np.argsort(codes, kind="stable"))
    # leaves of 8: the 2x2x2 blocks of the grid, in Morton order of the block, members ascending
    perm8, off8 = O.octree_partition(g, 8)
    assert np.array_equal(off8, 8 * np.arange(9))
    for b in range(8):
        idx = perm8[off8[b]:off8[b + 1]]
        assert np.all(np.diff(idx) > 0)
        cell = {(int(x) // 2, int(y) // 2, int(z) // 2) for x, y, z in g[idx]}
        assert len(cell) == 1
        (cx, cy, cz), = cell
        assert _morton(cx, cy, cz, 1) == b


def test_octree_clusters_and_limits():
    rng = np.random.default_rng(5)
    centres = np.array([[-5.0, -5.0, -5.0], [5.0, -5.0, 5.0], [-5.0, 5.0, 5.0], [5.0, 5.0, -5.0]])
    sizes = [5, 3, 5, 4]
    r = np.concatenate([c + 0.1 * rng.normal(size=(n, 3)) for c, n in zip(centres, sizes)])
    sh = rng.permutation(len(r))
    r = r[sh]
    label = np.repeat(np.arange(4), sizes)[sh]
    perm, off = O.octree_partition(r, 5)
    blocks = [set(label[perm[off[b]:off[b + 1]]].tolist()) for b in range(len(off) - 1)]
    assert len(blocks) == 4 and all(len(s) == 1 for s in blocks)
    # octant order of the cluster centres: (-,-,-)=0, (+,+,-)=3, (+,-,+)=5, (-,+,+)=6
    assert [s.pop() for s in blocks] == [0, 3, 1, 2]
    # leaf_max >= M: one block of every point, ascending
    perm, off = O.octree_partition(r, len(r))
    assert np.array_equal(off, [0, len(r)]) and np.array_equal(perm, np.arange(len(r)))
    # coincident points cannot be split: runs of leaf_max after the depth limit
    perm, off = O.octree_partition(np.zeros((7, 3)), 3)
    assert np.array_equal(off, [0, 3, 6, 7]) and np.array_equal(perm, np.arange(7))


def test_octree_leaves_are_disjoint_cells():
    s = I.small_protein(10, 74, seed=11)
    om = O.mol_from_system(s)
    for leaf in (800, 100, 37):
        perm, off = om.octree_partition(leaf)
        assert sorted(perm.tolist()) == list(range(om.M))
        sizes = np.diff(off)
        assert sizes.min() >= 1 and sizes.max() <= leaf
        boxes = [(om.r[perm[off[b]:off[b + 1]]].min(0), om.r[perm[off[b]:off[b + 1]]].max(0))
                 for b in range(len(sizes))]
        # points of different leaves lie in different octree cells: their bounding boxes
        # are separated (touching at most) along some axis
        for a in range(len(boxes)):
            for b in range(a + 1, len(boxes)):
                (la, ha), (lb, hb) = boxes[a], boxes[b]
                assert np.any((ha <= lb) | (hb <= la)), (leaf, a, b)


def test_octree_block_jacobi_limits(water, water_oracle):
    om = water_oracle
    sol = O.full_solution(om, water.P)
    b = -om.f * (sol["bz"] + sol["c"])
    x, it = om.pcg(b, 1e-10, precond="octree", block=32, A=sol["A"])
    assert np.linalg.norm(sol["A"] @ x - b) < 1e-10
    _, it_M = om.pcg(b, 1e-10, precond="octree", block=om.M, A=sol["A"])
    assert it_M == 1                          # one leaf: the exact inverse


# ------------------------------------------------------------------ threshold policies
def test_threshold_policies_follow_sec_4b_i():
    errs = [None, 0.3, 2e-2, 1.2e-3, 1e-3, 4e-3, 2e-4, 1e-6]
    assert O.threshold_schedule("fixed", errs, delta=1e-6) == [1e-6] * len(errs)
    # 2-delta: delta_1 = 1e4 delta_2 until the DIIS error reaches 1e-3, then delta_2 for good
    two = O.threshold_schedule("two_delta", errs, delta=1e-6, scale=1e4, switch_at=1e-3)
    assert two == [1e-2, 1e-2, 1e-2, 1e-2, 1e-6, 1e-6, 1e-6, 1e-6]
    dyn = O.threshold_schedule("dynamic", errs)
    assert dyn[0] == 1.0                      # first SCF step: delta = 1
    for e, d in zip(errs[1:], dyn[1:]):
        # Eq. 21 at the chosen delta predicts an error 1e-3 times the previous DIIS error
        assert 0.01 * d ** 1.07 == pytest.approx(1e-3 * e, rel=1e-12)
