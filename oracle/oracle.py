"""Python face of the FP64 oracle for the C-PCM / ISWIG path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  The arithmetic
lives in ``pcm_oracle.c`` (plain C, FP64, OpenMP); this wrapper marshals
arguments and uses numpy/scipy for the dense linear algebra (Cholesky solve,
block inverses) of Sec. 2, Eq. 1 and Sec. 4b of the paper.

Readings of the paper that this oracle takes:
* Eq. 3 constant: A_kk = sqrt(2/pi) zeta_k / S_k (the r -> 0 limit of Eq. 2
  for k = l), passed as ``diag_const``;
* sphere weights sum to 4 pi, so zeta_k = zeta0 / (rho_I sqrt(w_k)) (Eq. 7);
* in Eq. 9, R_J inside the erf terms is the cavity radius of atom J and the
  product runs over all atoms except the owner of point k;
* f = (eps - 1)/(eps + k) with k = 0 (Eq. 1);
* Eq. 20 residual: Euclidean norm of A q - b, absolute, in atomic units;
* Eq. 21 dynamic threshold: 0.01 delta^1.07 = 1e-3 e_prev, i.e.
  delta = (0.1 e_prev)^(1/1.07), clamped to [1e-10, 1], delta = 1 at the
  first SCF step;
* 2-delta switching (Sec. 4b-i): the switch to the tight threshold is made once,
  at the first step whose previous DIIS error is at or below 1e-3;
* octree block Jacobi (Sec. 4b-ii, the comparison scheme): the cell rules in
  ``octree_partition``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DIAG_CONST = math.sqrt(2.0 / math.pi)


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
                               "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        _lib.or_pairs.restype = ctypes.c_long
        _lib.or_surface.restype = ctypes.c_int
        _lib.or_rbj_partition.restype = ctypes.c_int
        _lib.or_rbj_partition.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def boys(mmax: int, T: float) -> np.ndarray:
    F = np.zeros(mmax + 1)
    lib().or_boys(ctypes.c_int(mmax), ctypes.c_double(T), _p(F))
    return F


def prim_block(la, lb, A, ea, B, eb, C, zeta) -> np.ndarray:
    """[chi_a|erf(zeta|r-C|)/|r-C||chi_b] for all Cartesian components (unnormalised primitives)."""
    out = np.zeros(ncart(la) * ncart(lb))
    lib().or_prim_block(ctypes.c_int(la), ctypes.c_int(lb), _p(_f64(A)), ctypes.c_double(ea), _p(_f64(B)),
                        ctypes.c_double(eb), _p(_f64(C)), ctypes.c_double(zeta), _p(out))
    return out.reshape(ncart(la), ncart(lb))


def prim_block_deriv(la, lb, A, ea, B, eb, C, zeta):
    na, nb = ncart(la), ncart(lb)
    dA = np.zeros(3 * na * nb)
    dB = np.zeros(3 * na * nb)
    lib().or_prim_block_deriv(ctypes.c_int(la), ctypes.c_int(lb), _p(_f64(A)), ctypes.c_double(ea), _p(_f64(B)),
                              ctypes.c_double(eb), _p(_f64(C)), ctypes.c_double(zeta), _p(dA), _p(dB))
    return dA.reshape(3, na, nb), dB.reshape(3, na, nb)


def dynamic_threshold(e_prev: float) -> float:
    """Eq. 21 used as in Sec. 4b-i: pick delta with 0.01 delta^1.07 = 1e-3 e_prev."""
    if e_prev is None or e_prev < 0:
        return 1.0
    if e_prev == 0:
        return 1e-10
    d = (0.1 * e_prev) ** (1.0 / 1.07)
    return min(1.0, max(1e-10, d))


def threshold_schedule(kind, diis_errors, delta=1e-6, scale=1e4, switch_at=1e-3):
    """CG thresholds of the SCF steps whose previous DIIS errors are ``diis_errors`` (None
    or a negative value for the first step), Sec. 4b-i:

    * fixed: delta at every step;
    * two_delta: the loose scale * delta until a previous DIIS error is at or below
      switch_at, the tight delta from that step on (reading: the switch is made once);
    * dynamic: Eq. 21 through ``dynamic_threshold``.
    """
    out, switched = [], False
    for e in diis_errors:
        first = e is None or e < 0
        if kind == "fixed":
            out.append(delta)
        elif kind == "two_delta":
            if not first and e <= switch_at:
                switched = True
            out.append(delta if switched else scale * delta)
        elif kind == "dynamic":
            out.append(dynamic_threshold(-1.0 if first else e))
        else:
            raise ValueError(f"unknown threshold policy {kind!r}")
    return out


OCTREE_MAX_DEPTH = 40


def octree_partition(r, leaf_max):
    """Spatial octree partition of points r[M, 3] for block Jacobi (the comparison
    preconditioner of Sec. 4b-ii): a leaf holds at most ``leaf_max`` points.

    Reading (the paper names the scheme only): the root is the cube centred on the
    midpoint of the bounding box with half-side half the largest extent; a cell with more
    than ``leaf_max`` points is cut into 8 octants at its centre, a point going to octant
    (x >= cx) + 2 (y >= cy) + 4 (z >= cz); children are visited depth first in octant
    order and empty cells are dropped; a leaf stores its points in ascending index.  A
    cell still too full at depth 40 (coincident points) is cut into consecutive runs of
    ``leaf_max`` points.  Returns (perm, off) like the randomized partition.
    """
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    M = r.shape[0]
    if M < 1 or leaf_max < 1:
        raise ValueError("octree_partition needs M >= 1 and leaf_max >= 1")
    lo, hi = r.min(axis=0), r.max(axis=0)
    centre = (lo + hi) * 0.5
    half = float((hi - lo).max()) * 0.5
    leaves = []

    def visit(idx, c, h, depth):
        if idx.size <= leaf_max:
            leaves.append(idx)
            return
        if depth == OCTREE_MAX_DEPTH:
            for s in range(0, idx.size, leaf_max):
                leaves.append(idx[s:s + leaf_max])
            return
        octant = ((r[idx, 0] >= c[0]).astype(np.int64) + 2 * (r[idx, 1] >= c[1]) + 4 * (r[idx, 2] >= c[2]))
        for o in range(8):
            sub = idx[octant == o]
            if sub.size == 0:
                continue
            cc = np.array([c[d] + (0.5 * h if (o >> d) & 1 else -0.5 * h) for d in range(3)])
            visit(sub, cc, 0.5 * h, depth + 1)

    visit(np.arange(M, dtype=np.int64), centre, half, 0)
    perm = np.concatenate(leaves).astype(np.int32)
    off = np.zeros(len(leaves) + 1, np.int32)
    off[1:] = np.cumsum([lf.size for lf in leaves])
    return perm, off


class OracleMol:
    """Surface, basis and pair lists of one solute, all in FP64 on the host."""

    def __init__(self, xyz, Z, radius, sph_dirs, sph_w, basis, eps=78.39, k_factor=0.0, zeta0=4.9,
                 switch_thresh=1e-8, schwarz_thresh=1e-12, diag_const=DIAG_CONST, keep_idx=None, r_override=None):
        L = lib()
        self.xyz = _f64(xyz).reshape(-1, 3)
        self.N = self.xyz.shape[0]
        self.Z = _f64(Z)
        self.rad = _f64(radius)
        self.dirs = _f64(sph_dirs).reshape(-1, 3)
        self.w = _f64(sph_w)
        self.nsph = self.dirs.shape[0]
        self.eps, self.k_factor = float(eps), float(k_factor)
        self.f = (self.eps - 1.0) / (self.eps + self.k_factor)
        self.zeta0, self.switch_thresh, self.schwarz_thresh = zeta0, switch_thresh, schwarz_thresh
        self.diag_const = diag_const
        # --- surface (Eqs. 3, 7, 9) ---
        nr = self.N * self.nsph
        r = np.zeros(3 * nr); z = np.zeros(nr); S = np.zeros(nr); Akk = np.zeros(nr); keep = np.zeros(nr, np.int32)
        L.or_surface(ctypes.c_int(self.N), _p(self.xyz), _p(self.rad), ctypes.c_int(self.nsph), _p(self.dirs),
                     _p(self.w), ctypes.c_double(zeta0), ctypes.c_double(switch_thresh), ctypes.c_double(diag_const),
                     _p(r), _p(z), _p(S), _p(Akk), _p(keep))
        if keep_idx is None:
            keep_idx = np.nonzero(keep)[0]
        self.keep_idx = np.asarray(keep_idx, dtype=np.int64)
        self.r = r.reshape(-1, 3)[self.keep_idx].copy()
        if r_override is not None:
            self.r = _f64(r_override).reshape(-1, 3).copy()
        self.zeta = z[self.keep_idx].copy()
        self.S = S[self.keep_idx].copy()
        self.Akk = Akk[self.keep_idx].copy()
        self.owner = _i32(self.keep_idx // self.nsph)
        self.sph_idx = _i32(self.keep_idx % self.nsph)
        if r_override is not None:
            self._recompute_switching()
        self.M = self.r.shape[0]
        # --- basis (Eqs. 11-12) ---
        b = basis
        self.sl, self.snp, self.soff, self.satom = _i32(b.shell_l), _i32(b.shell_nprim), _i32(b.shell_off), _i32(b.shell_atom)
        self.pexp, self.pcoef = _f64(b.prim_exp), _f64(b.prim_coef)
        self.ns = self.sl.shape[0]
        nc = (self.sl + 1) * (self.sl + 2) // 2
        self.bf_off = _i32(np.concatenate([[0], np.cumsum(nc)[:-1]]))
        self.nbf = int(nc.sum())
        self.cn_off = _i32(np.concatenate([[0], np.cumsum(nc * self.snp)[:-1]]))
        self.cn = np.zeros(int((nc * self.snp).sum()))
        L.or_norm_coefs(ctypes.c_int(self.ns), _p(self.sl), _p(self.snp), _p(self.soff), _p(self.pexp),
                        _p(self.pcoef), _p(self.cn_off), _p(self.cn))

    def _recompute_switching(self):
        """S_k and A_kk for explicitly placed points (Eq. 9, Eq. 3), same erfc form as the C code."""
        from scipy.special import erfc
        S = np.ones(self.r.shape[0])
        for k in range(self.r.shape[0]):
            I = self.owner[k]
            for J in range(self.N):
                if J == I:
                    continue
                d = math.sqrt(float(((self.r[k] - self.xyz[J]) ** 2).sum()))
                S[k] *= 0.5 * (erfc(self.zeta[k] * (self.rad[J] - d)) + erfc(self.zeta[k] * (self.rad[J] + d)))
        self.S = S
        self.Akk = self.diag_const * self.zeta / S

    # ------------------------------------------------------------------ pairs
    def pairs(self, P=None, thresh=None):
        """Screened primitive-pair list (Eq. 15; Eq. 18 with P).  Returns dict of arrays."""
        L = lib()
        thresh = self.schwarz_thresh if thresh is None else thresh
        Pp = None if P is None else _f64(P)
        args = [ctypes.c_int(self.ns), _p(self.sl), _p(self.snp), _p(self.soff), _p(self.satom), _p(self.pexp),
                _p(self.cn_off), _p(self.cn), _p(self.xyz.ravel()), _p(self.bf_off), ctypes.c_int(self.nbf),
                _p(Pp), ctypes.c_double(thresh)]
        n = L.or_pairs(*args, None, None, None, None, None, None)
        out = {k: np.zeros(n, np.int32) for k in ("cls", "a", "b", "i", "j")}
        out["w"] = np.zeros(n)
        L.or_pairs(*args, _p(out["cls"]), _p(out["a"]), _p(out["b"]), _p(out["i"]), _p(out["j"]), _p(out["w"]))
        return out

    def _basis_args(self):
        return [ctypes.c_int(self.ns), _p(self.sl), _p(self.snp), _p(self.soff), _p(self.satom), _p(self.pexp),
                _p(self.cn_off), _p(self.cn), _p(self.xyz.ravel()), _p(self.bf_off), ctypes.c_int(self.nbf)]

    # --------------------------------------------------------------- integrals
    def esp(self, P, kidx=None, pairs=None):
        """c_k = sum P L^k (Eqs. 5-6) for the points kidx (default all)."""
        P = _f64(P)
        pr = self.pairs(P) if pairs is None else pairs
        kk = None if kidx is None else _i32(kidx)
        nk = self.M if kk is None else kk.shape[0]
        out = np.zeros(nk)
        r = _f64(self.r.ravel())
        lib().or_esp(*self._basis_args(), _p(P), ctypes.c_long(pr["a"].shape[0]), _p(pr["a"]), _p(pr["b"]),
                     _p(pr["i"]), _p(pr["j"]), _p(pr["w"]), ctypes.c_int(self.M), _p(r), _p(self.zeta),
                     ctypes.c_int(nk), _p(kk), _p(out))
        return out

    def fock(self, q, shell_pairs=None, pairs=None):
        """F = sum_k q_k L^k (Eq. 10); optionally only for a set of (a, b) shell pairs."""
        pr = self.pairs() if pairs is None else pairs
        sel = None
        if shell_pairs is not None:
            sel = np.zeros(self.ns * self.ns, np.uint8)
            for a, b in shell_pairs:
                sel[a * self.ns + b] = 1
        F = np.zeros((self.nbf, self.nbf))
        r = _f64(self.r.ravel())
        L = lib()
        L.or_fock(*self._basis_args(), ctypes.c_long(pr["a"].shape[0]), _p(pr["a"]), _p(pr["b"]), _p(pr["i"]),
                  _p(pr["j"]), ctypes.c_int(self.M), _p(r), _p(self.zeta), _p(_f64(q)), _p(sel), _p(F))
        return F

    def bz(self):
        out = np.zeros(self.M)
        lib().or_bz(ctypes.c_int(self.M), _p(_f64(self.r.ravel())), _p(self.zeta), ctypes.c_int(self.N),
                    _p(self.xyz.ravel()), _p(self.Z), _p(out))
        return out

    def amat(self):
        A = np.zeros((self.M, self.M))
        lib().or_amat(ctypes.c_int(self.M), _p(_f64(self.r.ravel())), _p(self.zeta), _p(self.Akk), _p(A))
        return A

    def arow(self, k):
        row = np.zeros(self.M)
        lib().or_arow(ctypes.c_int(self.M), ctypes.c_int(k), _p(_f64(self.r.ravel())), _p(self.zeta),
                      _p(self.Akk), _p(row))
        return row

    def matvec(self, x, kidx=None):
        kk = None if kidx is None else _i32(kidx)
        nk = self.M if kk is None else kk.shape[0]
        y = np.zeros(nk)
        lib().or_matvec(ctypes.c_int(self.M), _p(_f64(self.r.ravel())), _p(self.zeta), _p(self.Akk),
                        _p(_f64(x)), ctypes.c_int(nk), _p(kk), _p(y))
        return y

    # ------------------------------------------------------------------ solve
    def solve_dense(self, v, A=None):
        """q = -f A^-1 v by Cholesky (Eq. 1)."""
        import scipy.linalg as sla
        A = self.amat() if A is None else A
        cf = sla.cho_factor(A, lower=True)
        return -self.f * sla.cho_solve(cf, v)

    def energy(self, bz, c, q, Aq=None):
        """Eq. 13: (Bz)^T q + c^T q + 1/(2f) q^T A q."""
        Aq = self.matvec(q) if Aq is None else Aq
        return float(bz @ q + c @ q + 0.5 / self.f * (q @ Aq))

    def rbj_partition(self, l, seed):
        perm = np.zeros(self.M, np.int32)
        off = np.zeros(self.M + 1, np.int32)
        nb = lib().or_rbj_partition(self.M, _p(_f64(self.r.ravel())), _p(self.zeta), int(l), int(seed),
                                    _p(perm), _p(off))
        return perm, off[: nb + 1].copy()

    def octree_partition(self, leaf_max):
        return octree_partition(self.r, leaf_max)

    def preconditioner(self, kind="jacobi", block=100, seed=0, A=None):
        """Return a function z = C r for kind in {none, jacobi, rbj, octree} (Sec. 4b-ii);
        for octree, ``block`` is the largest leaf."""
        if kind == "none":
            return lambda r: r.copy()
        if kind == "jacobi":
            d = 1.0 / self.Akk
            return lambda r: d * r
        if kind == "octree":
            perm, off = self.octree_partition(block)
        elif kind == "rbj":
            perm, off = self.rbj_partition(block, seed)
        else:
            raise ValueError(f"unknown preconditioner {kind!r}")
        blocks = []
        for b in range(off.shape[0] - 1):
            idx = perm[off[b]:off[b + 1]]
            if A is not None:
                Ab = A[np.ix_(idx, idx)]
            else:
                Ab = np.stack([self.arow(int(k))[idx] for k in idx])
            blocks.append((idx, np.linalg.inv(Ab)))

        def apply(r):
            z = np.zeros_like(r)
            for idx, Ainv in blocks:
                z[idx] = Ainv @ r[idx]
            return z
        return apply

    def pcg(self, b, tol, precond="jacobi", block=100, seed=0, x0=None, max_iter=10000, A=None):
        """Preconditioned CG on A x = b, stop when ||A x - b||_2 < tol (Eq. 20)."""
        mv = (lambda x: A @ x) if A is not None else self.matvec
        C = self.preconditioner(precond, block, seed, A)
        x = np.zeros_like(b) if x0 is None else x0.copy()
        r = b - mv(x) if x0 is not None else b.copy()
        it = 0
        if np.linalg.norm(r) < tol:
            return x, it
        z = C(r)
        p = z.copy()
        rz = r @ z
        while it < max_iter:
            Ap = mv(p)
            alpha = rz / (p @ Ap)
            x += alpha * p
            r -= alpha * Ap
            it += 1
            if np.linalg.norm(r) < tol:
                break
            z = C(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        return x, it

    # --------------------------------------------------------------- gradient
    def grad_terms(self, P, q, pairs=None):
        """Eq. 14 terms: dict with g_nuc/g_surf per term (B, c, A_off, A_diag) and totals."""
        P = _f64(P)
        pr = self.pairs(P) if pairs is None else pairs
        gn = np.zeros(4 * 3 * self.N)
        gs = np.zeros(4 * 3 * self.M)
        lib().or_grad(*self._basis_args(), _p(self.Z), _p(self.rad), ctypes.c_int(self.N), _p(P),
                      ctypes.c_long(pr["a"].shape[0]), _p(pr["a"]), _p(pr["b"]), _p(pr["i"]), _p(pr["j"]),
                      _p(pr["w"]), ctypes.c_int(self.M), _p(_f64(self.r.ravel())), _p(self.zeta), _p(self.Akk),
                      _p(self.owner), _p(_f64(q)), ctypes.c_double(self.f), _p(gn), _p(gs))
        gn = gn.reshape(4, self.N, 3)
        gs = gs.reshape(4, self.M, 3)
        return {"g_nuc_terms": gn, "g_surf_terms": gs, "g_nuc": gn.sum(0), "g_surf": gs.sum(0)}

    def grad_surface_points(self, P, q, kidx, pairs=None):
        """g_surf (sum of the Eq. 14 terms) for the listed points only: shape [len(kidx), 3]."""
        P = _f64(P)
        pr = self.pairs(P) if pairs is None else pairs
        kk = _i32(kidx)
        out = np.zeros(3 * kk.shape[0])
        lib().or_grad_points(*self._basis_args(), _p(self.Z), _p(self.rad), ctypes.c_int(self.N), _p(P),
                             ctypes.c_long(pr["a"].shape[0]), _p(pr["a"]), _p(pr["b"]), _p(pr["i"]), _p(pr["j"]),
                             _p(pr["w"]), ctypes.c_int(self.M), _p(_f64(self.r.ravel())), _p(self.zeta),
                             _p(self.Akk), _p(self.owner), _p(_f64(q)), ctypes.c_double(self.f),
                             ctypes.c_int(kk.shape[0]), _p(kk), _p(out))
        return out.reshape(-1, 3)

    def total_nuclear_gradient(self, g_nuc, g_surf):
        """Points move with their atom: total_I = g_nuc[I] + sum_{k in I} g_surf[k]."""
        tot = g_nuc.copy()
        np.add.at(tot, self.owner, g_surf)
        return tot


def mol_from_system(sysobj, **kw) -> OracleMol:
    return OracleMol(sysobj.xyz, sysobj.Z, sysobj.radius, sysobj.sph_dirs, sysobj.sph_w, sysobj.basis,
                     eps=sysobj.eps, zeta0=sysobj.zeta0, **kw)


def full_solution(om: OracleMol, P):
    """bz, c, q (dense Cholesky), E for one molecule: the whole path in FP64."""
    bz = om.bz()
    c = om.esp(P)
    A = om.amat()
    q = om.solve_dense(bz + c, A)
    E = om.energy(bz, c, q, A @ q)
    return {"bz": bz, "c": c, "q": q, "E": E, "A": A}
