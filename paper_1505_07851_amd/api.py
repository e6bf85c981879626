"""Thin Python face of the C ABI: argument marshalling only, every step runs in libpcm.so.

Device arrays are torch tensors (float64, contiguous, on the context's GPU); host inputs
(geometry, basis, sphere rule) are numpy arrays.  Work is enqueued on the torch stream that
was current when the Context was created.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib as C


class PCMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{C.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _hp(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dp(t):
    """Device pointer of a float64/int32 contiguous GPU tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t, n=None, name="array"):
    import torch
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return t


class Context:
    """Library context: model parameters, device, stream."""

    def __init__(self, eps=78.39, k_factor=0.0, zeta0=4.9, switch_thresh=1e-8, schwarz_thresh=1e-12,
                 diag_const=None, precision="fp64", stream=None, device=None, autotune=True,
                 dp_thresh=1e-6):
        import torch
        self.lib = C.lib()
        if device is not None:
            torch.cuda.set_device(device)
        self.device = torch.device("cuda", torch.cuda.current_device())
        p = C.pcm_params()
        self.lib.pcm_default_params(ctypes.byref(p))
        p.eps, p.k_factor, p.zeta0 = eps, k_factor, zeta0
        p.switch_thresh, p.schwarz_thresh = switch_thresh, schwarz_thresh
        if diag_const is not None:
            p.diag_const = diag_const
        p.precision = {"fp64": C.PCM_FP64, "mixed": C.PCM_MIXED, "dynamic": C.PCM_DYNAMIC}[precision]
        p.dp_thresh = float(dp_thresh)
        p.autotune = 1 if autotune else 0
        self.params = p
        self.precision = precision
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.pcm_create(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != C.PCM_OK:
            raise PCMError(st, "pcm_create failed")
        self.h = h
        self.f = (eps - 1.0) / (eps + k_factor)

    def check(self, st):
        if st != C.PCM_OK:
            raise PCMError(st, self.lib.pcm_last_error(self.h).decode())

    def profile(self, on=True):
        """Enable (clearing old records) or disable per-kernel HIP-event timing."""
        self.check(self.lib.pcm_profile_enable(self.h, 1 if on else 0))

    def profile_read(self):
        """{kernel name: {"ms": total, "launches": n, "work": units}} since the last enable."""
        n = self.lib.pcm_profile_collect(self.h)
        if n < 0:
            raise PCMError(C.PCM_E_HIP, "profile collection failed")
        out = {}
        buf = ctypes.create_string_buffer(64)
        for i in range(n):
            ms, cnt, work = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
            self.check(self.lib.pcm_profile_entry(self.h, i, buf, 64, ctypes.byref(ms), ctypes.byref(cnt),
                                                  ctypes.byref(work)))
            out[buf.value.decode()] = {"ms": ms.value, "launches": cnt.value, "work": work.value}
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.pcm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Molecule:
    """Surface + screened pair lists of one solute (pcm_build_surface)."""

    def __init__(self, ctx: Context, xyz, Z, radius, sph_dirs, sph_w, basis):
        self.ctx = ctx
        L = ctx.lib
        self._keep = []  # host arrays kept alive for the call
        xyz = _np(xyz, np.float64).reshape(-1, 3)
        Z = _np(Z, np.float64)
        radius = _np(radius, np.float64)
        dirs = _np(sph_dirs, np.float64).reshape(-1, 3)
        w = _np(sph_w, np.float64)
        b = C.pcm_basis()
        arrs = [_np(basis.shell_atom, np.int32), _np(basis.shell_l, np.int32), _np(basis.shell_nprim, np.int32),
                _np(basis.shell_off, np.int32), _np(basis.prim_exp, np.float64), _np(basis.prim_coef, np.float64)]
        b.n_shells = int(arrs[1].shape[0])
        b.shell_atom, b.shell_l, b.shell_nprim, b.shell_off, b.prim_exp, b.prim_coef = [
            _hp(a).value for a in arrs]
        h = ctypes.c_void_p()
        M = ctypes.c_int()
        st = L.pcm_build_surface(ctx.h, xyz.shape[0], _hp(xyz), _hp(Z), _hp(radius), dirs.shape[0], _hp(dirs),
                                 _hp(w), ctypes.byref(b), ctypes.byref(h), ctypes.byref(M))
        ctx.check(st)
        self.h = h
        self.M = M.value
        self.n_atoms = xyz.shape[0]
        n, nbf, na = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        L.pcm_mol_sizes(h, ctypes.byref(n), ctypes.byref(nbf), ctypes.byref(na), None, None, None, None)
        self.nbf = nbf.value

    @classmethod
    def from_system(cls, ctx: Context, s):
        return cls(ctx, s.xyz, s.Z, s.radius, s.sph_dirs, s.sph_w, s.basis)

    # ------------------------------------------------------------------ helpers
    def _zeros(self, *shape, dtype=None):
        import torch
        return torch.zeros(*shape, dtype=dtype or torch.float64, device=self.ctx.device)

    def sizes(self):
        pf = (ctypes.c_longlong * 6)()
        pe = (ctypes.c_longlong * 6)()
        sf = (ctypes.c_longlong * 6)()
        se = (ctypes.c_longlong * 6)()
        self.ctx.lib.pcm_mol_sizes(self.h, None, None, None, pf, pe, sf, se)
        return {"pairs_fock": list(pf), "pairs_esp": list(pe), "sp_fock": list(sf), "sp_esp": list(se)}

    def pair_list(self, which=0):
        n = sum(self.sizes()["pairs_fock" if which == 0 else "pairs_esp"])
        out = {k: np.zeros(max(n, 1), np.int32) for k in ("cls", "a", "b", "i", "j")}
        self.ctx.check(self.ctx.lib.pcm_pair_list(self.ctx.h, self.h, which, *[_hp(out[k]) for k in
                                                                                 ("cls", "a", "b", "i", "j")]))
        return {k: v[:n] for k, v in out.items()}

    # ----------------------------------------------------------------- the path
    def surface(self):
        import torch
        r = self._zeros(self.M, 3)
        z = self._zeros(self.M)
        S = self._zeros(self.M)
        Akk = self._zeros(self.M)
        own = self._zeros(self.M, dtype=torch.int32)
        sph = self._zeros(self.M, dtype=torch.int32)
        self.ctx.check(self.ctx.lib.pcm_surface_get(self.ctx.h, self.h, _dp(r), _dp(z), _dp(S), _dp(Akk),
                                                    _dp(own), _dp(sph)))
        return {"r": r, "zeta": z, "S": S, "Akk": Akk, "owner": own, "sph": sph}

    def update_geometry(self, xyz, r_surf=None):
        xyz = _np(xyz, np.float64).reshape(-1, 3)
        rs = None if r_surf is None else _np(r_surf, np.float64).reshape(-1, 3)
        self.ctx.check(self.ctx.lib.pcm_update_geometry(self.ctx.h, self.h, _hp(xyz),
                                                        None if rs is None else _hp(rs)))

    def esp(self, P, c=None, bz=None, want_bz=True):
        """c = L P (Eqs. 5-6) and optionally Bz (Eq. 4)."""
        P = _f64(P, self.nbf * self.nbf, "P").contiguous()
        c = self._zeros(self.M) if c is None else c
        if want_bz and bz is None:
            bz = self._zeros(self.M)
        self.ctx.check(self.ctx.lib.pcm_esp(self.ctx.h, self.h, _dp(P), _dp(c), _dp(bz) if want_bz else None))
        return (c, bz) if want_bz else c

    def esp_deriv(self, P, want_bz=True):
        """(c, bz, dc): c = L P (Eqs. 5-6), Bz (Eq. 4) and dc [M, 3] = d c_k / d r_k in one pass."""
        P = _f64(P, self.nbf * self.nbf, "P").contiguous()
        c = self._zeros(self.M)
        dc = self._zeros(self.M, 3)
        bz = self._zeros(self.M) if want_bz else None
        self.ctx.check(self.ctx.lib.pcm_esp_deriv(self.ctx.h, self.h, _dp(P), _dp(c), _dp(bz), _dp(dc)))
        return c, bz, dc

    def fock_grad(self, P, q, dc, F=None):
        """(F, g_nuc, g_surf): F += sum_k q_k L^k (Eq. 10) and the Eq. 14 gradient in one pass;
        dc from esp_deriv with the same P."""
        P = _f64(P, self.nbf * self.nbf, "P").contiguous()
        q = _f64(q, self.M, "q").contiguous()
        dc = _f64(dc, 3 * self.M, "dc").contiguous()
        F = self._zeros(self.nbf, self.nbf) if F is None else F
        gn = self._zeros(self.n_atoms, 3)
        gs = self._zeros(self.M, 3)
        self.ctx.check(self.ctx.lib.pcm_fock_grad(self.ctx.h, self.h, _dp(P), _dp(q), _dp(dc), _dp(F), _dp(gn),
                                                  _dp(gs)))
        return F, gn, gs

    def fock(self, q, F=None):
        """F += sum_k q_k L^k (Eq. 10); returns F."""
        q = _f64(q, self.M, "q").contiguous()
        F = self._zeros(self.nbf, self.nbf) if F is None else F
        self.ctx.check(self.ctx.lib.pcm_fock(self.ctx.h, self.h, _dp(q), _dp(F)))
        return F

    def solve(self, v, precond="jacobi", block=100, seed=0, tol=1e-6, max_iter=10000, q0=None,
              precision="fp64", inner_rtol=1e-4, q=None, raise_noconv=True):
        """q solving A q = -f v (Eq. 1); returns (q, info dict)."""
        v = _f64(v, self.M, "v").contiguous()
        o = _solve_opts(self.ctx.lib, precond, block, seed, tol, max_iter, precision, inner_rtol)
        if q is None:
            q = self._zeros(self.M)
        if q0 is not None:
            q.copy_(q0)
            o.warm_start = 1
        info = C.pcm_solve_info()
        st = self.ctx.lib.pcm_solve(self.ctx.h, self.h, _dp(v), ctypes.byref(o), _dp(q), ctypes.byref(info))
        res = _info_dict(info, st)
        if st != C.PCM_OK and (raise_noconv or st != C.PCM_E_NOCONV):
            self.ctx.check(st)
        return q, res

    def energy(self, bz, c, q):
        """Eq. 13 in FP64."""
        E = ctypes.c_double()
        self.ctx.check(self.ctx.lib.pcm_energy(self.ctx.h, self.h, _dp(bz.contiguous()), _dp(c.contiguous()),
                                               _dp(q.contiguous()), ctypes.byref(E)))
        return E.value

    def matvec_share(self, x, rank=0, nranks=1, y=None):
        """One rank's share of A x in the sharded matvec (tile pairs at positions = rank mod
        nranks); the shares of all ranks add up to A x."""
        x = _f64(x, self.M, "x").contiguous()
        y = self._zeros(self.M) if y is None else y
        self.ctx.check(self.ctx.lib.pcm_matvec_share(self.ctx.h, self.h, _dp(x), _dp(y), int(rank), int(nranks)))
        return y

    def matvec_share_noalloc(self, x, y, rank=0, nranks=1):
        """matvec_share through the allocation-free entry point: y (preallocated, M float64) is
        written asynchronously on the context's stream; intermediates live in the library's
        fixed per-GPU scratch array."""
        x = _f64(x, self.M, "x").contiguous()
        _f64(y, self.M, "y")
        self.ctx.check(self.ctx.lib.pcm_matvec_share_noalloc(self.ctx.h, self.h, _dp(x), _dp(y), int(rank),
                                                             int(nranks)))
        return y

    def grad(self, P, q):
        """(g_nuc [N,3], g_surf [M,3]) of Eq. 14 at fixed density."""
        P = _f64(P, self.nbf * self.nbf, "P").contiguous()
        q = _f64(q, self.M, "q").contiguous()
        gn = self._zeros(self.n_atoms, 3)
        gs = self._zeros(self.M, 3)
        self.ctx.check(self.ctx.lib.pcm_grad(self.ctx.h, self.h, _dp(P), _dp(q), _dp(gn), _dp(gs)))
        return gn, gs

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.pcm_mol_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _solve_opts(lib, precond, block, seed, tol, max_iter, precision, inner_rtol):
    o = C.pcm_solve_opts()
    lib.pcm_default_solve_opts(ctypes.byref(o))
    o.precond = {"none": C.PCM_PRECOND_NONE, "jacobi": C.PCM_PRECOND_JACOBI, "rbj": C.PCM_PRECOND_RBJ,
                 "octree": C.PCM_PRECOND_OCTREE}[precond]
    o.block, o.seed, o.tol, o.max_iter = int(block), int(seed), float(tol), int(max_iter)
    o.precision = C.PCM_MIXED if precision == "mixed" else C.PCM_FP64
    o.inner_rtol = float(inner_rtol)
    return o


def _info_dict(info, st):
    return {"iters": info.iters, "refinements": info.refinements, "resid": info.resid, "energy": info.energy,
            "setup_ms": info.setup_ms, "solve_ms": info.solve_ms, "status": st}


class Batch:
    """Molecules whose kernels run as one launch over a shared work table (pcm_batch_*).

    Destroy (close) the batch before its molecules."""

    def __init__(self, ctx: Context, mols):
        self.ctx = ctx
        self.mols = list(mols)
        n = len(self.mols)
        arr = (ctypes.c_void_p * n)(*[m.h for m in self.mols])
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.pcm_batch_create(ctx.h, arr, n, ctypes.byref(h)))
        self.h = h

    def _ptrs(self, ts):
        return (ctypes.c_void_p * len(ts))(*[_dp(t) for t in ts])

    def esp(self, Ps, want_bz=True):
        """(list of c, list of Bz or None) for every molecule (Eqs. 4-6)."""
        Ps = [_f64(P, m.nbf * m.nbf, "P").contiguous() for P, m in zip(Ps, self.mols)]
        cs = [m._zeros(m.M) for m in self.mols]
        bzs = [m._zeros(m.M) for m in self.mols] if want_bz else None
        st = self.ctx.lib.pcm_esp_batched(self.ctx.h, self.h, self._ptrs(Ps), self._ptrs(cs),
                                          self._ptrs(bzs) if want_bz else None)
        self.ctx.check(st)
        return cs, bzs

    def fock(self, qs, Fs=None):
        """F_i += sum_k q_ik L_i^k for every molecule (Eq. 10); returns the list of F."""
        qs = [_f64(q, m.M, "q").contiguous() for q, m in zip(qs, self.mols)]
        if Fs is None:
            Fs = [m._zeros(m.nbf, m.nbf) for m in self.mols]
        self.ctx.check(self.ctx.lib.pcm_fock_batched(self.ctx.h, self.h, self._ptrs(qs), self._ptrs(Fs)))
        return Fs

    def grad(self, Ps, qs):
        """[(g_nuc, g_surf)] of Eq. 14 at fixed density for every molecule, in shared launches."""
        Ps = [_f64(P, m.nbf * m.nbf, "P").contiguous() for P, m in zip(Ps, self.mols)]
        qs = [_f64(q, m.M, "q").contiguous() for q, m in zip(qs, self.mols)]
        gns = [m._zeros(m.n_atoms, 3) for m in self.mols]
        gss = [m._zeros(m.M, 3) for m in self.mols]
        self.ctx.check(self.ctx.lib.pcm_grad_batched(self.ctx.h, self.h, self._ptrs(Ps), self._ptrs(qs),
                                                     self._ptrs(gns), self._ptrs(gss)))
        return list(zip(gns, gss))

    def solve(self, vs, precond="jacobi", block=100, seed=0, tol=1e-6, max_iter=10000, q0s=None,
              precision="fp64", inner_rtol=1e-4, qs=None, raise_noconv=True):
        """Solve A_i q_i = -f v_i for every molecule; returns (list of q, list of info dicts)."""
        n = len(self.mols)
        if len(vs) != n:
            raise ValueError(f"expected {n} right-hand sides")
        vs = [_f64(v, m.M, "v").contiguous() for v, m in zip(vs, self.mols)]
        o = _solve_opts(self.ctx.lib, precond, block, seed, tol, max_iter, precision, inner_rtol)
        if qs is None:
            qs = [m._zeros(m.M) for m in self.mols]
        if q0s is not None:
            for q, q0 in zip(qs, q0s):
                q.copy_(q0)
            o.warm_start = 1
        va = (ctypes.c_void_p * n)(*[_dp(v) for v in vs])
        qa = (ctypes.c_void_p * n)(*[_dp(q) for q in qs])
        infos = (C.pcm_solve_info * n)()
        st = self.ctx.lib.pcm_solve_batched(self.ctx.h, self.h, va, ctypes.byref(o), qa, infos)
        res = [_info_dict(infos[i], st) for i in range(n)]
        if st != C.PCM_OK and (raise_noconv or st != C.PCM_E_NOCONV):
            self.ctx.check(st)
        return qs, res

    def capture(self, Ps, precond="rbj", block=100, seed=0, tol=1e-8, max_iter=500):
        """The whole pass (c, Bz, FP64 PCG with an iteration budget, E, F += L^T q) of every molecule
        captured as one hipGraph; returns a Graph whose replay() fills its c, bz, q, F, E."""
        g = Graph(self, Ps, precond, block, seed, tol, max_iter)
        self._graphs = getattr(self, "_graphs", []) + [g]
        return g

    def close(self):
        for g in getattr(self, "_graphs", []):
            g.close()
        if getattr(self, "h", None):
            self.ctx.lib.pcm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dynamic_threshold(e_prev: float) -> float:
    """Eq. 21 schedule (pure host)."""
    return C.lib().pcm_dynamic_threshold(float(-1.0 if e_prev is None else e_prev))


def rbj_partition(r, zeta, block: int, seed: int):
    """Randomized block-Jacobi partition on the host (Sec. 4b-ii); returns (perm, blk_off)."""
    r = _np(r, np.float64).reshape(-1, 3)
    zeta = _np(zeta, np.float64)
    M = r.shape[0]
    perm = np.zeros(M, np.int32)
    off = np.zeros(M + 1, np.int32)
    nb = C.lib().pcm_rbj_partition(M, _hp(r), _hp(zeta), int(block), int(seed), _hp(perm), _hp(off))
    if nb < 0:
        raise PCMError(C.PCM_E_ARG, "bad partition arguments")
    return perm, off[: nb + 1].copy()


def octree_partition(r, leaf_max: int):
    """Spatial octree partition on the host (the block-Jacobi scheme RBJ is compared with in
    Sec. 4b-ii); returns (perm, blk_off)."""
    r = _np(r, np.float64).reshape(-1, 3)
    M = r.shape[0]
    perm = np.zeros(M, np.int32)
    off = np.zeros(M + 1, np.int32)
    nb = C.lib().pcm_octree_partition(M, _hp(r), int(leaf_max), _hp(perm), _hp(off))
    if nb < 0:
        raise PCMError(C.PCM_E_ARG, "bad partition arguments")
    return perm, off[: nb + 1].copy()


class ThresholdPolicy:
    """CG threshold per SCF step (Sec. 4b-i): ``fixed`` (delta every step), ``two_delta``
    (scale * delta until the previous DIIS error reaches switch_at, delta afterwards) or
    ``dynamic`` (Eq. 21).  Call with the previous step's DIIS error (None on the first)."""

    KINDS = {"fixed": C.PCM_THRESH_FIXED, "two_delta": C.PCM_THRESH_TWO_DELTA, "dynamic": C.PCM_THRESH_DYNAMIC}

    def __init__(self, kind="dynamic", delta=1e-6, scale=1e4, switch_at=1e-3):
        self.kind = kind
        self._p = C.pcm_threshold_policy()
        C.lib().pcm_default_threshold_policy(ctypes.byref(self._p), self.KINDS[kind])
        self._p.delta, self._p.scale, self._p.switch_at = float(delta), float(scale), float(switch_at)

    @property
    def switched(self) -> bool:
        return bool(self._p.switched)

    def __call__(self, diis_err_prev=None) -> float:
        d = C.lib().pcm_cg_threshold(ctypes.byref(self._p), float(-1.0 if diis_err_prev is None else diis_err_prev))
        if d < 0:
            raise PCMError(C.PCM_E_ARG, "bad threshold policy")
        return d


def default_f(eps=78.39, k=0.0):
    return (eps - 1.0) / (eps + k)


__all__ = ["Context", "Molecule", "Batch", "Graph", "PCMError", "ThresholdPolicy", "dynamic_threshold",
           "octree_partition", "rbj_partition"]


class Graph:
    """A captured batched pass (pcm_graph_capture).  Buffers: Ps (read at each replay), cs, bzs, qs,
    Fs (F accumulates at each replay; zero it between replays for a fresh F) and E (energies).
    While it exists the batch and its molecules refuse other calls; close() it first."""

    def __init__(self, batch: "Batch", Ps, precond, block, seed, tol, max_iter):
        import torch
        self.batch, self.ctx = batch, batch.ctx
        mols = batch.mols
        self.Ps = [_f64(P, m.nbf * m.nbf, "P").contiguous() for P, m in zip(Ps, mols)]
        self.cs = [m._zeros(m.M) for m in mols]
        self.bzs = [m._zeros(m.M) for m in mols]
        self.qs = [m._zeros(m.M) for m in mols]
        self.Fs = [m._zeros(m.nbf, m.nbf) for m in mols]
        self.E = torch.zeros(len(mols), dtype=torch.float64, device="cuda")
        self.tol = float(tol)
        o = _solve_opts(self.ctx.lib, precond, block, seed, tol, max_iter, "fp64", 1e-4)
        h = ctypes.c_void_p()
        p = batch._ptrs
        self.ctx.check(self.ctx.lib.pcm_graph_capture(self.ctx.h, batch.h, p(self.Ps), p(self.cs), p(self.bzs),
                                                      p(self.qs), p(self.Fs), _dp(self.E), ctypes.byref(o),
                                                      ctypes.byref(h)))
        self.h = h

    def replay(self):
        self.ctx.check(self.ctx.lib.pcm_graph_launch(self.ctx.h, self.h))

    def info(self):
        """(list of info dicts, graph node count) after a replay; a molecule whose explicit residual
        is not below tol has 'converged' False."""
        n = len(self.batch.mols)
        infos = (C.pcm_solve_info * n)()
        nodes = ctypes.c_longlong()
        st = self.ctx.lib.pcm_graph_info(self.ctx.h, self.h, infos, ctypes.byref(nodes))
        if st not in (C.PCM_OK, C.PCM_E_NOCONV):
            self.ctx.check(st)
        out = []
        for i in infos:
            d = _info_dict(i, st)
            d["converged"] = i.resid < self.tol
            out.append(d)
        return out, nodes.value

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.pcm_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
