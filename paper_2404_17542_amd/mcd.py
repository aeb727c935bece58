"""Thin ctypes binding of libmcd (include/mcd.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Arrays are torch CUDA tensors (device memory owned by the caller);
their data pointers and the current HIP stream are passed through.  Loading
fails loudly when libmcd.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcd.so")

MCD_OK = 0
STATUS = {0: "MCD_OK", 1: "MCD_ERR_ARG", 2: "MCD_ERR_SINGULAR", 3: "MCD_ERR_NOT_CONVERGED",
          4: "MCD_ERR_BREAKDOWN", 5: "MCD_ERR_ROLE", 6: "MCD_ERR_HIP", 7: "MCD_ERR_OOM"}
ROLE_INNER, ROLE_VOID = -1, 0
BC_DIRICHLET, BC_NEUMANN = 0, 1
WEIGHT_COS2, WEIGHT_GAUSS = 0, 1
PREC_FP64, PREC_FP32_REFINE, PREC_FP32_MATRIX = 0, 1, 2
GUESS_ZERO, GUESS_CALLER = 0, 1
PRECOND_NONE, PRECOND_JACOBI, PRECOND_MG = 0, 1, 2
OP_PHI, OP_GRAD, OP_LAP, OP_DIV, OP_SHIFT = 0, 1, 2, 3, 4
MAX_IDS = 16
MAX_BODIES = 8
MAX_SETS = 4

EXPORTED = ("mcd_create", "mcd_destroy", "mcd_pending_destroys", "mcd_set_stream", "mcd_sync", "mcd_last_error", "mcd_update_dps",
            "mcd_build_stencils", "mcd_get_stencils", "mcd_apply", "mcd_remap", "mcd_advect_diffuse",
            "mcd_neumann_pressure", "mcd_project", "mcd_solve_ppe", "mcd_mg_apply", "mcd_ppe_residual",
            "mcd_ppe_residual_noalloc",
            "mcd_noalloc_scratch_bytes", "mcd_profile",
            "mcd_profile_read", "mcd_profile_read_split", "mcd_autotune", "mcd_set_shape", "mcd_get_shape", "mcd_fluid_force",
            "mcd_model_create", "mcd_model_destroy", "mcd_model_num_params", "mcd_model_set_params",
            "mcd_model_get_params", "mcd_model_get_grads", "mcd_model_output", "mcd_model_set_output_scale",
            "mcd_model_infer",
            "mcd_model_train_step", "mcd_graph_begin", "mcd_graph_end", "mcd_graph_launch",
            "mcd_graph_stats", "mcd_ppe_wide", "mcd_ppe_wide_matrix")


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("origin", C.c_double * 3), ("l0", C.c_double),
                ("periodic", C.c_int * 3), ("walls", C.c_int), ("wall_id", C.c_int)]


class Params(C.Structure):
    _fields_ = [("weight_kind", C.c_int), ("re_over_l0", C.c_double), ("rs_over_l0", C.c_double),
                ("kappa", C.c_double), ("band_over_l0", C.c_double), ("eps_relax", C.c_double),
                ("fit_alpha", C.c_double), ("fit_re_over_l0", C.c_double)]


class Body(C.Structure):
    _fields_ = [("id", C.c_int), ("centre", C.c_double * 3), ("radius", C.c_double),
                ("velocity", C.c_double * 3), ("dvdt", C.c_double * 3), ("omega", C.c_double * 3),
                ("domega_dt", C.c_double * 3), ("theta", C.c_double), ("axis", C.c_double * 3),
                ("sdf", C.c_void_p), ("sdf_n", C.c_int * 3), ("sdf_origin", C.c_double * 3),
                ("sdf_h", C.c_double)]


class WideInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("singular", C.c_int),
                ("true_rel_residual", C.c_double), ("build_ms", C.c_double), ("solve_ms", C.c_double)]


class BcTable(C.Structure):
    _fields_ = [("type", C.c_int * MAX_IDS), ("pin_first", C.c_int)]


class UpdateInfo(C.Structure):
    _fields_ = [("sweeps", C.c_int), ("band_cells", C.c_int), ("counts", C.c_int * 9), ("role_errors", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int), ("guess", C.c_int),
                ("inner_tol", C.c_double), ("max_outer", C.c_int), ("check_every", C.c_int),
                ("max_inner", C.c_int), ("fp64_below", C.c_double), ("precond", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("refinements", C.c_int), ("converged", C.c_int),
                ("true_rel_residual", C.c_double), ("rhs_norm", C.c_double)]


TUNE_MAX = 32


class Tuning(C.Structure):
    _fields_ = [("n", C.c_int), ("grid", C.c_int * TUNE_MAX), ("depth", C.c_int * TUNE_MAX),
                ("us_per_iter", C.c_double * TUNE_MAX), ("chosen", C.c_int)]


class McdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Loads libmcd.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmcd.so not found at {LIB_PATH}: build it with python -m paper_2404_17542_amd.build")
    lib = C.CDLL(LIB_PATH)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    P = C.POINTER
    sig = {
        "mcd_create": (i, [P(MeshDesc), P(Params), vp, P(vp)]),
        "mcd_destroy": (None, [vp]),
        "mcd_set_stream": (i, [vp, vp]),
        "mcd_sync": (i, [vp]),
        "mcd_last_error": (C.c_char_p, [vp]),
        "mcd_update_dps": (i, [vp, P(Body), i, i, vp, vp, vp, vp, vp, vp, P(UpdateInfo)]),
        "mcd_build_stencils": (i, [vp, i, vp, vp, vp, P(BcTable)]),
        "mcd_get_stencils": (i, [vp, i, vp, vp, vp]),
        "mcd_apply": (i, [vp, i, i, vp, i, vp, vp, vp]),
        "mcd_remap": (i, [vp, i, vp, vp, vp, vp, vp, P(Body), P(Body), i, vp]),
        "mcd_advect_diffuse": (i, [vp, i, vp, d, d, vp, vp, P(Body), i, vp, vp]),
        "mcd_neumann_pressure": (i, [vp, vp, vp, vp, P(Body), i, vp]),
        "mcd_project": (i, [vp, i, vp, vp, vp, d, vp, vp, P(Body), i, vp]),
        "mcd_solve_ppe": (i, [vp, i, vp, vp, vp, P(SolveOpts), P(SolveInfo)]),
        "mcd_ppe_residual": (i, [vp, i, vp, vp, vp, vp, P(d)]),
        "mcd_ppe_residual_noalloc": (i, [vp, i, vp, vp, vp, vp, P(d)]),
        "mcd_mg_apply": (i, [vp, i, vp, vp, P(i)]),
        "mcd_noalloc_scratch_bytes": (C.c_size_t, []),
        "mcd_pending_destroys": (i, []),
        "mcd_profile": (i, [vp, i]),
        "mcd_ppe_wide": (i, [vp, i, d, vp, vp, vp, P(BcTable), vp, vp, vp, d, i, P(WideInfo)]),
        "mcd_ppe_wide_matrix": (i, [vp, vp]),
        "mcd_graph_begin": (i, [vp, i]),
        "mcd_graph_end": (i, [vp, i, i]),
        "mcd_graph_launch": (i, [vp, i]),
        "mcd_graph_stats": (i, [vp, i, P(i), P(i)]),
        "mcd_model_create": (i, [vp, i, P(i), i, P(vp)]),
        "mcd_model_destroy": (None, [vp]),
        "mcd_model_num_params": (C.c_size_t, [vp]),
        "mcd_model_set_params": (i, [vp, vp, C.c_size_t]),
        "mcd_model_get_params": (i, [vp, vp, C.c_size_t]),
        "mcd_model_get_grads": (i, [vp, vp, C.c_size_t]),
        "mcd_model_output": (i, [vp, vp]),
        "mcd_model_set_output_scale": (i, [vp, d]),
        "mcd_model_infer": (i, [vp, vp, vp, vp, P(BcTable), vp]),
        "mcd_model_train_step": (i, [vp, vp, vp, vp, vp, P(BcTable), d, P(d)]),
        "mcd_profile_read": (i, [vp, P(d), P(C.c_longlong), P(d), P(C.c_longlong), i]),
        "mcd_profile_read_split": (i, [vp, P(d), P(C.c_longlong), i]),
        "mcd_autotune": (i, [vp, i, i, P(Tuning)]),
        "mcd_fluid_force": (i, [vp, i, i, vp, vp, vp, vp, vp, vp, P(Body), i, d, P(d), P(i)]),
        "mcd_set_shape": (i, [vp, i, i]),
        "mcd_get_shape": (i, [vp, P(i), P(i), P(i)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


_SIZES = {torch.float64: 8, torch.float32: 4, torch.int8: 1, torch.uint8: 1, torch.int32: 4}


def _ptr(t, numel=None, dtype=None):
    """Device pointer of a contiguous CUDA tensor; checks dtype and that it
    holds at least `numel` elements (kernels index up to that extent)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libmcd takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libmcd takes contiguous tensors")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"tensor has {t.numel()} elements, the call reads/writes {numel}")
    return C.c_void_p(t.data_ptr())


def _vec3(v):
    """A 3-vector from a sequence (zero padded) or, for a 2D angular
    quantity, a scalar (its z component)."""
    if isinstance(v, (int, float)):
        return (0.0, 0.0, float(v))
    return tuple(float(v[a]) if a < len(v) else 0.0 for a in range(3))


def bodies_array(bodies):
    """bodies: list of dicts with id, centre, radius, velocity, dvdt and
    optionally omega, domega_dt (3-vectors, or scalars about z in 2D) and,
    for a discrete-SDF body, theta, sdf (device tensor [ny][nx]), sdf_origin,
    sdf_h."""
    n = len(bodies)
    arr = (Body * max(n, 1))()
    for k, b in enumerate(bodies):
        arr[k].id = int(b["id"])
        arr[k].radius = float(b["radius"])
        for a in range(3):
            arr[k].centre[a] = float(b["centre"][a]) if a < len(b["centre"]) else 0.0
            v = b.get("velocity", ())
            arr[k].velocity[a] = float(v[a]) if a < len(v) else 0.0
            g = b.get("dvdt", ())
            arr[k].dvdt[a] = float(g[a]) if a < len(g) else 0.0
        w, dw = _vec3(b.get("omega", ())), _vec3(b.get("domega_dt", ()))
        for a in range(3):
            arr[k].omega[a] = w[a]
            arr[k].domega_dt[a] = dw[a]
        arr[k].theta = float(b.get("theta", 0.0))
        ax = b.get("axis", (0.0, 0.0, 1.0))
        for a in range(3):
            arr[k].axis[a] = float(ax[a])
        g = b.get("sdf")
        if g is not None:
            # a discrete SDF: a contiguous FP64 device tensor [ny][nx] or [nz][ny][nx]
            if not (isinstance(g, torch.Tensor) and g.is_cuda and g.dtype == torch.float64 and g.dim() in (2, 3)
                    and g.is_contiguous()):
                raise ValueError("sdf must be a contiguous 2D or 3D float64 device tensor")
            arr[k].sdf = g.data_ptr()
            shape = tuple(reversed(g.shape))
            for a in range(len(shape)):
                arr[k].sdf_n[a] = int(shape[a])
                arr[k].sdf_origin[a] = float(b["sdf_origin"][a])
            arr[k].sdf_h = float(b["sdf_h"])
    return arr, n


def bc_table(bc: dict, pin_first=False):
    t = BcTable()
    for k in range(MAX_IDS):
        t.type[k] = BC_DIRICHLET
    for bid, typ in bc.items():
        t.type[int(bid)] = int(typ)
    t.pin_first = 1 if pin_first else 0
    return t


class Context:
    """One libmcd context (mesh + workspaces) on the current device/stream."""

    def __init__(self, dim, n, origin, l0, periodic=(False, False, False), walls=False, wall_id=1,
                 weight="cos2", re_over_l0=2.5, rs_over_l0=1.0, kappa=0.2, band_over_l0=5.0, eps_relax=1e-6,
                 stream=None, fit_alpha=0.0, fit_re_over_l0=5.0):
        self.lib = load()
        md = MeshDesc()
        md.dim = dim
        for a in range(3):
            md.n[a] = int(n[a]) if a < dim else 1
            md.origin[a] = float(origin[a]) if a < dim else 0.0
            md.periodic[a] = int(bool(periodic[a])) if a < len(periodic) else 0
        md.l0 = float(l0)
        md.walls = int(bool(walls))
        md.wall_id = int(wall_id)
        pr = Params()
        pr.weight_kind = WEIGHT_COS2 if weight == "cos2" else WEIGHT_GAUSS
        pr.re_over_l0, pr.rs_over_l0, pr.kappa = re_over_l0, rs_over_l0, kappa
        pr.band_over_l0, pr.eps_relax = band_over_l0, eps_relax
        pr.fit_alpha, pr.fit_re_over_l0 = float(fit_alpha), float(fit_re_over_l0)
        self.dim = dim
        self.n = tuple(int(v) for v in n[:dim])
        self.Nc = 1
        for v in self.n:
            self.Nc *= v
        self.nb = 5 if dim == 2 else 9
        self.S = 9 if dim == 2 else 27
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        st = self.lib.mcd_create(C.byref(md), C.byref(pr), C.c_void_p(stream), C.byref(h))
        if st != MCD_OK:
            raise McdError(st, "mcd_create failed")
        self.h = h

    @classmethod
    def from_case(cls, case, **kw):
        from .configs import WALL_ID
        kw.setdefault("fit_alpha", case.fit_alpha)
        kw.setdefault("fit_re_over_l0", case.fit_re_over_l0)
        return cls(case.dim, case.n, case.origin, case.l0, case.periodic, case.walls, WALL_ID, case.weight,
                   case.re_over_l0, case.rs_over_l0, case.kappa, case.band_over_l0, case.eps_relax, **kw)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mcd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != MCD_OK:
            msg = self.lib.mcd_last_error(self.h)
            raise McdError(st, f"{what}: {msg.decode() if msg else ''}")

    @staticmethod
    def _vec(t, numel):
        return _ptr(t, numel, torch.float64)

    # --- calls -------------------------------------------------------------
    def sync(self):
        self._check(self.lib.mcd_sync(self.h), "mcd_sync")

    def update_dps(self, bodies, max_sweeps, pos, role, pos_prev, role_prev, trans, normal, info=True):
        arr, n = bodies_array(bodies)
        ui = UpdateInfo()
        V, D, N = self._vec, self.dim * self.Nc, self.Nc
        st = self.lib.mcd_update_dps(self.h, arr, n, int(max_sweeps), V(pos, D), _ptr(role, N, torch.int8),
                                     V(pos_prev, D), _ptr(role_prev, N, torch.int8), _ptr(trans, N, torch.uint8),
                                     V(normal, D), C.byref(ui) if info else None)
        self._check(st, "mcd_update_dps")
        if info:
            return {"sweeps": ui.sweeps, "band_cells": ui.band_cells, "counts": list(ui.counts),
                    "role_errors": ui.role_errors}
        return None

    def build_stencils(self, set_id, pos, role, normal, bc: dict, pin_first=False):
        t = bc_table(bc, pin_first)
        D, N = self.dim * self.Nc, self.Nc
        self._check(self.lib.mcd_build_stencils(self.h, int(set_id), self._vec(pos, D), _ptr(role, N, torch.int8),
                                                self._vec(normal, D), C.byref(t)), "mcd_build_stencils")

    def get_stencils(self, set_id, phi=None, masks=None, amat=None):
        N = self.Nc
        self._check(self.lib.mcd_get_stencils(self.h, int(set_id), self._vec(phi, self.nb * (self.S + 1) * N),
                                              _ptr(masks, 2 * N, (torch.int32,)), self._vec(amat, self.S * N)),
                    "mcd_get_stencils")

    def apply(self, set_id, op, inp, ncomp, out, neumann_f=None, shift=None):
        N = self.Nc
        n_out = {OP_PHI: self.nb, OP_GRAD: self.dim, OP_LAP: ncomp, OP_DIV: 1, OP_SHIFT: ncomp}.get(op, 0)
        V = self._vec
        self._check(self.lib.mcd_apply(self.h, int(set_id), int(op), V(inp, ncomp * N), int(ncomp),
                                       V(neumann_f, ncomp * N), V(shift, self.dim * N), V(out, n_out * N)),
                    "mcd_apply")

    def remap(self, set_prev, u, pos_prev, pos, role_prev, role, bodies_prev, bodies_new, out):
        bp, n = bodies_array(bodies_prev)
        bn, n2 = bodies_array(bodies_new)
        assert n == n2
        D, N, V = self.dim * self.Nc, self.Nc, self._vec
        self._check(self.lib.mcd_remap(self.h, int(set_prev), V(u, D), V(pos_prev, D), V(pos, D),
                                       _ptr(role_prev, N, torch.int8), _ptr(role, N, torch.int8), bp, bn, n,
                                       V(out, D)), "mcd_remap")

    def advect_diffuse(self, set_id, ut, dt, nu, role, bodies, ustar, rhs=None, pos=None):
        arr, n = bodies_array(bodies)
        D, N, V = self.dim * self.Nc, self.Nc, self._vec
        self._check(self.lib.mcd_advect_diffuse(self.h, int(set_id), V(ut, D), float(dt), float(nu), V(pos, D),
                                                _ptr(role, N, torch.int8), arr, n, V(ustar, D), V(rhs, N)),
                    "mcd_advect_diffuse")

    def neumann_pressure(self, role, normal, bodies, f, pos=None):
        arr, n = bodies_array(bodies)
        N, D = self.Nc, self.dim * self.Nc
        self._check(self.lib.mcd_neumann_pressure(self.h, self._vec(pos, D), _ptr(role, N, torch.int8),
                                                  self._vec(normal, D), arr, n, self._vec(f, N)),
                    "mcd_neumann_pressure")

    def project(self, set_id, P, f, ustar, dt, role, bodies, u, pos=None):
        arr, n = bodies_array(bodies)
        D, N, V = self.dim * self.Nc, self.Nc, self._vec
        self._check(self.lib.mcd_project(self.h, int(set_id), V(P, N), V(f, N), V(ustar, D), float(dt), V(pos, D),
                                         _ptr(role, N, torch.int8), arr, n, V(u, D)), "mcd_project")

    def solve_ppe(self, set_id, rhs, p, neumann_f=None, tol=1e-8, max_iter=20000, precision=PREC_FP64,
                  guess=GUESS_ZERO, inner_tol=None, max_outer=None, check_every=16, max_inner=None,
                  fp64_below=None, precond=PRECOND_NONE, raise_on_fail=True):
        if inner_tol is None:
            inner_tol = 0.03 if precision == PREC_FP32_MATRIX else 1e-2
        if max_outer is None:
            max_outer = 500 if precision == PREC_FP32_MATRIX else 40
        if fp64_below is None:
            fp64_below = 1e-2 if precision == PREC_FP32_MATRIX else 0.0
        o = SolveOpts()
        o.tol, o.max_iter, o.precision, o.guess = tol, int(max_iter), int(precision), int(guess)
        o.inner_tol, o.max_outer, o.check_every = inner_tol, int(max_outer), int(check_every)
        if max_inner is None:
            max_inner = max(200, int(4 * self.Nc ** (1.0 / self.dim)))
        o.max_inner = int(max_inner)
        o.fp64_below = float(fp64_below)
        o.precond = int(precond)
        info = SolveInfo()
        N, V = self.Nc, self._vec
        st = self.lib.mcd_solve_ppe(self.h, int(set_id), V(rhs, N), V(neumann_f, N), V(p, N), C.byref(o),
                                    C.byref(info))
        out = {"iterations": info.iterations, "restarts": info.restarts, "refinements": info.refinements,
               "converged": bool(info.converged), "true_rel_residual": info.true_rel_residual,
               "rhs_norm": info.rhs_norm, "status": st}
        if raise_on_fail:
            self._check(st, "mcd_solve_ppe")
        return out

    def ppe_residual(self, set_id, rhs, p, r, neumann_f=None, norms=True):
        """r := b_eff - A p on unknown rows; returns (||r||, ||b_eff||), or,
        with norms=False, only enqueues r (no wait, no input check) and
        returns None."""
        out = (C.c_double * 2)() if norms else None
        N, V = self.Nc, self._vec
        self._check(self.lib.mcd_ppe_residual(self.h, int(set_id), V(rhs, N), V(neumann_f, N), V(p, N), V(r, N),
                                              out), "mcd_ppe_residual")
        return (out[0], out[1]) if norms else None

    def mg_apply(self, set_id, inp, out):
        """One V-cycle of the set's multigrid preconditioner (mcd_mg_apply);
        returns the number of levels."""
        lv = C.c_int()
        N, V = self.Nc, self._vec
        self._check(self.lib.mcd_mg_apply(self.h, int(set_id), V(inp, N), V(out, N), C.byref(lv)), "mcd_mg_apply")
        return lv.value

    def ppe_residual_noalloc(self, set_id, rhs, p, r, neumann_f=None):
        """mcd_ppe_residual_noalloc: the same residual with the library's fixed
        per-device scratch (no allocation); returns (||r||, ||b_eff||)."""
        norms = (C.c_double * 2)()
        N, V = self.Nc, self._vec
        self._check(self.lib.mcd_ppe_residual_noalloc(self.h, int(set_id), V(rhs, N), V(neumann_f, N), V(p, N),
                                                      V(r, N), norms), "mcd_ppe_residual_noalloc")
        return norms[0], norms[1]

    def fluid_force(self, set_u, set_p, u, p, pos, role, normal, bodies, mu, neumann_f=None):
        """Force of the fluid on each body (2D; see mcd_fluid_force): returns
        ([(Fx, Fy)] per body, [(boundary DPs, fallbacks)] per body)."""
        arr, n = bodies_array(bodies)
        F = (C.c_double * (2 * n))()
        cnt = (C.c_int * (2 * n))()
        D, N, V = self.dim * self.Nc, self.Nc, self._vec
        self._check(self.lib.mcd_fluid_force(self.h, int(set_u), int(set_p), V(u, D), V(p, N), V(neumann_f, N),
                                             V(pos, D), _ptr(role, N, torch.int8), V(normal, D), arr, n, float(mu),
                                             F, cnt), "mcd_fluid_force")
        return [(F[2 * k], F[2 * k + 1]) for k in range(n)], [(cnt[2 * k], cnt[2 * k + 1]) for k in range(n)]

    def autotune(self, set_id, iters=32):
        """Times the stage-kernel shapes on the set's operator and applies the
        fastest (see mcd_autotune); returns the candidates and the choice."""
        t = Tuning()
        self._check(self.lib.mcd_autotune(self.h, int(set_id), int(iters), C.byref(t)), "mcd_autotune")
        cands = [{"grid": t.grid[k], "depth": t.depth[k], "us_per_iter": t.us_per_iter[k]} for k in range(t.n)]
        return {"candidates": cands, "chosen": t.chosen, "shape": self.get_shape()}

    def set_shape(self, grid, depth=None):
        if depth is None:
            depth = 8 if self.dim == 3 else 1
        self._check(self.lib.mcd_set_shape(self.h, int(grid), int(depth)), "mcd_set_shape")

    def get_shape(self):
        g, dp, b = C.c_int(), C.c_int(), C.c_int()
        self._check(self.lib.mcd_get_shape(self.h, C.byref(g), C.byref(dp), C.byref(b)), "mcd_get_shape")
        return {"grid": g.value, "depth": dp.value, "blocks": b.value}

    def ppe_wide(self, half, re_over_l0, pos, role, normal, bc, rhs, p, neumann_f=None, pin_first=False, tol=1e-8,
                 max_iter=20000, raise_on_fail=True):
        """PPE on the (2 half + 1)^2 support (see mcd_ppe_wide); returns its info."""
        info = WideInfo()
        D, N, V = self.dim * self.Nc, self.Nc, self._vec
        t = bc_table(bc, pin_first)
        st = self.lib.mcd_ppe_wide(self.h, int(half), float(re_over_l0), V(pos, D), _ptr(role, N, torch.int8),
                                   V(normal, D), C.byref(t), V(rhs, N), V(neumann_f, N), V(p, N), float(tol),
                                   int(max_iter), C.byref(info))
        out = {"iterations": info.iterations, "converged": bool(info.converged), "singular": info.singular,
               "true_rel_residual": info.true_rel_residual, "build_ms": info.build_ms, "solve_ms": info.solve_ms}
        if raise_on_fail or st not in (0, 3):
            self._check(st, "mcd_ppe_wide")
        return out

    def ppe_wide_matrix(self, half, out):
        S = (2 * half + 1) ** 2
        self._check(self.lib.mcd_ppe_wide_matrix(self.h, self._vec(out, S * self.Nc)), "mcd_ppe_wide_matrix")

    def graph_begin(self, slot):
        """Start recording the following calls into graph slot `slot` (see
        mcd_graph_begin); they run at graph_end."""
        self._check(self.lib.mcd_graph_begin(self.h, int(slot)), "mcd_graph_begin")

    def graph_end(self, slot, launch=True):
        """Stop recording; the slot's graph is instantiated the first time and
        updated in place later, and launched unless launch=False."""
        self._check(self.lib.mcd_graph_end(self.h, int(slot), 1 if launch else 0), "mcd_graph_end")

    def graph_launch(self, slot):
        self._check(self.lib.mcd_graph_launch(self.h, int(slot)), "mcd_graph_launch")

    def graph_stats(self, slot):
        a, b = C.c_int(), C.c_int()
        self._check(self.lib.mcd_graph_stats(self.h, int(slot), C.byref(a), C.byref(b)), "mcd_graph_stats")
        return {"instantiated": a.value, "updated": b.value}

    def profile(self, enable=True):
        self._check(self.lib.mcd_profile(self.h, int(bool(enable))), "mcd_profile")

    def profile_read(self, reset=True):
        mp, ms = C.c_double(), C.c_double()
        npp, ns = C.c_longlong(), C.c_longlong()
        self._check(self.lib.mcd_profile_read(self.h, C.byref(mp), C.byref(npp), C.byref(ms), C.byref(ns),
                                              int(bool(reset))), "mcd_profile_read")
        return {"p_ms": mp.value, "p_n": npp.value, "s_ms": ms.value, "s_n": ns.value}

    def profile_read_split(self, reset=True):
        """Stage timings split by the matrix copy the launches read:
        {'fp64': {p_ms, p_n, s_ms, s_n}, 'fp32': {...}}."""
        ms = (C.c_double * 4)()
        n = (C.c_longlong * 4)()
        self._check(self.lib.mcd_profile_read_split(self.h, ms, n, int(bool(reset))), "mcd_profile_read_split")
        return {"fp64": {"p_ms": ms[0], "p_n": n[0], "s_ms": ms[1], "s_n": n[1]},
                "fp32": {"p_ms": ms[2], "p_n": n[2], "s_ms": ms[3], "s_n": n[3]}}


class Model:
    """Learned initial guess (U-Net) bound to a context (2D or 3D mesh)."""

    def __init__(self, ctx: Context, channels=(16, 32, 64, 128), body_id=2):
        import numpy as np
        self.ctx = ctx
        self.lib = ctx.lib
        self.channels = tuple(int(c) for c in channels)
        arr = (C.c_int * len(self.channels))(*self.channels)
        h = C.c_void_p()
        ctx._check(self.lib.mcd_model_create(ctx.h, len(self.channels), arr, int(body_id), C.byref(h)),
                   "mcd_model_create")
        self.h = h
        self.n = int(self.lib.mcd_model_num_params(self.h))
        self._np = np

    def close(self):
        if getattr(self, "h", None):
            self.lib.mcd_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        t = self._np.ascontiguousarray(theta, dtype=self._np.float32)
        if t.size != self.n:
            raise ValueError(f"expected {self.n} parameters, got {t.size}")
        self.ctx._check(self.lib.mcd_model_set_params(self.h, t.ctypes.data_as(C.c_void_p), self.n),
                        "mcd_model_set_params")

    def get_params(self):
        t = self._np.zeros(self.n, dtype=self._np.float32)
        self.ctx._check(self.lib.mcd_model_get_params(self.h, t.ctypes.data_as(C.c_void_p), self.n),
                        "mcd_model_get_params")
        return t

    def get_grads(self):
        t = self._np.zeros(self.n, dtype=self._np.float32)
        self.ctx._check(self.lib.mcd_model_get_grads(self.h, t.ctypes.data_as(C.c_void_p), self.n),
                        "mcd_model_get_grads")
        return t

    def output(self, h):
        self.ctx._check(self.lib.mcd_model_output(self.h, _ptr(h, self.ctx.Nc, torch.float32)), "mcd_model_output")

    def set_output_scale(self, s):
        self.ctx._check(self.lib.mcd_model_set_output_scale(self.h, float(s)), "mcd_model_set_output_scale")

    def infer(self, resid, p_prev, role, bc: dict, p_out):
        """p_out := p_prev + s rms(resid) h; resid = PPE residual of p_prev."""
        t = bc_table(bc)
        N, V = self.ctx.Nc, self.ctx._vec
        self.ctx._check(self.lib.mcd_model_infer(self.h, V(resid, N), V(p_prev, N), _ptr(role, N, torch.int8),
                                                 C.byref(t), V(p_out, N)), "mcd_model_infer")

    def train_step(self, resid, p_prev, p_target, role, bc: dict, lr, want_loss=True):
        t = bc_table(bc)
        N, V = self.ctx.Nc, self.ctx._vec
        loss = C.c_double(float("nan"))
        self.ctx._check(self.lib.mcd_model_train_step(self.h, V(resid, N), V(p_prev, N), V(p_target, N),
                                                      _ptr(role, N, torch.int8), C.byref(t), float(lr),
                                                      C.byref(loss) if want_loss else None),
                        "mcd_model_train_step")
        return loss.value
