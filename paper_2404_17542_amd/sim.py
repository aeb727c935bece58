"""GPU time stepper: one MCD projection step through libmcd.

Order of one step k -> k+1 (Sec. 3.3 with the DP update of Sec. 2.3-2.4):
rearrange DPs and reassign roles at t^{k+1}; remap u^k to x^{k+1} with the
step-k velocity weights; build the velocity and pressure weights at x^{k+1};
u* and the PPE right-hand side; Neumann datum -dV/dt . n; the initial guess
(previous pressure, zero, or the previous pressure corrected by the learned
network); Bi-CGSTAB; project.
Every step runs in libmcd kernels; this module only sequences the calls and
owns the device arrays (torch tensors on one stream).
"""
from __future__ import annotations

import gc

import math

import numpy as np
import torch

from . import inputs
from .configs import WALL_ID
from . import mcd as M

SET_VEL = (0, 1)   # ping-pong: velocity weights of step k and step k+1
SET_P = 2


class GpuSim:
    def __init__(self, case, precision=M.PREC_FP64, device="cuda", check_every=16, update_info=True,
                 guess="warm", model=None, precond=M.PRECOND_NONE, graph=False):
        if graph and update_info:
            raise ValueError("graph mode records the DP update without its host-side info: pass update_info=False")
        self.case = case
        self.graph = graph
        self._ahead = None          # (k, slot, prepare results) recorded ahead in graph mode
        self.graph_fallbacks = 0    # parts run directly because a recording was invalidated
        self.guess = guess
        self.precond = precond
        self.model = model
        self.resid = None
        self.device = device
        self.precision = precision
        self.check_every = check_every
        self.update_info = update_info
        self.ctx = M.Context.from_case(case)
        dim, Nc = case.dim, case.n_cells
        f64 = dict(dtype=torch.float64, device=device)
        pos0 = inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed)
        self.pos = torch.tensor(pos0, **f64).contiguous()
        self.pos_prev = torch.zeros_like(self.pos)
        self.normal = torch.zeros_like(self.pos)
        self.role = torch.full((Nc,), M.ROLE_INNER, dtype=torch.int8, device=device)
        self.role_prev = torch.zeros_like(self.role)
        self.trans = torch.zeros((Nc,), dtype=torch.uint8, device=device)
        self.u = torch.zeros((dim, Nc), **f64)
        self.ut = torch.zeros_like(self.u)
        self.ustar = torch.zeros_like(self.u)
        self.rhs = torch.zeros((Nc,), **f64)
        self.P = torch.zeros((Nc,), **f64)
        self.fP = torch.zeros((Nc,), **f64)
        self.k = 0
        self.t = 0.0
        self.log = []
        self.same_sets = case.bc_pressure == case.bc_velocity
        # discrete SDFs of the bodies that have one, resident on the device
        self.sdf = {}
        for b in case.rigid_bodies:
            g = b.sdf_grid(case.l0, case.band_over_l0)
            if g is not None:
                self.sdf[b.body_id] = (torch.tensor(g[0], **f64).contiguous(), g[1], g[2])
        self.bodies = self.bodies_at(0.0, prev=None)
        # initial masking (its transitions from the placeholder roles are not meaningful)
        self.ctx.update_dps(self.bodies, 0, self.pos, self.role, self.pos_prev, self.role_prev, self.trans,
                            self.normal, info=False)
        try:
            self.ctx.sync()
        except M.McdError as e:
            if e.status != 5:
                raise
        n_init = case.n_relax_init if self.bodies else 0
        self.init_info = self.ctx.update_dps(self.bodies, n_init, self.pos, self.role, self.pos_prev,
                                             self.role_prev, self.trans, self.normal, info=True)
        role_h = self.role.cpu().numpy()
        if case.name.startswith("C1"):
            u0 = inputs.tgv_velocity(self.pos.cpu().numpy(), 0.0, case.nu)
        else:
            u0 = np.zeros((dim, Nc))
        pos_h = self.pos.cpu().numpy()
        for b in self.bodies:
            sel = role_h == b["id"]
            w = b["omega"]
            r = [pos_h[a, sel] - b["centre"][a] for a in range(dim)] + [0.0] * (3 - dim)
            rot = (w[1] * r[2] - w[2] * r[1], w[2] * r[0] - w[0] * r[2], w[0] * r[1] - w[1] * r[0])   # omega x r
            for a in range(dim):
                u0[a, sel] = b["velocity"][a] + rot[a] if any(w) else b["velocity"][a]
        self.u.copy_(torch.tensor(u0, **f64))
        self.vel_slot = 0
        self.ctx.build_stencils(SET_VEL[self.vel_slot], self.pos, self.role, self.normal, case.bc_velocity,
                                case.pin_first if self.same_sets else False)
        torch.cuda.synchronize()

    def bodies_at(self, t, prev):
        out = []
        for i, b in enumerate(self.case.rigid_bodies):
            vel = b.motion.velocity(t)
            w = b.motion.omega_vector(t)
            if prev is None:
                dvdt, dw = (0.0,) * len(vel), (0.0, 0.0, 0.0)
            else:
                dvdt = tuple((vn - vo) / self.case.dt for vn, vo in zip(vel, prev[i]["velocity"]))
                dw = tuple((wn - wo) / self.case.dt for wn, wo in zip(w, prev[i]["omega"]))
            d = {"id": b.body_id, "centre": b.motion.centre(t), "radius": b.radius, "velocity": vel,
                 "dvdt": dvdt, "omega": w, "domega_dt": dw, "theta": b.motion.theta(t),
                 "axis": b.posture_axis()}
            if b.body_id in self.sdf:
                g, o, h = self.sdf[b.body_id]
                d.update(sdf=g, sdf_origin=o, sdf_h=h)
            out.append(d)
        return out

    def prepare(self):
        """First half of a step: DP update at t^{k+1}, remap, weights, u* and
        the PPE data.  Leaves (pset, bodies_new, update info).  Direct calls
        (step() in graph mode runs the same calls as recorded graphs)."""
        self._ahead = None
        return self._prepare()

    def _prepare(self):
        case, ctx = self.case, self.ctx
        tn = (self.k + 1) * case.dt
        bodies_new = self.bodies_at(tn, self.bodies) if self.bodies else []
        upd = ctx.update_dps(bodies_new, case.n_relax, self.pos, self.role, self.pos_prev, self.role_prev,
                             self.trans, self.normal, info=self.update_info)
        old = SET_VEL[self.vel_slot]
        new = SET_VEL[1 - self.vel_slot]
        ctx.remap(old, self.u, self.pos_prev, self.pos, self.role_prev, self.role, self.bodies, bodies_new, self.ut)
        # one set serves both fields when their boundary conditions agree (the pin
        # only shapes the PPE matrix of a set, never its weights)
        ctx.build_stencils(new, self.pos, self.role, self.normal, case.bc_velocity,
                           case.pin_first if self.same_sets else False)
        pset = new
        if not self.same_sets:
            ctx.build_stencils(SET_P, self.pos, self.role, self.normal, case.bc_pressure, case.pin_first)
            pset = SET_P
        ctx.advect_diffuse(new, self.ut, case.dt, case.nu, self.role, bodies_new, self.ustar, self.rhs, pos=self.pos)
        ctx.neumann_pressure(self.role, self.normal, bodies_new, self.fP, pos=self.pos)
        return pset, bodies_new, upd

    def forces(self):
        """Fluid force on each body at the current step (after finish()):
        velocity weights of this step, pressure weights of its solve, mu = nu
        (unit density).  2D."""
        vset = SET_VEL[self.vel_slot]
        pset = vset if self.same_sets else SET_P
        return self.ctx.fluid_force(vset, pset, self.u, self.P, self.pos, self.role, self.normal, self.bodies,
                                    self.case.nu, self.fP)

    def tuning_set(self):
        """A built pressure set at the current positions, for the stage-kernel
        autotuner (the velocity set when both fields share one; otherwise the
        pressure set is built now, which the next step rebuilds anyway)."""
        if self.same_sets:
            return SET_VEL[self.vel_slot]
        self.ctx.build_stencils(SET_P, self.pos, self.role, self.normal, self.case.bc_pressure, self.case.pin_first)
        return SET_P

    def initial_guess(self, pset, mode):
        """Prepares the solver's initial guess and returns the solver's guess
        flag: 'warm' keeps P^k, 'zero' starts from 0 at the unknowns,
        'learned' adds the network's correction to P^k (the network reads the
        PPE residual of P^k under the new weights)."""
        if mode == "warm":
            return M.GUESS_CALLER
        if mode == "zero":
            return M.GUESS_ZERO
        if mode != "learned" or self.model is None:
            raise ValueError(f"unknown initial guess {mode!r} (or no model for 'learned')")
        if self.resid is None:
            self.resid = torch.zeros_like(self.P)
        # enqueued only: the solve that follows checks the same right-hand side
        self.ctx.ppe_residual(pset, self.rhs, self.P, self.resid, self.fP, norms=False)
        self.model.infer(self.resid, self.P, self.role, self.case.bc_pressure, self.P)
        return M.GUESS_CALLER

    def finish(self, pset, bodies_new, info, upd):
        self._project(pset, bodies_new)
        return self._advance(bodies_new, info, upd)

    def _project(self, pset, bodies_new):
        self.ctx.project(pset, self.P, self.fP, self.ustar, self.case.dt, self.role, bodies_new, self.u,
                         pos=self.pos)

    def _advance(self, bodies_new, info, upd):
        case = self.case
        self.vel_slot = 1 - self.vel_slot
        self.bodies = bodies_new
        self.k += 1
        self.t = (self.k) * case.dt
        rec = {"k": self.k, "iters": info["iterations"], "restarts": info["restarts"],
               "refinements": info["refinements"], "rel_res": info["true_rel_residual"],
               "converged": info["converged"]}
        if upd is not None:
            rec.update({"sweeps": upd["sweeps"], "trans": upd["counts"]})
        self.log.append(rec)
        return rec

    def solve(self, pset, guess=M.GUESS_CALLER, precond=None):
        return self.ctx.solve_ppe(pset, self.rhs, self.P, self.fP, tol=self.case.tol, precision=self.precision,
                                  guess=guess, check_every=self.check_every,
                                  precond=self.precond if precond is None else precond)

    def step(self):
        if self.graph:
            return self._step_graphs()
        pset, bodies_new, upd = self.prepare()
        info = self.solve(pset, self.initial_guess(pset, self.guess))
        return self.finish(pset, bodies_new, info, upd)

    def _record(self, slot, fn):
        """Records the calls made by fn() into graph slot `slot` (not run) and
        returns fn's result, or None when the runtime invalidated the
        recording (nothing ran; the caller then makes the calls directly, with
        the same results)."""
        # no garbage collection while recording: a collected context would free
        # device memory in the middle of the recording
        gc_on = gc.isenabled()
        gc.disable()
        try:
            return self._record_calls(slot, fn)
        finally:
            if gc_on:
                gc.enable()

    def _record_calls(self, slot, fn):
        self.ctx.graph_begin(slot)
        try:
            out = fn()
        except M.McdError as e:
            try:
                self.ctx.graph_end(slot, launch=False)
            except M.McdError:
                pass
            if e.status == 6:          # MCD_ERR_HIP: the recording, not the call, failed
                self.graph_fallbacks += 1
                return None
            raise
        except BaseException:
            try:
                self.ctx.graph_end(slot, launch=False)
            except M.McdError:
                pass
            raise
        try:
            self.ctx.graph_end(slot, launch=False)
        except M.McdError as e:
            if e.status != 6:
                raise
            self.graph_fallbacks += 1
            return None
        return out

    def _step_graphs(self):
        """One step as graphs: the preparation (recorded during the previous
        step), the solve's chunk graphs, the projection.  While the GPU runs
        this step, the host records its projection and the next step's
        preparation, so no recording sits between GPU work.  Preparations use
        slots 0 and 2, projections 1 and 3, alternating by step parity: a slot
        is recorded again only after its previous launch has completed (the
        solve of the step in between has returned)."""
        pre = self._ahead
        self._ahead = None
        if pre is not None and pre[0] == self.k:
            _, slot, out = pre
            self.ctx.graph_launch(slot)
        else:
            slot = 2 * (self.k % 2)
            out = self._record(slot, self._prepare)
            if out is None:
                out = self._prepare()
            else:
                self.ctx.graph_launch(slot)
        pset, bodies_new, upd = out
        guess = self.initial_guess(pset, self.guess)
        post = 1 + 2 * (self.k % 2)
        post_ok = self._record(post, lambda: self._project(pset, bodies_new) or True) is not None
        saved = (self.k, self.vel_slot, self.bodies)
        self.k, self.vel_slot, self.bodies = self.k + 1, 1 - self.vel_slot, bodies_new
        try:
            nslot = 2 * (self.k % 2)
            ahead = self._record(nslot, self._prepare)
            nxt = (self.k, nslot, ahead) if ahead is not None else None
        finally:
            self.k, self.vel_slot, self.bodies = saved
        info = self.solve(pset, guess)
        if post_ok:
            self.ctx.graph_launch(post)
        else:
            self._project(pset, bodies_new)
        self._ahead = nxt
        return self._advance(bodies_new, info, upd)

    def ctx_unknown_count(self):
        """PPE unknowns of the current step (inner and Neumann DPs, minus a pin)."""
        unk = self.role == M.ROLE_INNER
        for bid, typ in self.case.bc_pressure.items():
            if typ == M.BC_NEUMANN:
                unk |= self.role == bid
        return int(unk.sum().item()) - (1 if self.case.pin_first else 0)

    def n_active(self):
        return int((self.role != M.ROLE_VOID).sum().item())

    def kinetic_energy(self):
        sel = self.role == M.ROLE_INNER
        return float((self.u[:, sel] ** 2).sum().item())
