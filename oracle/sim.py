"""Oracle time stepper: one MCD projection step on the CPU in FP64.

TEST INFRASTRUCTURE (see mcd_oracle).  Order of one step k -> k+1
(Sec. 3.3 and Sec. 2.3-2.4):

 1. body state at t^{k+1}; dV_trans/dt and d omega/dt by the backward
    differences of Eq. (dvdt_moving_boundary);
 2. DP rearrangement and role reassignment at t^{k+1};
 3. remap u^k -> u~ at x^{k+1} with the step-k velocity weights (Eq. ale_vel,
    Appendix A);
 4. MLS weights at x^{k+1} for the velocity and the pressure sets;
 5. u* = F_MOC + nu dt lap u~ (Eq. intermed_vel);
 6. b = div u* / dt and the Neumann datum -dV/dt . n (Eqs. pressure_poisson,
    neumann_moving_boundary);
 7. Bi-CGSTAB solve of the PPE;
 8. u^{k+1} = u* - dt grad P (Eq. projection).
"""
from __future__ import annotations

import time

import numpy as np

from . import mcd_oracle as O
from paper_2404_17542_amd import inputs


def oracle_bodies(case, t):
    """Body states at time t; a body with a discrete SDF carries its grid
    (the MLS weight and r_e / l0 of the case, in units of the grid step)."""
    out = []
    for b in case.rigid_bodies:
        grid = None
        g = b.sdf_grid(case.l0, case.band_over_l0)
        if g is not None:
            grid = O.SdfGrid(g[0], g[1], g[2], case.re_over_l0, case.weight,
                             O.sdf_far_radius(b.radius, case.l0, case.band_over_l0))
        out.append(O.BodyState(b.motion.centre(t), b.radius, b.body_id, b.motion.velocity(t),
                               b.motion.omega_vector(t), b.motion.theta(t), grid, b.posture_axis()))
    return out


class OracleSim:
    def __init__(self, case, mixed=False):
        self.case = case
        self.mesh = O.Mesh.from_case(case)
        self.consts = O.RelaxConsts.make(case.l0, case.kappa, case.eps_relax, case.band_over_l0,
                                         case.fit_alpha, case.fit_re_over_l0)
        self.re = case.re_over_l0 * case.l0
        self.rs = case.rs_over_l0 * case.l0
        self.mixed = mixed
        self.t = 0.0
        self.k = 0
        self.timings = {}
        self.log = []
        self.last_ppe = None        # (A, b_eff, unknown indices) of the last plain solve
        pos = inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed)
        bodies = self.bodies_at(0.0)
        role0 = O.roles(self.mesh, bodies)
        up = O.update_dps(self.mesh, self.consts, bodies, pos, role0,
                          case.n_relax_init if bodies else 0)
        self.pos, self.role, self.normal = up.pos, up.role, up.normal
        self.init_sweeps = up.sweeps
        dim = case.dim
        if case.name.startswith("C1"):
            self.u = inputs.tgv_velocity(self.pos, 0.0, case.nu)
        else:
            self.u = np.zeros((dim, self.mesh.Nc))
        for b in bodies:
            sel = self.role == b.body_id
            V = O.body_point_velocity(b, self.pos[:, sel])
            for a in range(dim):
                self.u[a, sel] = V[a]
        self.P = np.zeros(self.mesh.Nc)
        self.bodies = bodies
        self.st_vel = self._build(case.bc_velocity)

    def bodies_at(self, t):
        return oracle_bodies(self.case, t)

    def _build(self, bc):
        return O.mls_build(self.mesh, self.pos, self.role, self.normal, bc, self.re, self.rs,
                           self.case.weight)

    def step(self):
        case, mesh = self.case, self.mesh
        t0 = time.perf_counter()
        tn = (self.k + 1) * case.dt
        bodies_new = self.bodies_at(tn)
        dvdt = {b.body_id: tuple((vn - vo) / case.dt for vn, vo in zip(b.velocity, bo.velocity))
                for b, bo in zip(bodies_new, self.bodies)}
        domega = {b.body_id: tuple((wn - wo) / case.dt for wn, wo in zip(b.omega, bo.omega))
                  for b, bo in zip(bodies_new, self.bodies)}
        up = O.update_dps(mesh, self.consts, bodies_new, self.pos, self.role, case.n_relax)
        t1 = time.perf_counter()
        ut, rstats = O.remap_velocity(mesh, self.st_vel, self.u, self.pos, up.pos, self.role, up.role,
                                      self.bodies, bodies_new)
        self.pos, self.role, self.normal = up.pos, up.role, up.normal
        st_vel = self._build(case.bc_velocity)
        st_p = st_vel if case.bc_pressure == case.bc_velocity else self._build(case.bc_pressure)
        t2 = time.perf_counter()
        ustar = O.moc_viscous(mesh, st_vel, ut, case.dt, case.nu, self.role, bodies_new, pos=self.pos)
        b = O.divergence(mesh, st_vel, ustar) / case.dt
        f_p = O.neumann_pressure_data(mesh, self.role, self.normal, bodies_new, dvdt, domega, pos=self.pos)
        unk = O.unknown_mask(self.role, case.bc_pressure, case.pin_first)
        p_in = np.where(unk, self.P, 0.0)
        t3 = time.perf_counter()
        if self.mixed:
            P, info = O.solve_ppe_mixed(mesh, st_p, self.role, case.bc_pressure, b, p_in, f_p, case.tol,
                                        case.pin_first, guess="caller")
            self.last_ppe = None
        else:
            P, info, self.last_ppe = O.solve_ppe(mesh, st_p, self.role, case.bc_pressure, b, p_in, f_p, case.tol,
                                                 case.pin_first, guess="caller")
        t4 = time.perf_counter()
        self.u = O.project(mesh, st_p, P, f_p, ustar, case.dt, self.role, bodies_new, pos=self.pos)
        self.P = P
        self.st_vel = st_vel
        self.bodies = bodies_new
        self.k += 1
        self.t = tn
        t5 = time.perf_counter()
        rec = {"k": self.k, "sweeps": up.sweeps, "iters": info.iterations, "restarts": info.restarts,
               "rel_res": info.true_rel_residual, "converged": info.converged,
               "trans": np.bincount(up.trans, minlength=9).tolist(), "remap": rstats,
               "t_update": t1 - t0, "t_build": t2 - t1, "t_glue": (t3 - t2) + (t5 - t4), "t_solve": t4 - t3}
        self.log.append(rec)
        return rec

    def kinetic_energy(self):
        sel = self.role == O.INNER
        return float(np.sum(self.u[:, sel] ** 2))
