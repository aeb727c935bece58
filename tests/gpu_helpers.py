"""Shared helpers of the GPU parity tests (imports torch/libmcd lazily)."""
import numpy as np

from oracle import mcd_oracle as O


def np_(t):
    return t.detach().cpu().numpy()


def oracle_bodies(case, t):
    from oracle.sim import oracle_bodies as ob
    return ob(case, t)


_SDF = {}


def gpu_bodies(case, t, dvdt=None):
    """Body dicts for the C ABI; discrete SDFs are uploaded once per case."""
    import torch
    out = []
    for b in case.rigid_bodies:
        d = {"id": b.body_id, "centre": b.motion.centre(t), "radius": b.radius,
             "velocity": b.motion.velocity(t), "dvdt": dvdt or (0.0,) * case.dim,
             "omega": b.motion.omega_vector(t), "theta": b.motion.theta(t), "axis": b.posture_axis()}
        g = b.sdf_grid(case.l0, case.band_over_l0)
        if g is not None:
            key = (case.name, b.body_id)
            if key not in _SDF:
                _SDF[key] = torch.tensor(g[0], dtype=torch.float64, device="cuda").contiguous()
            d.update(sdf=_SDF[key], sdf_origin=g[1], sdf_h=g[2])
        out.append(d)
    return out


def bits_equal(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    if a.dtype == np.float64:
        return np.array_equal(a.view(np.int64), b.view(np.int64))
    return np.array_equal(a, b)


def weights_rel_err(phi_gpu, phi_ora, idx_mask=None):
    """Per DP and per basis component b: max_s |dc| / max_s |c_ora| (slots S+1)."""
    num = np.abs(phi_gpu - phi_ora).max(axis=1)
    den = np.abs(phi_ora).max(axis=1)
    rel = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
    if idx_mask is not None:
        rel = rel[:, idx_mask]
    return rel


def masks_from_kind(st, S, centre):
    vm = np.zeros(st.kind.shape[1], dtype=np.int64)
    nm = np.zeros(st.kind.shape[1], dtype=np.int64)
    for s in range(S):
        if s == centre:
            nm |= np.where(st.kind[s] == 2, 1 << S, 0)
            continue
        vm |= np.where(st.kind[s] == 1, 1 << s, 0)
        nm |= np.where(st.kind[s] == 2, 1 << s, 0)
    return vm, nm
