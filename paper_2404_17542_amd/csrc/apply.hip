// Applying MLS weights (Eq. intrp_chi_1 and its derivatives) and the
// fractional-step glue of Sec. 3.3 / Appendix A.  One thread per DP; the
// weight planes are read coalesced, neighbour field values hit L1/L2.
// Vector fields (velocity components) share one pass over the weights: each
// weight is read once and applied to every component, since the weight
// planes (NB x (S+1) doubles per DP, 2 KB in 3D) are most of the bytes.
#include "common.h"

namespace mcd {

// Phi of NC scalar fields at cell c in one pass over the weight planes:
// Phi[k] = sum_value W_j (f_kj - f_kc) + sum_Neumann W^N_j g_kj, field k at
// fld + k Nc, its Neumann data at fneu + k Nc (fneu may be null).  Per
// component the operations and their order are those of a single field.
// Only basis components q < Q1 are formed (Q1 = DIM: the gradient), the
// others are left 0, so a first-derivative operator reads DIM of the NB
// weight planes.
template <int DIM, int NC, int Q1 = Dims<DIM>::NB, bool FLAT = false>
__device__ __forceinline__ void poly_multi(const MeshDev& m, const SetDev& st, int c, const int ijk[3],
                                           const double* __restrict__ fld, const double* __restrict__ fneu,
                                           double (&Phi)[NC][Dims<DIM>::NB]) {
    constexpr int NB = Dims<DIM>::NB, S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    const size_t Nc = (size_t)m.Nc;
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int q = 0; q < NB; ++q) Phi[k][q] = 0.0;
    const uint32_t vm = st.vmask[c], nm = st.nmask[c];
    if ((vm | nm) == 0) return;
    double fc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) fc[k] = fld[k * Nc + c];
    if constexpr (FLAT) {
        // for a few scattered cells (latency, not throughput, bounds them):
        // every slot without branches, a plane of slots at a time, so that
        // their loads overlap; a slot that is no row of the fit has zero
        // weights (the build writes them) and a zero difference
#pragma unroll 1
        for (int s0 = 0; s0 < S; s0 += 9) {
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int s = s0 + t;
                if (s == CEN) continue;
                const bool v = (vm >> s) & 1u;
                const bool n = fneu != nullptr && ((nm >> s) & 1u);
                int j;
                double sh[3];
                neighbour_or_self<DIM>(m, ijk, s, c, j, sh);
                double d[NC];
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    const double fj = fld[k * Nc + j];
                    const double gj = fneu != nullptr ? fneu[k * Nc + j] : 0.0;
                    d[k] = v ? fj - fc[k] : (n ? gj : 0.0);
                }
#pragma unroll
                for (int q = 0; q < Q1; ++q) {
                    const double w = ld_stream(st.phi + ((size_t)q * (S + 1) + s) * m.mps + c);
#pragma unroll
                    for (int k = 0; k < NC; ++k) Phi[k][q] += w * d[k];
                }
            }
        }
    } else
    for (int s = 0; s < S; ++s) {
        if (s == CEN) continue;
        const bool v = (vm >> s) & 1u;
        const bool n = fneu && ((nm >> s) & 1u);
        if (!v && !n) continue;
        int j;
        double sh[3];
        neighbour<DIM>(m, ijk, s, j, sh);
        double d[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) d[k] = v ? fld[k * Nc + j] - fc[k] : fneu[k * Nc + j];
#pragma unroll
        for (int q = 0; q < Q1; ++q) {
            const double w = ld_stream(st.phi + ((size_t)q * (S + 1) + s) * m.mps + c);
#pragma unroll
            for (int k = 0; k < NC; ++k) Phi[k][q] += w * d[k];
        }
    }
    if (fneu && ((nm >> S) & 1u)) {
#pragma unroll
        for (int q = 0; q < Q1; ++q) {
            const double w = ld_stream(st.phi + ((size_t)q * (S + 1) + S) * m.mps + c);
#pragma unroll
            for (int k = 0; k < NC; ++k) Phi[k][q] += w * fneu[k * Nc + c];
        }
    }
}

// Phi at cell c for scalar field fld: sum_value W_j (f_j - f_c) + sum_Neumann W^N_j g_j.
template <int DIM>
__device__ __forceinline__ void poly_at(const MeshDev& m, const SetDev& st, int c, const int ijk[3],
                                        const double* __restrict__ fld, const double* __restrict__ fneu, double* Phi) {
    constexpr int NB = Dims<DIM>::NB, S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    const size_t Nc = (size_t)m.Nc;
#pragma unroll
    for (int q = 0; q < NB; ++q) Phi[q] = 0.0;
    const uint32_t vm = st.vmask[c], nm = st.nmask[c];
    if ((vm | nm) == 0) return;
    const double fc = fld[c];
    for (int s = 0; s < S; ++s) {
        if (s == CEN) continue;
        const bool v = (vm >> s) & 1u;
        const bool n = fneu && ((nm >> s) & 1u);
        if (!v && !n) continue;
        int j;
        double sh[3];
        neighbour<DIM>(m, ijk, s, j, sh);
        const double d = v ? fld[j] - fc : fneu[j];
#pragma unroll
        for (int q = 0; q < NB; ++q) Phi[q] += ld_stream(st.phi + ((size_t)q * (S + 1) + s) * m.mps + c) * d;
    }
    if (fneu && ((nm >> S) & 1u)) {
        const double fcn = fneu[c];
#pragma unroll
        for (int q = 0; q < NB; ++q) Phi[q] += ld_stream(st.phi + ((size_t)q * (S + 1) + S) * m.mps + c) * fcn;
    }
}

template <int DIM>
__device__ __forceinline__ double taylor(double fc, const double* Phi, const double* shift, double rs) {
    constexpr int NB = Dims<DIM>::NB;
    double X[DIM], p[NB];
#pragma unroll
    for (int a = 0; a < DIM; ++a) X[a] = shift[a] / rs;
    basis<DIM>(X, p);
    double acc = fc;
#pragma unroll
    for (int q = 0; q < NB; ++q) acc += p[q] * Phi[q];
    return acc;
}

// One kernel per operator (OP = MCD_OP_*), so that each keeps only its own
// registers.
template <int DIM, int OP>
__global__ __launch_bounds__(kBlock) void k_apply(MeshDev m, SetDev st, const double* __restrict__ in,
                                                  int ncomp, const double* __restrict__ fneu,
                                                  const double* __restrict__ shift, double* __restrict__ out,
                                                  double scale) {
    constexpr int NB = Dims<DIM>::NB;
    const size_t Nc = (size_t)m.Nc;
    const double rs = st.rs;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        int ijk[3];
        cell_ijk(m, c, ijk);
        double Phi[NB];
        if constexpr (OP == MCD_OP_PHI) {
            poly_at<DIM>(m, st, c, ijk, in, fneu, Phi);
#pragma unroll
            for (int q = 0; q < NB; ++q) out[q * Nc + c] = Phi[q] * scale;
        } else if constexpr (OP == MCD_OP_GRAD) {
            double P1[1][NB];
            poly_multi<DIM, 1, DIM>(m, st, c, ijk, in, fneu, P1);
#pragma unroll
            for (int a = 0; a < DIM; ++a) out[a * Nc + c] = P1[0][a] / rs * scale;
        } else if constexpr (OP == MCD_OP_DIV) {
            double P3[DIM][NB];
            poly_multi<DIM, DIM, DIM>(m, st, c, ijk, in, fneu, P3);
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) acc += P3[a][a] / rs;
            out[c] = acc * scale;
        } else if constexpr (OP == MCD_OP_LAP) {
            if (ncomp == DIM) {
                double P3[DIM][NB];
                poly_multi<DIM, DIM>(m, st, c, ijk, in, fneu, P3);
#pragma unroll
                for (int k = 0; k < DIM; ++k) out[k * Nc + c] = diag2<DIM>(P3[k]) / (rs * rs) * scale;
            } else {
                for (int k = 0; k < ncomp; ++k) {
                    poly_at<DIM>(m, st, c, ijk, in + k * Nc, fneu ? fneu + k * Nc : nullptr, Phi);
                    out[k * Nc + c] = diag2<DIM>(Phi) / (rs * rs) * scale;
                }
            }
        } else {  // MCD_OP_SHIFT
            double sv[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) sv[a] = shift[a * Nc + c];
            if (ncomp == DIM) {
                double P3[DIM][NB];
                poly_multi<DIM, DIM>(m, st, c, ijk, in, fneu, P3);
#pragma unroll
                for (int k = 0; k < DIM; ++k) out[k * Nc + c] = taylor<DIM>(in[k * Nc + c], P3[k], sv, rs);
            } else {
                for (int k = 0; k < ncomp; ++k) {
                    poly_at<DIM>(m, st, c, ijk, in + k * Nc, fneu ? fneu + k * Nc : nullptr, Phi);
                    out[k * Nc + c] = taylor<DIM>(in[k * Nc + c], Phi, sv, rs);
                }
            }
        }
    }
}

// Appendix A remap: u~ = u^k(x^{k+1}) with the step-k weights.  Two
// launches over the cells: TRANS = false takes every cell except the inner
// DPs that were not inner at step k, TRANS = true takes exactly those (the
// shifted support of Eq. A.2); the rare second case kept out of the first
// launch leaves it the registers and schedule of a plain weight application.
template <int DIM, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_remap(MeshDev m, SetDev sp, const double* __restrict__ u,
                                                  const double* __restrict__ pos_prev,
                                                  const double* __restrict__ pos,
                                                  const int8_t* __restrict__ role_prev,
                                                  const int8_t* __restrict__ role, BodiesDev Bp, BodiesDev Bn,
                                                  double* __restrict__ out, int* counters) {
    constexpr int NB = Dims<DIM>::NB;
    const size_t Nc = (size_t)m.Nc;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const int rn = role[c];
        const bool moved_in = rn == MCD_ROLE_INNER && role_prev[c] != MCD_ROLE_INNER;
        if (moved_in != TRANS) continue;
        if (rn == MCD_ROLE_INNER) {
            int src = c;
            const int rp = role_prev[c];
            if constexpr (TRANS) {
                int ijk[3];
                cell_ijk(m, c, ijk);
                int off[3] = {0, 0, 0};
                for (int b = 0; b < Bp.n; ++b) {
                    if (rp != Bp.id[b]) continue;
                    // sign of grad psi at x^k: (x - c) for a circle/sphere
                    double gv[DIM];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) gv[a] = pos_prev[a * Nc + c] - Bp.c[b][a];
                    if (Bp.sdf[b]) {
                        double xp[DIM];
#pragma unroll
                        for (int a = 0; a < DIM; ++a) xp[a] = pos_prev[a * Nc + c];
                        sdf_eval<DIM>(Bp, b, xp, gv);
                    }
#pragma unroll
                    for (int a = 0; a < DIM; ++a) off[a] = gv[a] > 0.0 ? 1 : (gv[a] < 0.0 ? -1 : 0);
                }
                bool ok = true;
                int cp = 0, stride = 1;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const int ii = ijk[a] + off[a];
                    ok = ok && ii >= 0 && ii < m.n[a];
                    cp += (ii < 0 ? 0 : (ii >= m.n[a] ? m.n[a] - 1 : ii)) * stride;
                    stride *= m.n[a];
                }
                const bool good = ok && role_prev[cp] == MCD_ROLE_INNER;
                src = good ? cp : c;
                wave_count_add(&counters[0], good);
                wave_count_add(&counters[1], !good);
            }
            int sijk[3];
            cell_ijk(m, src, sijk);
            double dx[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) dx[a] = pos[a * Nc + c] - pos_prev[a * Nc + src];
            double P3[DIM][NB];
            poly_multi<DIM, DIM, Dims<DIM>::NB, TRANS>(m, sp, src, sijk, u, nullptr, P3);
#pragma unroll
            for (int a = 0; a < DIM; ++a) out[a * Nc + c] = taylor<DIM>(u[a * Nc + src], P3[a], dx, sp.rs);
        } else {
            double v[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) v[a] = 0.0;
            for (int b = 0; b < Bn.n; ++b)
                if (rn == Bn.id[b]) body_velocity<DIM>(Bn, b, pos, Nc, c, v);
#pragma unroll
            for (int a = 0; a < DIM; ++a) out[a * Nc + c] = v[a];
        }
    }
}

// u* = F_MOC + nu dt lap u~ (Eq. intermed_vel) at inner DPs.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_advect_diffuse(MeshDev m, SetDev st, const double* __restrict__ ut,
                                                           double dt, double nu, const double* __restrict__ pos,
                                                           const int8_t* __restrict__ role, BodiesDev B,
                                                           double* __restrict__ ustar) {
    constexpr int NB = Dims<DIM>::NB;
    const size_t Nc = (size_t)m.Nc;
    const double rs = st.rs;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const int rn = role[c];
        if (rn == MCD_ROLE_INNER) {
            int ijk[3];
            cell_ijk(m, c, ijk);
            double sh[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) sh[a] = -ut[a * Nc + c] * dt;
            double P3[DIM][NB];
            poly_multi<DIM, DIM>(m, st, c, ijk, ut, nullptr, P3);
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const double fm = taylor<DIM>(ut[a * Nc + c], P3[a], sh, rs);
                ustar[a * Nc + c] = fm + nu * dt * (diag2<DIM>(P3[a]) / (rs * rs));
            }
        } else {
            double v[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) v[a] = 0.0;
            for (int b = 0; b < B.n; ++b)
                if (rn == B.id[b]) body_velocity<DIM>(B, b, pos, Nc, c, v);
#pragma unroll
            for (int a = 0; a < DIM; ++a) ustar[a * Nc + c] = v[a];
        }
    }
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_neumann_pressure(MeshDev m, const double* __restrict__ pos,
                                                             const int8_t* __restrict__ role,
                                                             const double* __restrict__ normal, BodiesDev B,
                                                             double* __restrict__ f) {
    const size_t Nc = (size_t)m.Nc;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const int rn = role[c];
        double v = 0.0;
        for (int b = 0; b < B.n; ++b)
            if (rn == B.id[b]) v = -body_accel_dot_n<DIM>(B, b, pos, normal, Nc, c);
        f[c] = v;
    }
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_project(MeshDev m, SetDev st, const double* __restrict__ P,
                                                    const double* __restrict__ f, const double* __restrict__ ustar,
                                                    double dt, const double* __restrict__ pos,
                                                    const int8_t* __restrict__ role, BodiesDev B,
                                                    double* __restrict__ u) {
    constexpr int NB = Dims<DIM>::NB;
    const size_t Nc = (size_t)m.Nc;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const int rn = role[c];
        if (rn == MCD_ROLE_INNER) {
            int ijk[3];
            cell_ijk(m, c, ijk);
            double P1[1][NB];
            poly_multi<DIM, 1, DIM>(m, st, c, ijk, P, f, P1);
#pragma unroll
            for (int a = 0; a < DIM; ++a) u[a * Nc + c] = ustar[a * Nc + c] - dt * (P1[0][a] / st.rs);
        } else {
            double v[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) v[a] = 0.0;
            for (int b = 0; b < B.n; ++b)
                if (rn == B.id[b]) body_velocity<DIM>(B, b, pos, Nc, c, v);
#pragma unroll
            for (int a = 0; a < DIM; ++a) u[a * Nc + c] = v[a];
        }
    }
}

// ---------------------------------------------------------------------------
// Fluid force on a moving body (Sec. 3.4, evaluation of fluid forces acting on
// moving boundaries), 2D: F = sum over the body's boundary DPs of t_i dGamma_i,
// t = (-P I + mu (grad u + grad u^T)) . n.  One block per body: the body's
// boundary DPs (found in a box around it) are ordered by a libm-free polar
// angle about the body centre; dGamma_i is the mean distance to the angular
// predecessor and successor; P and grad u at x_i come from the fit of the
// cell shifted by sign(n) (per axis), evaluated at x_i (chi_c = 1
// reconstruction), or from the DP's own fit when that cell is not inner.
// ---------------------------------------------------------------------------

constexpr int kForceMax = 4096;      // boundary DPs per body
constexpr int kForceBlock = 1024;

struct ForceBoxes {
    int lo[kMaxBodies][2], hi[kMaxBodies][2];
};

// monotone stand-in for the polar angle in [0, 4), from + - / only
__device__ __forceinline__ double diamond_angle(double dx, double dy) {
#pragma clang fp contract(off)
    if (dy >= 0.0) return dx >= 0.0 ? dy / (dx + dy) : 1.0 - dx / (-dx + dy);
    return dx < 0.0 ? 2.0 - dy / (-dx - dy) : 3.0 + dx / (dx - dy);
}

__device__ __forceinline__ double seg_len(const double* __restrict__ pos, size_t Nc, int a, int b) {
#pragma clang fp contract(off)
    const double dx = pos[a] - pos[b], dy = pos[Nc + a] - pos[Nc + b];
    return sqrt(dx * dx + dy * dy);
}

__global__ __launch_bounds__(kForceBlock) void k_force(MeshDev m, SetDev su, SetDev sp, const double* __restrict__ u,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ fneu,
                                                      const double* __restrict__ pos,
                                                      const int8_t* __restrict__ role,
                                                      const double* __restrict__ normal, BodiesDev B, ForceBoxes box,
                                                      double mu, double* __restrict__ out, int* __restrict__ cnt) {
    __shared__ int list[kForceMax];
    __shared__ double key[kForceMax];
    __shared__ double fy[kForceMax];
    __shared__ int count, fallbacks;
    const int b = blockIdx.x;
    const size_t Nc = (size_t)m.Nc;
    const double rs = su.rs;
    if (threadIdx.x == 0) {
        count = 0;
        fallbacks = 0;
    }
    __syncthreads();
    // 1. the body's boundary DPs in its box (in arbitrary order)
    const int nx = box.hi[b][0] - box.lo[b][0] + 1, ny = box.hi[b][1] - box.lo[b][1] + 1;
    for (int e = threadIdx.x; e < nx * ny; e += kForceBlock) {
        const int c = box.lo[b][0] + e % nx + m.n[0] * (box.lo[b][1] + e / nx);
        if (role[c] == B.id[b]) {
            const int k = atomicAdd(&count, 1);
            if (k < kForceMax) list[k] = c;
        }
    }
    __syncthreads();
    const int n = count;
    if (n > kForceMax || n == 0) {
        if (threadIdx.x == 0) {
            out[2 * b] = 0.0;
            out[2 * b + 1] = 0.0;
            cnt[3 * b] = n;
            cnt[3 * b + 1] = 0;
            cnt[3 * b + 2] = n > kForceMax ? 1 : 0;
        }
        return;
    }
    // 2. sort by (angle, cell index): bitonic over the next power of two
    int P2 = 1;
    while (P2 < n) P2 <<= 1;
    for (int k = threadIdx.x; k < P2; k += kForceBlock) {
        if (k < n) {
            const int c = list[k];
            key[k] = diamond_angle(pos[c] - B.c[b][0], pos[Nc + c] - B.c[b][1]);
        } else {
            key[k] = 1e300;
            list[k] = 0x7fffffff;
        }
    }
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P2; i += kForceBlock) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const bool gt = key[i] > key[l] || (key[i] == key[l] && list[i] > list[l]);
                    if (gt == up) {
                        const double tk = key[i];
                        key[i] = key[l];
                        key[l] = tk;
                        const int tl = list[i];
                        list[i] = list[l];
                        list[l] = tl;
                    }
                }
            }
            __syncthreads();
        }
    }
    // 3. traction times surface element per DP, in sorted order (key reused for the x part)
    double fx_k[kForceMax / kForceBlock], fy_k[kForceMax / kForceBlock];
    int nk = 0;
    for (int k = threadIdx.x; k < n; k += kForceBlock, ++nk) {
        const int c = list[k];
        const int cp = list[(k + n - 1) % n], cn = list[(k + 1) % n];
        const double dgam = 0.5 * (seg_len(pos, Nc, c, cp) + seg_len(pos, Nc, c, cn));
        int ijk[3];
        cell_ijk(m, c, ijk);
        const double nv[2] = {normal[c], normal[Nc + c]};
        const int ii = ijk[0] + (nv[0] > 0.0 ? 1 : (nv[0] < 0.0 ? -1 : 0));
        const int jj = ijk[1] + (nv[1] > 0.0 ? 1 : (nv[1] < 0.0 ? -1 : 0));
        int ci = -1;
        if (ii >= 0 && ii < m.n[0] && jj >= 0 && jj < m.n[1]) ci = ii + m.n[0] * jj;
        if (ci < 0 || role[ci] != MCD_ROLE_INNER) {
            ci = c;
            atomicAdd(&fallbacks, 1);
        }
        int cijk[3];
        cell_ijk(m, ci, cijk);
        double Pu[2][5], Pp[1][5];
        poly_multi<2, 2>(m, su, ci, cijk, u, nullptr, Pu);
        poly_multi<2, 1>(m, sp, ci, cijk, p, fneu, Pp);
        const double X[2] = {(pos[c] - pos[ci]) / rs, (pos[Nc + c] - pos[Nc + ci]) / rs};
        double pv[5];
        basis<2>(X, pv);
        double P = p[ci];
#pragma unroll
        for (int q = 0; q < 5; ++q) P += pv[q] * Pp[0][q];
        // d p / d X_x = (1, 0, X, Y, 0), d p / d X_y = (0, 1, 0, X, Y)
        double G[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            G[a][0] = (Pu[a][0] + X[0] * Pu[a][2] + X[1] * Pu[a][3]) / rs;
            G[a][1] = (Pu[a][1] + X[0] * Pu[a][3] + X[1] * Pu[a][4]) / rs;
        }
        double t[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            t[a] = -P * nv[a];
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) t[a] += mu * (G[a][bb] + G[bb][a]) * nv[bb];
        }
        fx_k[nk] = t[0] * dgam;
        fy_k[nk] = t[1] * dgam;
    }
    __syncthreads();      // every thread is done reading key and list
    nk = 0;
    for (int k = threadIdx.x; k < n; k += kForceBlock, ++nk) {
        key[k] = fx_k[nk];
        fy[k] = fy_k[nk];
    }
    __syncthreads();
    // 4. sums in the sorted order
    if (threadIdx.x == 0) {
        double sx = 0.0, sy = 0.0;
        for (int k = 0; k < n; ++k) {
            sx += key[k];
            sy += fy[k];
        }
        out[2 * b] = sx;
        out[2 * b + 1] = sy;
        cnt[3 * b] = n;
        cnt[3 * b + 1] = fallbacks;
        cnt[3 * b + 2] = 0;
    }
}

hipError_t launch_force(const MeshDev& m, const SetDev& su, const SetDev& sp, const double* u, const double* p,
                        const double* fneu, const double* pos, const int8_t* role, const double* normal,
                        const BodiesDev& B, double mu, double* out, int* cnt, hipStream_t st) {
    ForceBoxes box{};
    for (int b = 0; b < B.n; ++b)
        for (int a = 0; a < 2; ++a) {
            // cells within R + 2 l0 of the centre hold every boundary DP of the body
            const double ext = B.R[b] + 2.0 * m.l0;
            int lo = (int)floor((B.c[b][a] - ext - m.origin[a]) / m.l0);
            int hi = (int)floor((B.c[b][a] + ext - m.origin[a]) / m.l0);
            box.lo[b][a] = lo < 0 ? 0 : (lo >= m.n[a] ? m.n[a] - 1 : lo);
            box.hi[b][a] = hi < 0 ? 0 : (hi >= m.n[a] ? m.n[a] - 1 : hi);
        }
    hipLaunchKernelGGL(k_force, dim3(B.n), dim3(kForceBlock), 0, st, m, su, sp, u, p, fneu, pos, role, normal, B, box,
                       mu, out, cnt);
    return hipGetLastError();
}

static inline int grid_cells(int n) {
    int g = (n + kBlock - 1) / kBlock;
    return g < 1 ? 1 : (g > 8192 ? 8192 : g);
}

#define MCD_DISPATCH(KERNEL, ...)                                                                       \
    do {                                                                                                \
        if (m.dim == 2)                                                                                 \
            hipLaunchKernelGGL(KERNEL<2>, dim3(grid_cells(m.Nc)), dim3(kBlock), 0, st, __VA_ARGS__);    \
        else                                                                                            \
            hipLaunchKernelGGL(KERNEL<3>, dim3(grid_cells(m.Nc)), dim3(kBlock), 0, st, __VA_ARGS__);    \
    } while (0)

template <int OP>
static void launch_apply_op(const MeshDev& m, const SetDev& set, const double* in, int ncomp, const double* fneu,
                            const double* shift, double* out, double scale, hipStream_t st) {
    const dim3 g(grid_cells(m.Nc));
    if (m.dim == 2)
        hipLaunchKernelGGL((k_apply<2, OP>), g, dim3(kBlock), 0, st, m, set, in, ncomp, fneu, shift, out, scale);
    else
        hipLaunchKernelGGL((k_apply<3, OP>), g, dim3(kBlock), 0, st, m, set, in, ncomp, fneu, shift, out, scale);
}

hipError_t launch_apply(const MeshDev& m, const SetDev& set, int op, const double* in, int ncomp,
                        const double* fneu, const double* shift, double* out, double scale, hipStream_t st) {
    switch (op) {
        case MCD_OP_PHI: launch_apply_op<MCD_OP_PHI>(m, set, in, ncomp, fneu, shift, out, scale, st); break;
        case MCD_OP_GRAD: launch_apply_op<MCD_OP_GRAD>(m, set, in, ncomp, fneu, shift, out, scale, st); break;
        case MCD_OP_DIV: launch_apply_op<MCD_OP_DIV>(m, set, in, ncomp, fneu, shift, out, scale, st); break;
        case MCD_OP_LAP: launch_apply_op<MCD_OP_LAP>(m, set, in, ncomp, fneu, shift, out, scale, st); break;
        default: launch_apply_op<MCD_OP_SHIFT>(m, set, in, ncomp, fneu, shift, out, scale, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_remap(const MeshDev& m, const SetDev& set_prev, const double* u, const double* pos_prev,
                        const double* pos, const int8_t* role_prev, const int8_t* role, const BodiesDev& Bprev,
                        const BodiesDev& Bnew, double* out, int* counters, hipStream_t st) {
    const dim3 g(grid_cells(m.Nc));
    if (m.dim == 2) {
        hipLaunchKernelGGL((k_remap<2, false>), g, dim3(kBlock), 0, st, m, set_prev, u, pos_prev, pos, role_prev, role,
                           Bprev, Bnew, out, counters);
        hipLaunchKernelGGL((k_remap<2, true>), g, dim3(kBlock), 0, st, m, set_prev, u, pos_prev, pos, role_prev, role,
                           Bprev, Bnew, out, counters);
    } else {
        hipLaunchKernelGGL((k_remap<3, false>), g, dim3(kBlock), 0, st, m, set_prev, u, pos_prev, pos, role_prev, role,
                           Bprev, Bnew, out, counters);
        hipLaunchKernelGGL((k_remap<3, true>), g, dim3(kBlock), 0, st, m, set_prev, u, pos_prev, pos, role_prev, role,
                           Bprev, Bnew, out, counters);
    }
    return hipGetLastError();
}

hipError_t launch_advect_diffuse(const MeshDev& m, const SetDev& set, const double* ut, double dt, double nu,
                                 const double* pos, const int8_t* role, const BodiesDev& B, double* ustar,
                                 hipStream_t st) {
    MCD_DISPATCH(k_advect_diffuse, m, set, ut, dt, nu, pos, role, B, ustar);
    return hipGetLastError();
}

hipError_t launch_neumann_pressure(const MeshDev& m, const double* pos, const int8_t* role, const double* normal,
                                   const BodiesDev& B, double* f, hipStream_t st) {
    MCD_DISPATCH(k_neumann_pressure, m, pos, role, normal, B, f);
    return hipGetLastError();
}

hipError_t launch_project(const MeshDev& m, const SetDev& set, const double* P, const double* f,
                          const double* ustar, double dt, const double* pos, const int8_t* role, const BodiesDev& B,
                          double* u, hipStream_t st) {
    MCD_DISPATCH(k_project, m, set, P, f, ustar, dt, pos, role, B, u);
    return hipGetLastError();
}

}  // namespace mcd
