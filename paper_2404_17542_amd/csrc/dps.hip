// DP masking, rearrangement and normals (Sec. 2.2 - 2.4).
//
// Bit-exact contract: every floating-point result here is produced by the
// same sequence of correctly rounded + - * / sqrt min max as the reference
// definition, so contraction into fused multiply-adds is switched off for
// the whole file (and the file is compiled with -ffp-contract=off).
#pragma clang fp contract(off)

#include "common.h"

namespace mcd {

// ---------------------------------------------------------------------------
// Masks from vertex SDF signs, transition codes, band flags, wall projection
// ---------------------------------------------------------------------------

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_roles(MeshDev m, BodiesDev B, double band_l0, int8_t* role,
                                                  int8_t* role_prev, double* pos, double* pos_prev,
                                                  uint8_t* trans, uint8_t* band, int* counts, int* latch) {
    __shared__ int hist[11];
    if (threadIdx.x < 11) hist[threadIdx.x] = 0;
    __syncthreads();
    const size_t Nc = (size_t)m.Nc;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        int ijk[3];
        cell_ijk(m, c, ijk);
        const int old = role[c];
        role_prev[c] = (int8_t)old;
        double x[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            x[a] = pos[a * Nc + c];
            pos_prev[a * Nc + c] = x[a];
        }
        // vertices with psi >= 0 (outside every body): |v - c|^2 >= R^2 for a
        // circle/sphere, the interpolated psi for a discrete SDF
        int count = 0;
#pragma unroll
        for (int v = 0; v < (1 << DIM); ++v) {
            double vx[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) vx[a] = m.origin[a] + (double)(ijk[a] + ((v >> a) & 1)) * m.l0;
            bool fluid = true;
            for (int b = 0; b < B.n; ++b) {
                if (B.sdf[b]) {
                    double g[DIM];
                    fluid = fluid && (sdf_eval<DIM>(B, b, vx, g) >= 0.0);
                    continue;
                }
                double d2 = 0.0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    double da = vx[a] - B.c[b][a];
                    d2 = d2 + da * da;
                }
                fluid = fluid && (d2 >= B.R2[b]);
            }
            count += fluid ? 1 : 0;
        }
        const int full = 1 << DIM, half = full >> 1;
        int r = (count == full) ? MCD_ROLE_INNER : (count >= half ? 1 : MCD_ROLE_VOID);
        // nearest body at the centroid: boundary id and band membership
        double best = INFINITY;
        int best_id = 0;
        if (B.n > 0) {
            double cen[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) cen[a] = m.origin[a] + ((double)ijk[a] + 0.5) * m.l0;
            for (int b = 0; b < B.n; ++b) {
                double apsi;
                bool done = false;
                if (B.sdf[b]) {
                    double g[DIM];
                    apsi = fabs(sdf_eval<DIM>(B, b, cen, g));
                    done = true;
                }
                if (!done) {
                    double d2 = 0.0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        double da = cen[a] - B.c[b][a];
                        d2 = d2 + da * da;
                    }
                    apsi = fabs(sqrt(d2) - B.R[b]);
                }
                if (apsi < best) {
                    best = apsi;
                    best_id = B.id[b];
                }
            }
            if (r == 1) r = best_id;
        }
        bool wall = false;
        if (m.walls) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) wall = wall || ijk[a] == 0 || ijk[a] == m.n[a] - 1;
        }
        if (wall) {
            r = m.wall_id;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                if (ijk[a] == 0) pos[a * Nc + c] = m.origin[a];
                if (ijk[a] == m.n[a] - 1) pos[a * Nc + c] = m.origin[a] + (double)m.n[a] * m.l0;
            }
        }
        role[c] = (int8_t)r;
        const int co = old == 0 ? 0 : (old < 0 ? 1 : 2);
        const int cn = r == 0 ? 0 : (r < 0 ? 1 : 2);
        const int code = 3 * co + cn;
        trans[c] = (uint8_t)code;
        const bool inband = (r != MCD_ROLE_VOID) && !wall && (best < band_l0);
        band[c] = inband ? 1 : 0;
        atomicAdd(&hist[code], 1);
        if (inband) atomicAdd(&hist[9], 1);
        if (code == 1 || code == 3) atomicAdd(&hist[10], 1);
    }
    __syncthreads();
    if (threadIdx.x < 11 && hist[threadIdx.x] != 0) atomicAdd(&counts[threadIdx.x], hist[threadIdx.x]);
    if (threadIdx.x == 10 && hist[10] != 0) atomicAdd(latch, hist[10]);
}

// ---------------------------------------------------------------------------
// One Jacobi relaxation sweep over the band (spring forces, SDF projection,
// mesh-constraint clamp) with an exact max-displacement reduction.
// state[0]: converged flag, state[1]: sweeps executed.
// ---------------------------------------------------------------------------

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_relax(MeshDev m, BodiesDev B, double kl0, double sp1, double sp2,
                                                  double sp3, double eps_l0, FitDev fit,
                                                  const int8_t* __restrict__ role,
                                                  const uint8_t* __restrict__ band, const double* __restrict__ pin,
                                                  double* __restrict__ pout, int lo0, int lo1, int lo2, int bn0,
                                                  int bn1, int bn2, unsigned long long* dmax, int sweep,
                                                  int* state) {
    __shared__ double red[kBlock / 64];
    const bool done = state[0] != 0 || (sweep > 0 && __longlong_as_double((long long)dmax[sweep - 1]) <= eps_l0);
    if (done && blockIdx.x == 0 && threadIdx.x == 0) state[0] = 1;
    const size_t Nc = (size_t)m.Nc;
    const int nbox = bn0 * bn1 * bn2;
    double local = 0.0;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nbox; q += gridDim.x * blockDim.x) {
        int ijk[3];
        ijk[0] = lo0 + q % bn0;
        ijk[1] = lo1 + (q / bn0) % bn1;
        ijk[2] = lo2 + q / (bn0 * bn1);
        const int c = ijk[0] + m.n[0] * (ijk[1] + m.n[1] * ijk[2]);
        if (!band[c]) continue;
        double x[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) x[a] = pin[a * Nc + c];
        if (done) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) pout[a * Nc + c] = x[a];
            continue;
        }
        double F[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) F[a] = 0.0;
        constexpr int S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
        // every slot without branches, so that the square roots and divisions
        // of different neighbours overlap; a slot that is no spring (outside
        // the mesh, a void neighbour, a coincident one) adds an exact zero,
        // which leaves the sum's bits unchanged (F is never -0)
#pragma unroll 1
        for (int s0 = 0; s0 < S; s0 += 9) {      // one plane of 3 x 3 slots at a time
#pragma unroll
          for (int t = 0; t < 9; ++t) {
            const int s = s0 + t;
            if (s == CEN) continue;
            int j;
            double sh[3];
            const bool inm = neighbour_or_self<DIM>(m, ijk, s, c, j, sh);
            const bool live = inm && role[j] != MCD_ROLE_VOID;
            double d[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) d[a] = (pin[a * Nc + j] + sh[a]) - x[a];
            double d2 = d[0] * d[0];
#pragma unroll
            for (int a = 1; a < DIM; ++a) d2 = d2 + d[a] * d[a];
            const double dist = sqrt(d2);
            const bool ok = live && dist > 0.0;   // a coincident neighbour has no direction
            const int nz = slot_nonzeros<DIM>(s);
            const double L = nz == 1 ? sp1 : (nz == 2 ? sp2 : sp3);
            const double g = 1.0 - dist / L;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const double term = g * (d[a] / dist);
                F[a] = F[a] + (ok ? term : 0.0);
            }
          }
        }
        double xs[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) xs[a] = x[a] - kl0 * F[a];
        const int rc = role[c];
        for (int b = 0; b < B.n; ++b) {
            if (rc != B.id[b]) continue;
            if (B.sdf[b]) {
                // x** = x* - psi grad psi / |grad psi|
                double g[DIM];
                const double psi = sdf_eval<DIM>(B, b, xs, g);
                double g2 = g[0] * g[0];
#pragma unroll
                for (int a = 1; a < DIM; ++a) g2 = g2 + g[a] * g[a];
                const double t = psi / sqrt(g2);
#pragma unroll
                for (int a = 0; a < DIM; ++a) xs[a] = xs[a] - t * g[a];
                continue;
            }
            double dd[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) dd[a] = xs[a] - B.c[b][a];
            double r2 = dd[0] * dd[0];
#pragma unroll
            for (int a = 1; a < DIM; ++a) r2 = r2 + dd[a] * dd[a];
            const double r = sqrt(r2);
            const double psi = r - B.R[b];
            const double t = psi / r;
#pragma unroll
            for (int a = 0; a < DIM; ++a) xs[a] = xs[a] - t * dd[a];
        }
        if (fit.half_alpha > 0.0 && rc == MCD_ROLE_INNER && B.n > 0) {
            // boundary-fitted arrangement: towards the nearest body (bodies
            // are in ascending id order; ties keep the lower id)
            double best = 0.0, rb = 1.0, db[DIM];
            for (int b = 0; b < B.n; ++b) {
                // direction and its norm: (x - c, |x - c|), or (grad psi, |grad psi|)
                double dd[DIM], r, psi;
                bool done = false;
                if (B.sdf[b]) {
                    psi = sdf_eval<DIM>(B, b, xs, dd);
                    double g2 = dd[0] * dd[0];
#pragma unroll
                    for (int a = 1; a < DIM; ++a) g2 = g2 + dd[a] * dd[a];
                    r = sqrt(g2);
                    done = true;
                }
                if (!done) {
#pragma unroll
                    for (int a = 0; a < DIM; ++a) dd[a] = xs[a] - B.c[b][a];
                    double r2 = dd[0] * dd[0];
#pragma unroll
                    for (int a = 1; a < DIM; ++a) r2 = r2 + dd[a] * dd[a];
                    r = sqrt(r2);
                    psi = r - B.R[b];
                }
                if (b == 0 || psi < best) {
                    best = psi;
                    rb = r;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) db[a] = dd[a];
                }
            }
            if (best < fit.re) {
                const double beta = fit.half_alpha * (1.0 + series_cos(best * fit.pi_over_re));
                const double t = (beta * best) / rb;
#pragma unroll
                for (int a = 0; a < DIM; ++a) xs[a] = xs[a] - t * db[a];
            }
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double lo = m.origin[a] + (double)ijk[a] * m.l0;
            const double hi = m.origin[a] + (double)(ijk[a] + 1) * m.l0;
            const double xn = fmin(fmax(xs[a], lo), hi);
            pout[a * Nc + c] = xn;
            local = fmax(local, fabs(xn - x[a]));
        }
    }
    if (done) return;
    double w = wave_max(local);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = red[0];
        for (int q = 1; q < kBlock / 64; ++q) v = fmax(v, red[q]);
        // non-negative doubles order like their bit patterns
        atomicMax(&dmax[sweep], (unsigned long long)__double_as_longlong(v));
        if (blockIdx.x == 0) state[1] = sweep + 1;
    }
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_copy_band(MeshDev m, const uint8_t* band, const double* src, double* dst,
                                                      int lo0, int lo1, int lo2, int bn0, int bn1, int bn2) {
    const size_t Nc = (size_t)m.Nc;
    const int nbox = bn0 * bn1 * bn2;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nbox; q += gridDim.x * blockDim.x) {
        const int c = (lo0 + q % bn0) + m.n[0] * ((lo1 + (q / bn0) % bn1) + m.n[1] * (lo2 + q / (bn0 * bn1)));
        if (!band[c]) continue;
#pragma unroll
        for (int a = 0; a < DIM; ++a) dst[a * Nc + c] = src[a * Nc + c];
    }
}

// Unit normal into the fluid: body DPs (x - c)/|x - c|; wall DPs the sum of
// the inward axis normals of the walls the cell touches, normalised.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_normals(MeshDev m, BodiesDev B, const int8_t* role, const double* pos,
                                                    double* normal) {
    const size_t Nc = (size_t)m.Nc;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const int r = role[c];
        double nv[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) nv[a] = 0.0;
        if (m.walls && r == m.wall_id) {
            int ijk[3];
            cell_ijk(m, c, ijk);
            double sv[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) sv[a] = ijk[a] == 0 ? 1.0 : (ijk[a] == m.n[a] - 1 ? -1.0 : 0.0);
            double s2 = sv[0] * sv[0];
#pragma unroll
            for (int a = 1; a < DIM; ++a) s2 = s2 + sv[a] * sv[a];
            const double nn = sqrt(s2);
#pragma unroll
            for (int a = 0; a < DIM; ++a) nv[a] = sv[a] / nn;
        } else if (r >= 1) {
            for (int b = 0; b < B.n; ++b) {
                if (r != B.id[b]) continue;
                if (B.sdf[b]) {
                    double xp[DIM], g[DIM];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) xp[a] = pos[a * Nc + c];
                    sdf_eval<DIM>(B, b, xp, g);
                    double g2 = g[0] * g[0];
#pragma unroll
                    for (int a = 1; a < DIM; ++a) g2 = g2 + g[a] * g[a];
                    const double gn = sqrt(g2);
#pragma unroll
                    for (int a = 0; a < DIM; ++a) nv[a] = g[a] / gn;
                    continue;
                }
                double dd[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) dd[a] = pos[a * Nc + c] - B.c[b][a];
                double r2 = dd[0] * dd[0];
#pragma unroll
                for (int a = 1; a < DIM; ++a) r2 = r2 + dd[a] * dd[a];
                const double rr = sqrt(r2);
#pragma unroll
                for (int a = 0; a < DIM; ++a) nv[a] = dd[a] / rr;
            }
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) normal[a * Nc + c] = nv[a];
    }
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_i32(int* p, int n, int v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static inline int grid_for(long long n) {
    long long g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

hipError_t launch_roles(const MeshDev& m, const BodiesDev& B, double band_l0, int8_t* role, int8_t* role_prev,
                        double* pos, double* pos_prev, uint8_t* trans, uint8_t* band, int* counts,
                        int* latch, hipStream_t st) {
    const int g = grid_for(m.Nc);
    if (m.dim == 2)
        hipLaunchKernelGGL(k_roles<2>, dim3(g), dim3(kBlock), 0, st, m, B, band_l0, role, role_prev, pos, pos_prev,
                           trans, band, counts, latch);
    else
        hipLaunchKernelGGL(k_roles<3>, dim3(g), dim3(kBlock), 0, st, m, B, band_l0, role, role_prev, pos, pos_prev,
                           trans, band, counts, latch);
    return hipGetLastError();
}

hipError_t launch_relax(const MeshDev& m, const BodiesDev& B, double kl0, const double* spring, double eps_l0,
                        const FitDev& fit, const int8_t* role, const uint8_t* band, const double* pin, double* pout,
                        const int box_lo[3], const int box_n[3], unsigned long long* dmax, int sweep,
                        int* state, hipStream_t st) {
    const long long nbox = (long long)box_n[0] * box_n[1] * box_n[2];
    const int g = grid_for(nbox);
    if (m.dim == 2)
        hipLaunchKernelGGL(k_relax<2>, dim3(g), dim3(kBlock), 0, st, m, B, kl0, spring[1], spring[2], spring[3],
                           eps_l0, fit, role, band, pin, pout, box_lo[0], box_lo[1], box_lo[2], box_n[0], box_n[1],
                           box_n[2], dmax, sweep, state);
    else
        hipLaunchKernelGGL(k_relax<3>, dim3(g), dim3(kBlock), 0, st, m, B, kl0, spring[1], spring[2], spring[3],
                           eps_l0, fit, role, band, pin, pout, box_lo[0], box_lo[1], box_lo[2], box_n[0], box_n[1],
                           box_n[2], dmax, sweep, state);
    return hipGetLastError();
}

hipError_t launch_copy_band(const MeshDev& m, const uint8_t* band, const double* src, double* dst,
                            const int box_lo[3], const int box_n[3], hipStream_t st) {
    const long long nbox = (long long)box_n[0] * box_n[1] * box_n[2];
    const int g = grid_for(nbox);
    if (m.dim == 2)
        hipLaunchKernelGGL(k_copy_band<2>, dim3(g), dim3(kBlock), 0, st, m, band, src, dst, box_lo[0], box_lo[1],
                           box_lo[2], box_n[0], box_n[1], box_n[2]);
    else
        hipLaunchKernelGGL(k_copy_band<3>, dim3(g), dim3(kBlock), 0, st, m, band, src, dst, box_lo[0], box_lo[1],
                           box_lo[2], box_n[0], box_n[1], box_n[2]);
    return hipGetLastError();
}

hipError_t launch_normals(const MeshDev& m, const BodiesDev& B, const int8_t* role, const double* pos,
                          double* normal, hipStream_t st) {
    const int g = grid_for(m.Nc);
    if (m.dim == 2)
        hipLaunchKernelGGL(k_normals<2>, dim3(g), dim3(kBlock), 0, st, m, B, role, pos, normal);
    else
        hipLaunchKernelGGL(k_normals<3>, dim3(g), dim3(kBlock), 0, st, m, B, role, pos, normal);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace mcd
