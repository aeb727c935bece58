// MLS stencil build (Sec. 3.2, chi_c = 1): one thread per DP, FP64.
//
// For DP c the fit minimises J of Eq. (obj_func) with phi_c fixed:
//   M Phi = sum_value w_j p_j (phi_j - phi_c) + sum_Neumann w_j pN_j r_s f_j,
//   M     = sum_value w_j p_j p_j^T + sum_Neumann w_j pN_j pN_j^T.
// Pass 1 gathers the 3x3(x3) block and accumulates M (packed lower
// triangle, registers); M is Cholesky-factored in registers; pass 2
// re-gathers each row and writes W_j = M^-1 (w_j a_j) into the slot planes
// (coalesced: consecutive threads write consecutive cells of a plane), plus
// the PPE Laplacian matrix over unknown rows/columns in FP64 and FP32.
#include "common.h"

namespace mcd {

__device__ __forceinline__ double mls_weight(double r, double re, int kind) {
    if (r > re) return 0.0;
    if (kind == MCD_WEIGHT_COS2) {
        const double t = cos(M_PI * r / (2.0 * re));
        return t * t;
    }
    return exp(-4.0 * r * r / (re * re));
}

template <int DIM>
__device__ __forceinline__ int row_of(const MeshDev& m, const double* __restrict__ pos, const int8_t* __restrict__ role,
                                      const double* __restrict__ normal, const BcDev& bc, const int ijk[3],
                                      const double* xc, int s, double re, double rs, int wkind, int& j, double& w,
                                      double* a) {
    constexpr int CEN = Dims<DIM>::CEN;
    double sh[3];
    if (!neighbour<DIM>(m, ijk, s, j, sh)) return 0;
    int kind = row_kind(role[j], bc);
    if (s == CEN && kind != 2) return 0;   // the DP itself: only its Neumann row
    if (kind == 0) return 0;
    const size_t Nc = (size_t)m.Nc;
    double d[DIM], X[DIM];
    double r2 = 0.0;
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        d[q] = (pos[q * Nc + j] + sh[q]) - xc[q];
        r2 += d[q] * d[q];
        X[q] = d[q] / rs;
    }
    w = mls_weight(sqrt(r2), re, wkind);
    if (kind == 1) {
        basis<DIM>(X, a);
    } else {
        double nv[DIM];
#pragma unroll
        for (int q = 0; q < DIM; ++q) nv[q] = normal[q * Nc + j];
        basis_normal<DIM>(X, nv, a);
    }
    return kind;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_mls_build(MeshDev m, const double* __restrict__ pos,
                                                      const int8_t* __restrict__ role,
                                                      const double* __restrict__ normal, BcDev bc, double re,
                                                      double rs, int wkind, SetDev st, int* counters,
                                                      int* latch) {
    constexpr int NB = Dims<DIM>::NB, S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    constexpr int NP = NB * (NB + 1) / 2;
    const size_t Nc = (size_t)m.Nc;
    const int nblk = gridDim.x;
    const int lb = xcd_block(blockIdx.x, nblk);
    for (int c = lb * blockDim.x + threadIdx.x; c < m.Nc; c += nblk * blockDim.x) {
        const int rc = role[c];
        int ijk[3];
        cell_ijk(m, c, ijk);
        double xc[DIM];
#pragma unroll
        for (int q = 0; q < DIM; ++q) xc[q] = pos[q * Nc + c];
        const bool unk_c = is_unknown(rc, c, bc);
        st.unknown[c] = unk_c ? 1 : 0;
        double M[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) M[q] = 0.0;
        uint32_t vm = 0, nm = 0;
        int nrows = 0;
        if (rc != MCD_ROLE_VOID) {
            for (int s = 0; s < S; ++s) {
                int j;
                double w, a[NB];
                const int kind = row_of<DIM>(m, pos, role, normal, bc, ijk, xc, s, re, rs, wkind, j, w, a);
                if (!kind) continue;
                if (kind == 1)
                    vm |= 1u << s;
                else
                    nm |= 1u << (s == CEN ? S : s);
                nrows += (w > 0.0) ? 1 : 0;
                int q = 0;
#pragma unroll
                for (int r = 0; r < NB; ++r) {
                    const double wa = w * a[r];
#pragma unroll
                    for (int k = 0; k <= r; ++k) M[q++] += wa * a[k];
                }
            }
        }
        // Cholesky M = L L^T in place (packed lower triangle); the diagonal
        // slots keep 1 / L_jj, so that the triangular solves of pass 2
        // multiply instead of divide
        double tr = 0.0;
#pragma unroll
        for (int r = 0; r < NB; ++r) tr += M[r * (r + 1) / 2 + r];
        bool sing = (rc == MCD_ROLE_VOID);
        if (!sing) {
            // fewer rows of positive weight than basis terms: M is rank-deficient
            if (nrows < NB) sing = true;
#pragma unroll
            for (int jc = 0; jc < NB; ++jc) {
                double dsum = M[jc * (jc + 1) / 2 + jc];
#pragma unroll
                for (int k = 0; k < jc; ++k) dsum -= M[jc * (jc + 1) / 2 + k] * M[jc * (jc + 1) / 2 + k];
                if (!(dsum > 1e-12 * tr / NB)) {
                    sing = true;
                    dsum = 1.0;
                }
                const double ljj = sqrt(dsum);
                const double inv = 1.0 / ljj;
                M[jc * (jc + 1) / 2 + jc] = inv;
#pragma unroll
                for (int i = jc + 1; i < NB; ++i) {
                    double acc = M[i * (i + 1) / 2 + jc];
#pragma unroll
                    for (int k = 0; k < jc; ++k) acc -= M[i * (i + 1) / 2 + k] * M[jc * (jc + 1) / 2 + k];
                    M[i * (i + 1) / 2 + jc] = acc * inv;
                }
            }
            if (sing) {
                atomicAdd(&counters[rc == MCD_ROLE_INNER ? 0 : 1], 1);
                if (rc == MCD_ROLE_INNER) {
                    atomicMin(&counters[2], c);
                    atomicAdd(latch, 1);
                }
            }
        }
        if (sing) {
            vm = 0;
            nm = 0;
        }
        st.vmask[c] = vm;
        st.nmask[c] = nm;
        double cacc[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) cacc[q] = 0.0;
        double diag_sum = 0.0, off_sum = 0.0;
        for (int s = 0; s < S; ++s) {
            const int slot = (s == CEN) ? S : s;
            const bool isv = (vm >> s) & 1u, isn = (nm >> slot) & 1u;
            double y[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) y[q] = 0.0;
            int j = -1;
            if (isv || isn) {
                double w, a[NB];
                row_of<DIM>(m, pos, role, normal, bc, ijk, xc, s, re, rs, wkind, j, w, a);
#pragma unroll
                for (int q = 0; q < NB; ++q) y[q] = w * a[q];
                // forward L z = y, backward L^T y = z
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    double acc = y[i];
#pragma unroll
                    for (int k = 0; k < i; ++k) acc -= M[i * (i + 1) / 2 + k] * y[k];
                    y[i] = acc * M[i * (i + 1) / 2 + i];
                }
#pragma unroll
                for (int i = NB - 1; i >= 0; --i) {
                    double acc = y[i];
#pragma unroll
                    for (int k = i + 1; k < NB; ++k) acc -= M[k * (k + 1) / 2 + i] * y[k];
                    y[i] = acc * M[i * (i + 1) / 2 + i];
                }
                if (isn) {
#pragma unroll
                    for (int q = 0; q < NB; ++q) y[q] *= rs;
                } else {
#pragma unroll
                    for (int q = 0; q < NB; ++q) cacc[q] += y[q];
                }
            }
            if (s != CEN) {
#pragma unroll
                for (int q = 0; q < NB; ++q) st.phi[((size_t)q * (S + 1) + s) * Nc + c] = y[q];
                double lap = 0.0;
                if (isv && unk_c) {
                    lap = diag2<DIM>(y) / (rs * rs);
                    diag_sum += lap;
                    if (!is_unknown(role[j], j, bc)) lap = 0.0;
                }
                if (st.amat) {
                    st.amat[(size_t)s * Nc + c] = lap;
                    st.amat32[(size_t)s * Nc + c] = (float)lap;
                    off_sum += lap;
                }
            } else {
#pragma unroll
                for (int q = 0; q < NB; ++q) st.phi[((size_t)q * (S + 1) + S) * Nc + c] = y[q];
            }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) st.phi[((size_t)q * (S + 1) + CEN) * Nc + c] = -cacc[q];
        if (st.amat) {
            // FP32 copy in difference form: its centre slot holds the row sum
            // (zero for rows without known neighbours), so that products
            // sum a_j (x_j - x_c) + rowsum x_c and keep the exact
            // cancellation of the stencil on smooth fields
            const double dg = unk_c ? -diag_sum : 0.0;
            st.amat[(size_t)CEN * Nc + c] = dg;
            st.amat32[(size_t)CEN * Nc + c] = (float)(dg + off_sum);
        }
    }
}

hipError_t launch_mls_build(const MeshDev& m, const double* pos, const int8_t* role, const double* normal,
                            const BcDev& bc, double re, double rs, int wkind, const SetDev& set, int* counters,
                            int* latch, hipStream_t st) {
    long long g = ((long long)m.Nc + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    g = (g + 7) / 8 * 8;
    if (m.dim == 2)
        hipLaunchKernelGGL(k_mls_build<2>, dim3((int)g), dim3(kBlock), 0, st, m, pos, role, normal, bc, re, rs, wkind,
                           set, counters, latch);
    else
        hipLaunchKernelGGL(k_mls_build<3>, dim3((int)g), dim3(kBlock), 0, st, m, pos, role, normal, bc, re, rs, wkind,
                           set, counters, latch);
    return hipGetLastError();
}

}  // namespace mcd
