// MLS stencil build (Sec. 3.2, chi_c = 1): one thread per DP, FP64.
//
// For DP c the fit minimises J of Eq. (obj_func) with phi_c fixed:
//   M Phi = sum_value w_j p_j (phi_j - phi_c) + sum_Neumann w_j pN_j r_s f_j,
//   M     = sum_value w_j p_j p_j^T + sum_Neumann w_j pN_j pN_j^T.
// Pass 1 gathers the 3x3(x3) block and accumulates M (packed lower
// triangle, registers); M is Cholesky-factored in registers; pass 2
// re-gathers each row and writes W_j = M^-1 (w_j a_j) into the slot planes
// (coalesced: consecutive threads write consecutive cells of a plane; the
// planes are written once and read by later kernels only, so the stores are
// non-temporal), plus the PPE Laplacian matrix of the unknown rows in FP64
// and FP32.  Its FP32 copy holds only the unknown columns; the FP64 slots
// of an unknown row also keep the weights of its known value neighbours
// (the operands of every product with it are zero there), so that the
// centre is minus the sum of the row's other slots in slot order, the sum
// the build forms, and need not be read.
//
// Rounding: built without contraction (no FMA), with the series weight
// functions and one reciprocal per Cholesky pivot, and every sum taken in
// slot and basis order, the weights have the same bits as a plain
// evaluation of the same formulas in that order (IEEE + - * / sqrt).
#include "common.h"

#include <cmath>
#include <type_traits>

namespace mcd {

// cos^2(pi r / (2 r_e)) (Sec. 3.2) or the truncated Gaussian, with the
// series cosine / exponential of common.h.
template <int WK>
__device__ __forceinline__ double mls_weight(double r, double re) {
    if (r > re) return 0.0;
    if (WK == MCD_WEIGHT_COS2) {
        const double t = series_cos(M_PI * r / (2.0 * re));
        return t * t;
    }
    return series_exp_neg(4.0 * r * r / (re * re));
}

// Tiles of the build: 64 x 4 cells (2D) or 32 x 4 x 2 (3D), one cell per
// thread of a 256-thread block; the tile plus a one-cell halo is staged in
// LDS (positions already shifted to the periodic image seen from the tile,
// normals, roles, cell indices), so the 2 x 27 neighbour reads per DP of the
// two passes are LDS reads.
template <int DIM> struct MlsTile;
template <> struct MlsTile<2> { static constexpr int X = 64, Y = 4, Z = 1; };
template <> struct MlsTile<3> { static constexpr int X = 32, Y = 4, Z = 2; };

template <int DIM>
struct MlsHalo {
    static constexpr int X = MlsTile<DIM>::X + 2, Y = MlsTile<DIM>::Y + 2, Z = DIM == 3 ? MlsTile<DIM>::Z + 2 : 1;
    static constexpr int N = X * Y * Z;
    // 3D reads the normals of its (rare) Neumann rows from global memory, so
    // that the LDS left over holds every row's weight between the passes
    static constexpr bool NV = DIM == 2;
    double p[DIM][N];      // neighbour position (periodic image)
    double nv[NV ? DIM : 1][NV ? N : 1];   // neighbour normal (2D)
    int j[N];              // cell index, -1 outside a non-periodic mesh
    int8_t r[N];           // role
    int8_t kd[N];          // row kind (0 none, 1 value row, 2 Neumann row)
};

// halo slot of the neighbour at stencil slot s of tile cell (lx, ly, lz)
template <int DIM>
__device__ __forceinline__ int halo_slot(int lx, int ly, int lz, int s) {
    using H = MlsHalo<DIM>;
    const int ox = s % 3 - 1, oy = (s / 3) % 3 - 1, oz = DIM == 3 ? s / 9 - 1 : 0;
    const int hz = DIM == 3 ? lz + 1 + oz : 0;
    return (hz * H::Y + (ly + 1 + oy)) * H::X + (lx + 1 + ox);
}

// Row of neighbour slot e: kind (0 none, 1 value, 2 Neumann), its basis
// vector a (value or normal-derivative row, Eq. obj_func) and, when
// want_w, its weight.
template <int DIM, bool POW2, int WK>
__device__ __forceinline__ int row_lds(const MlsHalo<DIM>& H, int e, bool centre,
                                       const double* xc, double re, double rs, double rs_inv, bool want_w,
                                       const double* __restrict__ normal, size_t Nc, double& w, double* a) {
    if (H.j[e] < 0) return 0;
    const int kind = H.kd[e];
    if (centre && kind != 2) return 0;     // the DP itself: only its Neumann row
    if (kind == 0) return 0;
    double d[DIM], X[DIM];
    double r2 = 0.0;
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        d[q] = H.p[q][e] - xc[q];
        r2 += d[q] * d[q];
        X[q] = POW2 ? d[q] * rs_inv : d[q] / rs;
    }
    if (want_w) w = mls_weight<WK>(sqrt(r2), re);
    if (kind == 1) {
        basis<DIM>(X, a);
    } else {
        double nv[DIM];
#pragma unroll
        for (int q = 0; q < DIM; ++q) nv[q] = MlsHalo<DIM>::NV ? H.nv[q][e] : normal[q * Nc + H.j[e]];
        basis_normal<DIM>(X, nv, a);
    }
    return kind;
}

// Unknown of a PPE (inner, or a boundary DP whose row is a Neumann row, minus
// the pinned DP), from the staged role r and row kind.
__device__ __forceinline__ bool mls_unknown(int r, int kind, int j, bool pin) {
    if (pin && j == 0) return false;
    return r == MCD_ROLE_INNER || (r > 0 && kind == 2);
}

template <int DIM>
__device__ __forceinline__ void mls_tile_origin(const MeshDev& m, int tile, int o[3]) {
    using T = MlsTile<DIM>;
    const int ntx = (m.n[0] + T::X - 1) / T::X, nty = (m.n[1] + T::Y - 1) / T::Y;
    o[0] = (tile % ntx) * T::X;
    o[1] = ((tile / ntx) % nty) * T::Y;
    o[2] = (tile / (ntx * nty)) * T::Z;
}

// Stages the tile at origin o and its halo into H: positions shifted to the
// periodic image seen from the tile, roles, row kinds, cell indices, 2D
// normals.  No barrier.
template <int DIM>
__device__ __forceinline__ void mls_stage(const MeshDev& m, MlsHalo<DIM>& H, const int o[3],
                                          const double* __restrict__ pos, const int8_t* __restrict__ role,
                                          const double* __restrict__ normal, const BcDev& bc) {
    using HT = MlsHalo<DIM>;
    const size_t Nc = (size_t)m.Nc;
    for (int e = threadIdx.x; e < HT::N; e += kBlock) {
        const int h[3] = {e % HT::X, (e / HT::X) % HT::Y, e / (HT::X * HT::Y)};
        int idx = 0, stride = 1;
        bool in = true;
        double sh[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            int ii = o[a] - 1 + h[a];
            // beyond every active cell's neighbourhood (a tile wider than
            // the mesh): not a neighbour of anything, left outside
            if (ii < -1 || ii > m.n[a]) in = false;
            if (ii < 0) {
                in = in && m.periodic[a];
                ii += m.n[a];
                sh[a] = -m.length[a];
            } else if (ii >= m.n[a]) {
                in = in && m.periodic[a];
                ii -= m.n[a];
                sh[a] = m.length[a];
            }
            idx += ii * stride;
            stride *= m.n[a];
        }
        const int8_t rr = in ? role[idx] : (int8_t)0;
        H.j[e] = in ? idx : -1;
        H.r[e] = rr;
        H.kd[e] = (int8_t)(in ? row_kind(rr, bc) : 0);
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
            H.p[q][e] = in ? pos[q * Nc + idx] + sh[q] : 0.0;
            if (HT::NV) H.nv[q][e] = in ? normal[q * Nc + idx] : 0.0;
        }
    }
}

// The fit of the DP at tile cell (lx, ly, lz), cell c, written to the set st.
// wc: this thread's weight cache between the passes (each row's weight, the
// same bits as recomputing it).
template <int DIM, bool POW2, int WK>
__device__ __forceinline__ void mls_fit(const MeshDev& m, const MlsHalo<DIM>& H, double* wc, int lx, int ly, int lz,
                                        int c, bool pin, const SetDev& st, const double* __restrict__ normal,
                                        double re, double rs, int* counters, int* latch) {
    constexpr int NB = Dims<DIM>::NB, S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    constexpr int NP = NB * (NB + 1) / 2;
    const size_t Nc = (size_t)m.Nc;
    const double rs_inv = 1.0 / rs, rr_inv = 1.0 / (rs * rs);     // exact when POW2
    const int ecen = halo_slot<DIM>(lx, ly, lz, CEN);
    const int rc = H.r[ecen];
    double xc[DIM];
#pragma unroll
    for (int q = 0; q < DIM; ++q) xc[q] = H.p[q][ecen];
    const bool unk_c = mls_unknown(rc, H.kd[ecen], c, pin);
    st.unknown[c] = unk_c ? 1 : 0;
    double M[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) M[q] = 0.0;
    uint32_t vm = 0, nm = 0;
    int nrows = 0;
    if (rc != MCD_ROLE_VOID) {
        for (int s = 0; s < S; ++s) {
            double w = 0.0, a[NB];
            const int kind = row_lds<DIM, POW2, WK>(H, halo_slot<DIM>(lx, ly, lz, s), s == CEN, xc, re, rs, rs_inv,
                                                    true, normal, Nc, w, a);
            wc[s * kBlock] = w;
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
        wave_count_add(&counters[0], sing && rc == MCD_ROLE_INNER);
        wave_count_add(&counters[1], sing && rc != MCD_ROLE_INNER);
        if (sing && rc == MCD_ROLE_INNER) {
            atomicMin(&counters[2], c);
            atomicAdd(latch, 1);
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
    uint32_t km = 0;
    for (int s = 0; s < S; ++s) {
        const int slot = (s == CEN) ? S : s;
        const bool isv = (vm >> s) & 1u, isn = (nm >> slot) & 1u;
        const int e = halo_slot<DIM>(lx, ly, lz, s);
        double y[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) y[q] = 0.0;
        if (isv || isn) {
            double w = wc[s * kBlock], a[NB];
            row_lds<DIM, POW2, WK>(H, e, s == CEN, xc, re, rs, rs_inv, false, normal, Nc, w, a);
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
            for (int q = 0; q < NB; ++q) __builtin_nontemporal_store(y[q], st.phi + ((size_t)q * (S + 1) + s) * m.mps + c);
            // lap: the matrix entry (0 in the columns of known value
            // neighbours); lapk: the FP64 slot, which keeps those weights
            // too, so that the centre is minus the sum of the row's slots
            double lap = 0.0, lapk = 0.0;
            if (isv && unk_c) {
                lap = POW2 ? diag2<DIM>(y) * rr_inv : diag2<DIM>(y) / (rs * rs);
                diag_sum += lap;
                lapk = lap;
                if (!mls_unknown(H.r[e], H.kd[e], H.j[e], pin)) {
                    lap = 0.0;
                    km |= 1u << s;
                }
            }
            if (st.amat) {
                __builtin_nontemporal_store(lapk, st.amat + (size_t)s * m.mps + c);
                __builtin_nontemporal_store((float)lap, st.amat32 + (size_t)s * m.mps + c);
                off_sum += lap;
            }
        } else {
#pragma unroll
            for (int q = 0; q < NB; ++q) __builtin_nontemporal_store(y[q], st.phi + ((size_t)q * (S + 1) + S) * m.mps + c);
        }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) __builtin_nontemporal_store(-cacc[q], st.phi + ((size_t)q * (S + 1) + CEN) * m.mps + c);
    st.kmask[c] = km;
    if (st.amat) {
        // FP32 copy in difference form: its centre slot holds the row sum (zero
        // for rows without known neighbours), so that products sum
        // a_j (x_j - x_c) + rowsum x_c and keep the exact cancellation of the
        // stencil on smooth fields
        const double dg = unk_c ? -diag_sum : 0.0;
        __builtin_nontemporal_store(dg, st.amat + (size_t)CEN * m.mps + c);
        __builtin_nontemporal_store((float)(dg + off_sum), st.amat32 + (size_t)CEN * m.mps + c);
    }
}

// POW2: r_s is a power of two, so x / r_s and x * (1 / r_s) are the same
// real number and round to the same double; the kernel then multiplies (the
// divisions by r_s and r_s^2 are most of its division work).  WK: the weight
// function (one instantiation each, so that only its series constants
// occupy scalar registers).  Two blocks per CU (the register budget of two
// waves per SIMD).
template <int DIM, bool POW2, int WK>
__global__ __launch_bounds__(kBlock, 2) void k_mls_build(MeshDev m, const double* __restrict__ pos,
                                                      const int8_t* __restrict__ role,
                                                      const double* __restrict__ normal, BcDev bc, double re,
                                                      double rs, SetDev st, int* counters, int* latch) {
    using T = MlsTile<DIM>;
    static_assert(T::X * T::Y * T::Z == kBlock, "one tile cell per thread");
    __shared__ MlsHalo<DIM> H;
    // each row's weight stays in LDS between the passes (in 3D the halo holds
    // no normals, so that two blocks still fit on a CU)
    __shared__ double wc[Dims<DIM>::S][kBlock];
    const int ntiles = ((m.n[0] + T::X - 1) / T::X) * ((m.n[1] + T::Y - 1) / T::Y) *
                       (DIM == 3 ? (m.n[2] + T::Z - 1) / T::Z : 1);
    const int lx = threadIdx.x % T::X, ly = (threadIdx.x / T::X) % T::Y, lz = threadIdx.x / (T::X * T::Y);
    const int nblk = gridDim.x;
    const int lb = xcd_block(blockIdx.x, nblk);
    for (int tile = lb; tile < ntiles; tile += nblk) {
        int o[3];
        mls_tile_origin<DIM>(m, tile, o);
        mls_stage<DIM>(m, H, o, pos, role, normal, bc);
        __syncthreads();
        const int gx = o[0] + lx, gy = o[1] + ly, gz = DIM == 3 ? o[2] + lz : 0;
        if (gx < m.n[0] && gy < m.n[1] && (DIM == 2 || gz < m.n[2]))
            mls_fit<DIM, POW2, WK>(m, H, &wc[0][threadIdx.x], lx, ly, lz, gx + m.n[0] * (gy + m.n[1] * gz),
                                   bc.pin_first, st, normal, re, rs, counters, latch);
        __syncthreads();
    }
}

hipError_t launch_mls_build(const MeshDev& m, const double* pos, const int8_t* role, const double* normal,
                            const BcDev& bc, double re, double rs, int wkind, const SetDev& set, int* counters,
                            int* latch, hipStream_t st) {
    // one tile per block and round, at most 4096 blocks looping over the tiles
    long long g = m.dim == 2 ? (long long)((m.n[0] + 63) / 64) * ((m.n[1] + 3) / 4)
                             : (long long)((m.n[0] + 31) / 32) * ((m.n[1] + 3) / 4) * ((m.n[2] + 1) / 2);
    if (g > 4096) g = 4096;
    // r_s and r_s^2 powers of two, within the normal range
    int e1 = 0, e2 = 0;
    const bool pow2 = std::isnormal(rs) && std::isnormal(rs * rs) && std::frexp(rs, &e1) == 0.5 &&
                      std::frexp(rs * rs, &e2) == 0.5 && std::isnormal(1.0 / (rs * rs));
    const dim3 gd((int)g), bd(kBlock);
    auto go = [&](auto dim_c, auto pow2_c, auto wk_c) {
        constexpr int D = decltype(dim_c)::value;
        constexpr bool P2 = decltype(pow2_c)::value;
        constexpr int WK = decltype(wk_c)::value;
        hipLaunchKernelGGL((k_mls_build<D, P2, WK>), gd, bd, 0, st, m, pos, role, normal, bc, re, rs, set, counters,
                           latch);
    };
    using C2 = std::integral_constant<int, 2>;
    using C3 = std::integral_constant<int, 3>;
    using T = std::true_type;
    using F = std::false_type;
    using WC = std::integral_constant<int, MCD_WEIGHT_COS2>;
    using WG = std::integral_constant<int, MCD_WEIGHT_GAUSS>;
    const bool cos2 = wkind == MCD_WEIGHT_COS2;
    if (m.dim == 2) {
        if (pow2)
            cos2 ? go(C2{}, T{}, WC{}) : go(C2{}, T{}, WG{});
        else
            cos2 ? go(C2{}, F{}, WC{}) : go(C2{}, F{}, WG{});
    } else {
        if (pow2)
            cos2 ? go(C3{}, T{}, WC{}) : go(C3{}, T{}, WG{});
        else
            cos2 ? go(C3{}, F{}, WC{}) : go(C3{}, F{}, WG{});
    }
    return hipGetLastError();
}

}  // namespace mcd
