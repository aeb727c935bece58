// Multigrid preconditioner of the PPE and the right-preconditioned
// Bi-CGSTAB that uses it (MCD_PRECOND_MG).  Not from the paper: the solver
// the paper names (Sec. 3.3, Bi-CGSTAB) with one V-cycle as its right
// preconditioner, so that the iteration count no longer grows with the mesh.
//
// Hierarchy (rebuilt for every solve, the operator changes every step):
// level 0 is the PPE matrix on the background mesh; level l+1 halves every
// axis (rounded up; periodic axes must be even, no axis below 3 cells) and
// stops at 64 cells or fewer.  A coarse cell is unknown when any of its 2^d
// children is.  Prolongation P: a fine cell takes 3/4 of its parent cell and
// 1/4 of the parent's neighbour on its side, per axis, over unknown coarse
// cells inside the mesh, renormalised; restriction R: the mean of the
// children; coarse operators A_(l+1) = R A_l P (Galerkin), which stay within
// the 3^d block and inherit the boundary rows of the fine operator.  V(1,1)
// cycle with damped Jacobi (w = 0.8): x = w D^-1 b; coarse rhs R (b - A x);
// x += P (cycle); x += w D^-1 (b - A x); the coarsest level is solved with
// its dense inverse.  The cycle runs in FP32 (level 0 reads the FP32 copy of
// the matrix, in difference form); the Galerkin products accumulate in FP64.
//
// Outer solver: Bi-CGSTAB in FP64 with the FP64 matrix, right-preconditioned
// (v = A M^-1 p, t = A M^-1 s, x += alpha M^-1 p + omega M^-1 s), inner
// products from per-block partial sums added in a fixed order, scalars on
// the host; stopping on ||r|| <= tol ||b|| confirmed by the true residual.
#include "common.h"

#include <cmath>

namespace mcd {

constexpr int kMgMaxLevels = 16;
constexpr int kMgMaxCoarse = 64;
constexpr float kMgOmega = 0.8f;
constexpr int kMgParts = 1024;          // outer-solver blocks (partial sums)

struct MgLevel {
    MeshDev m{};                 // dims, periodic; m.mps = plane stride of A
    float* A = nullptr;          // [S][mps] Galerkin operator (levels >= 1)
    float* dinv = nullptr;       // [N] 1 / diag at unknown cells, 0 elsewhere
    uint8_t* unk = nullptr;      // [N] unknown flags (level 0: the set's)
    float* x = nullptr;          // [N] work
    float* y = nullptr;          // [N] the level's cycle result
    float* b = nullptr;          // [N] the level's right-hand side
    float* pn = nullptr;         // [N] 1 / row sum of the raw prolongation weights into the next level
};

struct MgWork {
    int L = 0;
    bool usable = false;         // the coarsest level has at most kMgMaxCoarse cells
    MgLevel lev[kMgMaxLevels];
    double* dense = nullptr;     // [Nc][Nc] coarsest matrix (FP64)
    float* inv = nullptr;        // [Nc][Nc] its inverse
    double* part = nullptr;      // [4][kMgParts] partial sums of the outer solver
    double* tot = nullptr;       // [4] totals
    double* host = nullptr;      // [4] pinned copy of the totals
    int* flag = nullptr;         // [1] singular coarsest matrix
};

// ---------------------------------------------------------------------------
// Level geometry
// ---------------------------------------------------------------------------

__device__ __forceinline__ int mg_cell(const MeshDev& m, const int* ijk) {
    return ijk[0] + m.n[0] * (ijk[1] + m.n[1] * ijk[2]);
}

// Coarse coordinate along axis a, wrapped on a periodic axis; false outside.
__device__ __forceinline__ bool mg_coord(const MeshDev& mc, int a, int& v) {
    if (v < 0 || v >= mc.n[a]) {
        if (!mc.periodic[a]) return false;
        v = (v + mc.n[a]) % mc.n[a];
    }
    return true;
}

// Sum of the raw prolongation weights of fine cell j (coordinates jf) over
// its valid coarse cells (inside the mesh or wrapped, unknown): the
// normalisation of P's row j.
template <int DIM>
__device__ __forceinline__ float mg_pweight_sum(const MeshDev& mc, const uint8_t* __restrict__ unk_c, const int jf[3]) {
    float tot = 0.0f;
#pragma unroll
    for (int corner = 0; corner < (1 << DIM); ++corner) {
        int k[3] = {0, 0, 0};
        float wt = 1.0f;
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int far = (corner >> a) & 1;
            const int side = (jf[a] % 2 == 0) ? -1 : 1;
            int v = jf[a] / 2 + side * far;
            ok = ok && mg_coord(mc, a, v);
            k[a] = v;
            wt *= far ? 0.25f : 0.75f;
        }
        if (ok && unk_c[mg_cell(mc, k)]) tot += wt;
    }
    return tot;
}

// Calls f(K, w) for every valid coarse cell K of fine cell j with its raw
// weight w (3/4 or 1/4 per axis; divide by mg_pweight_sum for P).
template <int DIM, typename F>
__device__ __forceinline__ void mg_pvisit(const MeshDev& mc, const uint8_t* __restrict__ unk_c, const int jf[3], F f) {
#pragma unroll
    for (int corner = 0; corner < (1 << DIM); ++corner) {
        int k[3] = {0, 0, 0};
        float wt = 1.0f;
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int far = (corner >> a) & 1;
            const int side = (jf[a] % 2 == 0) ? -1 : 1;
            int v = jf[a] / 2 + side * far;
            ok = ok && mg_coord(mc, a, v);
            k[a] = v;
            wt *= far ? 0.25f : 0.75f;
        }
        if (ok && unk_c[mg_cell(mc, k)]) f(k, wt);
    }
}

// Slot of the coarse offset K - I (periodic axes wrapped into -1..1).
template <int DIM>
__device__ __forceinline__ int mg_slot(const MeshDev& mc, const int* K, const int* I) {
    int s = 0, mul = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int d = K[a] - I[a];
        if (mc.periodic[a]) {
            if (d > 1) d -= mc.n[a];
            if (d < -1) d += mc.n[a];
        }
        s += (d + 1) * mul;
        mul *= 3;
    }
    return s;
}

// Element offset of stencil slot s for a cell away from the mesh edges.
template <int DIM>
__device__ __forceinline__ int mg_off(const MeshDev& m, int s) {
    return (s % 3 - 1) + (DIM > 1 ? ((s / 3) % 3 - 1) * m.n[0] : 0) + (DIM > 2 ? (s / 9 - 1) * m.n[0] * m.n[1] : 0);
}

template <int DIM>
__device__ __forceinline__ bool mg_interior(const MeshDev& m, const int ijk[3]) {
    bool in = ijk[0] > 0 && ijk[0] < m.n[0] - 1 && ijk[1] > 0 && ijk[1] < m.n[1] - 1;
    if (DIM == 3) in = in && ijk[2] > 0 && ijk[2] < m.n[2] - 1;
    return in;
}

// (A x)_c of a level operator: FP32 difference form (level 0: sum a_j (x_j -
// x_c) + rowsum x_c) or plain form (coarse levels).  Cells away from the
// mesh edges use constant slot offsets.
template <int DIM, bool DIFF>
__device__ __forceinline__ float mg_spmv(const MeshDev& m, const float* __restrict__ A, int c,
                                         const float* __restrict__ x) {
    constexpr int S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    int ijk[3];
    cell_ijk(m, c, ijk);
    const float xc = x[c];
    float acc = 0.0f;
    if (mg_interior<DIM>(m, ijk)) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float a = ld_stream(A + (size_t)s * m.mps + c);
            if (s == CEN)
                acc += a * xc;
            else
                acc += DIFF ? a * (x[c + mg_off<DIM>(m, s)] - xc) : a * x[c + mg_off<DIM>(m, s)];
        }
        return acc;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const float a = ld_stream(A + (size_t)s * m.mps + c);
        if (s == CEN) {
            acc += a * xc;
            continue;
        }
        int j;
        double sh[3];
        if (!neighbour<DIM>(m, ijk, s, j, sh)) continue;
        acc += DIFF ? a * (x[j] - xc) : a * x[j];
    }
    return acc;
}

// (A x)_c of the FP64 PPE matrix (plain form, planes at stride m.mps).
template <int DIM, typename F>
__device__ __forceinline__ double mg_spmv64(const MeshDev& m, const double* __restrict__ A, int c, F val) {
    constexpr int S = Dims<DIM>::S;
    int ijk[3];
    cell_ijk(m, c, ijk);
    double acc = 0.0;
    if (mg_interior<DIM>(m, ijk)) {
#pragma unroll
        for (int s = 0; s < S; ++s) acc += ld_stream(A + (size_t)s * m.mps + c) * val(c + mg_off<DIM>(m, s));
        return acc;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const double a = ld_stream(A + (size_t)s * m.mps + c);
        int j;
        double sh[3];
        if (!neighbour<DIM>(m, ijk, s, j, sh)) continue;
        acc += a * val(j);
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Set-up kernels
// ---------------------------------------------------------------------------

// Level 0: 1 / diag of the FP64 matrix at unknown cells.
__global__ void k_mg_diag0(MeshDev m, const double* __restrict__ A, const uint8_t* __restrict__ unk, int cen,
                           float* __restrict__ dinv) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const double d = unk[c] ? A[(size_t)cen * m.mps + c] : 0.0;
        dinv[c] = (d != 0.0 && isfinite(d)) ? (float)(1.0 / d) : 0.0f;
    }
}

template <int DIM>
__global__ void k_mg_flags(MeshDev mf, const uint8_t* __restrict__ unk_f, MeshDev mc, uint8_t* __restrict__ unk_c) {
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < mc.Nc; I += gridDim.x * blockDim.x) {
        int ic[3];
        cell_ijk(mc, I, ic);
        uint8_t any = 0;
#pragma unroll
        for (int ch = 0; ch < (1 << DIM); ++ch) {
            int f[3] = {0, 0, 0};
            bool in = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                f[a] = 2 * ic[a] + ((ch >> a) & 1);
                in = in && f[a] < mf.n[a];
            }
            if (in) any |= unk_f[mg_cell(mf, f)];
        }
        unk_c[I] = any ? 1 : 0;
    }
}

// 1 / (sum of the raw prolongation weights) of every unknown fine cell (0 at
// other cells): P[j][K] = w(j, K) * pn[j].
template <int DIM>
__global__ void k_mg_pnorm(MeshDev mf, const uint8_t* __restrict__ unk_f, MeshDev mc, const uint8_t* __restrict__ unk_c,
                           float* __restrict__ pn) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < mf.Nc; j += gridDim.x * blockDim.x) {
        float v = 0.0f;
        if (unk_f[j]) {
            int fj[3];
            cell_ijk(mf, j, fj);
            const float t = mg_pweight_sum<DIM>(mc, unk_c, fj);
            v = t > 0.0f ? 1.0f / t : 0.0f;
        }
        pn[j] = v;
    }
}

// A_c = R A_f P.  A block takes kMgGalCells coarse cells; each of its
// threads takes one child i of one of them and adds a_s(i) P[j(i, s)][K] to
// its own row of LDS accumulators at the slot of K - I (FP64); the 2^DIM
// children's rows are then summed in child order per slot.
template <int DIM> struct MgGal;
template <> struct MgGal<2> { static constexpr int CELLS = 64; };
template <> struct MgGal<3> { static constexpr int CELLS = 32; };

// Per-axis prolongation weight, away from the mesh edges and unknown-cell
// boundaries: a fine cell at offset o from child c of coarse cell I (q = c +
// o + 1 in 0..3) lies in coarse cell I + floor((c + o) / 2) (weight 3/4) and
// takes 1/4 from that cell's neighbour on its side; e in 0..2 is the coarse
// offset + 1.
__device__ __forceinline__ double mg_w1(int q, int e) {
    const int big = (q + 1) >> 1;
    const int small = big + ((q & 1) ? -1 : 1);
    return e == big ? 0.75 : (e == small ? 0.25 : 0.0);
}

// Interior rows of R A P for one child (parity c[]), whose every coarse
// neighbour is inside the mesh and unknown (so P's rows are the full
// multilinear stencils with unit sum): the 3^d fine row contracts with the
// per-axis weights one axis at a time.
template <int DIM, typename TA>
__device__ __forceinline__ void mg_gal_interior(const MeshDev& mf, const TA* __restrict__ Af, int i, const int* c,
                                                double* row) {
    constexpr int S = Dims<DIM>::S;
    double a[S];
#pragma unroll
    for (int s = 0; s < S; ++s) a[s] = (double)Af[(size_t)s * mf.mps + i];
    if (DIM == 2) {
        double t1[3][3];   // [oy][ex]
#pragma unroll
        for (int oy = 0; oy < 3; ++oy)
#pragma unroll
            for (int ex = 0; ex < 3; ++ex) {
                double v = 0.0;
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) v += a[ox + 3 * oy] * mg_w1(c[0] + ox, ex);
                t1[oy][ex] = v;
            }
#pragma unroll
        for (int ey = 0; ey < 3; ++ey)
#pragma unroll
            for (int ex = 0; ex < 3; ++ex) {
                double v = 0.0;
#pragma unroll
                for (int oy = 0; oy < 3; ++oy) v += t1[oy][ex] * mg_w1(c[1] + oy, ey);
                row[ex + 3 * ey] = v;
            }
    } else {
        double t1[3][3][3];   // [oz][oy][ex]
#pragma unroll
        for (int oz = 0; oz < 3; ++oz)
#pragma unroll
            for (int oy = 0; oy < 3; ++oy)
#pragma unroll
                for (int ex = 0; ex < 3; ++ex) {
                    double v = 0.0;
#pragma unroll
                    for (int ox = 0; ox < 3; ++ox) v += a[ox + 3 * oy + 9 * oz] * mg_w1(c[0] + ox, ex);
                    t1[oz][oy][ex] = v;
                }
        double t2[3][3][3];   // [oz][ey][ex]
#pragma unroll
        for (int oz = 0; oz < 3; ++oz)
#pragma unroll
            for (int ey = 0; ey < 3; ++ey)
#pragma unroll
                for (int ex = 0; ex < 3; ++ex) {
                    double v = 0.0;
#pragma unroll
                    for (int oy = 0; oy < 3; ++oy) v += t1[oz][oy][ex] * mg_w1(c[1] + oy, ey);
                    t2[oz][ey][ex] = v;
                }
#pragma unroll
        for (int ez = 0; ez < 3; ++ez)
#pragma unroll
            for (int ey = 0; ey < 3; ++ey)
#pragma unroll
                for (int ex = 0; ex < 3; ++ex) {
                    double v = 0.0;
#pragma unroll
                    for (int oz = 0; oz < 3; ++oz) v += t2[oz][ey][ex] * mg_w1(c[2] + oz, ez);
                    row[ex + 3 * ey + 9 * ez] = v;
                }
    }
}

// True when every coarse cell of the 3^d block around I is inside the mesh
// (no wrap) and unknown.
template <int DIM>
__device__ __forceinline__ bool mg_full_block(const MeshDev& mc, const uint8_t* __restrict__ unk_c, const int* ic) {
    constexpr int S = Dims<DIM>::S;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        if (ic[a] < 1 || ic[a] > mc.n[a] - 2) return false;
    bool all = true;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k[3] = {ic[0] + s % 3 - 1, ic[1] + (s / 3) % 3 - 1, DIM == 3 ? ic[2] + s / 9 - 1 : 0};
        all = all && unk_c[mg_cell(mc, k)];
    }
    return all;
}

template <int DIM, typename TA>
__global__ __launch_bounds__(kBlock) void k_mg_galerkin(MeshDev mf, const TA* __restrict__ Af,
                                                        const uint8_t* __restrict__ unk_f,
                                                        const float* __restrict__ pn, MeshDev mc,
                                                        const uint8_t* __restrict__ unk_c, float* __restrict__ Ac,
                                                        float* __restrict__ dinv_c) {
    constexpr int S = Dims<DIM>::S, CEN = Dims<DIM>::CEN, CH = 1 << DIM, CELLS = MgGal<DIM>::CELLS;
    static_assert(CELLS * CH == kBlock, "one child per thread");
    __shared__ double acc[CELLS][CH][S];
    const int cl = threadIdx.x / CH, ch = threadIdx.x % CH;
    for (int base = blockIdx.x * CELLS; base < mc.Nc; base += gridDim.x * CELLS) {
        const int I = base + cl;
        double* row = acc[cl][ch];
#pragma unroll
        for (int t = 0; t < S; ++t) row[t] = 0.0;
        if (I < mc.Nc && unk_c[I]) {
            int ic[3];
            cell_ijk(mc, I, ic);
            int fi[3] = {0, 0, 0};
            bool in = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                fi[a] = 2 * ic[a] + ((ch >> a) & 1);
                in = in && fi[a] < mf.n[a];
            }
            const int i = in ? mg_cell(mf, fi) : 0;
            const int par[3] = {ch & 1, (ch >> 1) & 1, (ch >> 2) & 1};
            if (in && unk_f[i] && mg_full_block<DIM>(mc, unk_c, ic)) {
                mg_gal_interior<DIM, TA>(mf, Af, i, par, row);
            } else if (in && unk_f[i]) {
                for (int s = 0; s < S; ++s) {
                    const double a = (double)Af[(size_t)s * mf.mps + i];
                    if (a == 0.0) continue;
                    int j;
                    double sh[3];
                    if (!neighbour<DIM>(mf, fi, s, j, sh)) continue;
                    int fj[3];
                    cell_ijk(mf, j, fj);
                    const double aw = a * (double)pn[j];
                    mg_pvisit<DIM>(mc, unk_c, fj, [&](const int* K, float w) {
                        row[mg_slot<DIM>(mc, K, ic)] += aw * (double)w;
                    });
                }
            }
        }
        __syncthreads();
        if (I < mc.Nc) {
            const double scale = 1.0 / (double)CH;
            for (int t = ch; t < S; t += CH) {
                double v = 0.0;
#pragma unroll
                for (int c = 0; c < CH; ++c) v += acc[cl][c][t];
                v *= scale;
                Ac[(size_t)t * mc.mps + I] = (float)v;
                if (t == CEN) dinv_c[I] = (unk_c[I] && v != 0.0 && isfinite(v)) ? (float)(1.0 / v) : 0.0f;
            }
        }
        __syncthreads();
    }
}

// Dense matrix of the coarsest level (rows and columns of non-unknown cells
// replaced by the identity).
template <int DIM, typename TA>
__global__ void k_mg_dense(MeshDev mc, const TA* __restrict__ Ac, const uint8_t* __restrict__ unk,
                           double* __restrict__ D) {
    constexpr int S = Dims<DIM>::S;
    const int N = mc.Nc;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) D[e] = 0.0;
    __syncthreads();
    for (int I = threadIdx.x; I < N; I += blockDim.x) {
        if (!unk[I]) {
            D[I * N + I] = 1.0;
            continue;
        }
        int ic[3];
        cell_ijk(mc, I, ic);
        for (int s = 0; s < S; ++s) {
            int J;
            double sh[3];
            if (!neighbour<DIM>(mc, ic, s, J, sh)) continue;
            if (!unk[J]) continue;
            D[I * N + J] += (double)Ac[(size_t)s * mc.mps + I];
        }
    }
}

// Gauss-Jordan inversion with partial pivoting of the N x N (N <= 64)
// coarsest matrix, one block, in LDS.  flag = 1 when a pivot vanishes.
__global__ __launch_bounds__(256) void k_mg_invert(const double* __restrict__ D, int N, float* __restrict__ inv,
                                                   int* flag) {
    __shared__ double M[kMgMaxCoarse][2 * kMgMaxCoarse];
    __shared__ double fac[kMgMaxCoarse];
    __shared__ int piv;
    const int W = 2 * N;
    for (int e = threadIdx.x; e < N * W; e += blockDim.x) {
        const int r = e / W, c = e % W;
        M[r][c] = c < N ? D[r * N + c] : (c - N == r ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        if (threadIdx.x == 0) {
            int best = k;
            for (int r = k + 1; r < N; ++r)
                if (fabs(M[r][k]) > fabs(M[best][k])) best = r;
            piv = best;
            if (!(fabs(M[best][k]) > 0.0)) *flag = 1;
        }
        __syncthreads();
        const int p = piv;
        if (p != k)
            for (int c = threadIdx.x; c < W; c += blockDim.x) {
                const double t = M[k][c];
                M[k][c] = M[p][c];
                M[p][c] = t;
            }
        __syncthreads();
        const double d = M[k][k];
        const double id = d != 0.0 ? 1.0 / d : 0.0;
        __syncthreads();
        for (int c = threadIdx.x; c < W; c += blockDim.x) M[k][c] *= id;
        for (int r = threadIdx.x; r < N; r += blockDim.x) fac[r] = r == k ? 0.0 : M[r][k];
        __syncthreads();
        for (int e = threadIdx.x; e < N * W; e += blockDim.x) {
            const int r = e / W, c = e % W;
            if (r != k) M[r][c] -= fac[r] * M[k][c];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) inv[e] = (float)M[e / N][N + e % N];
}

// ---------------------------------------------------------------------------
// Cycle kernels (FP32)
// ---------------------------------------------------------------------------

__global__ void k_mg_scale(int N, const float* __restrict__ dinv, const float* __restrict__ b, float* __restrict__ x) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x)
        x[c] = kMgOmega * dinv[c] * b[c];
}

// r = b - A x at unknown cells (0 elsewhere).
template <int DIM, bool DIFF>
__global__ void k_mg_resid(MeshDev m, const float* __restrict__ A, const uint8_t* __restrict__ unk,
                           const float* __restrict__ x, const float* __restrict__ b, float* __restrict__ r) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x)
        r[c] = unk[c] ? b[c] - mg_spmv<DIM, DIFF>(m, A, c, x) : 0.0f;
}

// Coarse right-hand side: the mean of the children's residuals (R).
template <int DIM>
__global__ void k_mg_average(MeshDev mf, const float* __restrict__ rf, MeshDev mc, float* __restrict__ bc) {
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < mc.Nc; I += gridDim.x * blockDim.x) {
        int ic[3];
        cell_ijk(mc, I, ic);
        float sum = 0.0f;
#pragma unroll
        for (int ch = 0; ch < (1 << DIM); ++ch) {
            int f[3] = {0, 0, 0};
            bool in = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                f[a] = 2 * ic[a] + ((ch >> a) & 1);
                in = in && f[a] < mf.n[a];
            }
            if (in) sum += rf[mg_cell(mf, f)];
        }
        bc[I] = sum * (1.0f / (float)(1 << DIM));
    }
}

template <int DIM>
__global__ void k_mg_prolong(MeshDev mf, const uint8_t* __restrict__ unk_f, const float* __restrict__ pn,
                             float* __restrict__ xf, MeshDev mc, const uint8_t* __restrict__ unk_c,
                             const float* __restrict__ yc) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < mf.Nc; j += gridDim.x * blockDim.x) {
        if (!unk_f[j]) continue;
        int fj[3];
        cell_ijk(mf, j, fj);
        float add = 0.0f;
        mg_pvisit<DIM>(mc, unk_c, fj, [&](const int* K, float w) { add += w * yc[mg_cell(mc, K)]; });
        xf[j] += add * pn[j];
    }
}

template <int DIM, bool DIFF>
__global__ void k_mg_smooth(MeshDev m, const float* __restrict__ A, const uint8_t* __restrict__ unk,
                            const float* __restrict__ dinv, const float* __restrict__ b, const float* __restrict__ x,
                            float* __restrict__ y) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x)
        y[c] = unk[c] ? x[c] + kMgOmega * dinv[c] * (b[c] - mg_spmv<DIM, DIFF>(m, A, c, x)) : 0.0f;
}

__global__ __launch_bounds__(256) void k_mg_coarse_solve(const float* __restrict__ inv, int N,
                                                         const uint8_t* __restrict__ unk,
                                                         const float* __restrict__ b, float* __restrict__ y) {
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
        float acc = 0.0f;
        for (int k = 0; k < N; ++k) acc += inv[r * N + k] * b[k];
        y[r] = unk[r] ? acc : 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Host side: allocation, set-up, cycle
// ---------------------------------------------------------------------------

static int grid_for(int n) {
    const int g = (n + kBlock - 1) / kBlock;
    return g > 4096 ? 4096 : (g < 1 ? 1 : g);
}

hipError_t mg_alloc(const MeshDev& m, MgWork** out) {
    MgWork* w = new MgWork();
    *out = w;
    hipError_t e = hipSuccess;
    auto falloc = [&](float** p, size_t n) {
        if (e == hipSuccess) e = hipMalloc((void**)p, n * sizeof(float));
        if (e == hipSuccess) e = hipMemset(*p, 0, n * sizeof(float));
    };
    MeshDev cur = m;
    const int S = m.dim == 3 ? 27 : 9;
    for (int l = 0; l < kMgMaxLevels && e == hipSuccess; ++l) {
        MgLevel& L = w->lev[l];
        L.m = cur;
        if (l > 0) {
            falloc(&L.A, (size_t)S * cur.mps);
            if (e == hipSuccess) e = hipMalloc((void**)&L.unk, (size_t)cur.Nc);
            if (e == hipSuccess) e = hipMemset(L.unk, 0, (size_t)cur.Nc);
        }
        falloc(&L.dinv, (size_t)cur.Nc);
        falloc(&L.x, (size_t)cur.Nc);
        falloc(&L.y, (size_t)cur.Nc);
        falloc(&L.b, (size_t)cur.Nc);
        falloc(&L.pn, (size_t)cur.Nc);
        w->L = l + 1;
        // the next level, unless this one is the coarsest
        MeshDev nx = cur;
        bool more = cur.Nc > kMgMaxCoarse;
        long long N = 1;
        for (int a = 0; a < m.dim; ++a) {
            if (cur.periodic[a] && (cur.n[a] % 2)) more = false;
            nx.n[a] = (cur.n[a] + 1) / 2;
            if (nx.n[a] < 3) more = false;
            N *= nx.n[a];
            nx.length[a] = cur.length[a];
        }
        if (!more) {
            w->usable = cur.Nc <= kMgMaxCoarse;      // otherwise the mesh cannot be coarsened far enough
            break;
        }
        nx.Nc = (int)N;
        nx.l0 = cur.l0 * 2.0;
        nx.mps = padded_plane_stride((size_t)N);
        cur = nx;
    }
    const int Nc = w->usable ? w->lev[w->L - 1].m.Nc : 1;
    if (e == hipSuccess) e = hipMalloc((void**)&w->dense, (size_t)Nc * Nc * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&w->inv, (size_t)Nc * Nc * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&w->part, 4 * kMgParts * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&w->tot, 4 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&w->flag, sizeof(int));
    if (e == hipSuccess) e = hipHostMalloc((void**)&w->host, 4 * sizeof(double), hipHostMallocDefault);
    return e;
}

bool mg_usable(const MgWork* w) { return w && w->usable; }

void mg_free(MgWork* w) {
    if (!w) return;
    for (int l = 0; l < w->L; ++l) {
        MgLevel& L = w->lev[l];
        // level 0 borrows the set's matrix and flags while a solve runs
        float* f[6] = {l > 0 ? L.A : nullptr, L.dinv, L.x, L.y, L.b, L.pn};
        for (float* p : f)
            if (p) (void)hipFree(p);
        if (l > 0 && L.unk) (void)hipFree(L.unk);
    }
    if (w->dense) (void)hipFree(w->dense);
    if (w->inv) (void)hipFree(w->inv);
    if (w->part) (void)hipFree(w->part);
    if (w->tot) (void)hipFree(w->tot);
    if (w->flag) (void)hipFree(w->flag);
    if (w->host) (void)hipHostFree(w->host);
    delete w;
}

__global__ void k_mg_zero_flag(int* f) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *f = 0;
}

// Hierarchy of the set's PPE matrix.  Level 0 uses the set's FP32 matrix and
// flags; coarse operators come from the FP64 matrix at the first coarsening.
template <int DIM>
static hipError_t mg_setup_dim(MgWork& w, const SetDev& set, hipStream_t st) {
    constexpr int CEN = Dims<DIM>::CEN;
    MgLevel& L0 = w.lev[0];
    L0.A = set.amat32;
    L0.unk = set.unknown;
    hipLaunchKernelGGL(k_mg_diag0, dim3(grid_for(L0.m.Nc)), dim3(kBlock), 0, st, L0.m, set.amat, set.unknown, CEN,
                       L0.dinv);
    for (int l = 0; l + 1 < w.L; ++l) {
        MgLevel& F = w.lev[l];
        MgLevel& C = w.lev[l + 1];
        hipLaunchKernelGGL(k_mg_flags<DIM>, dim3(grid_for(C.m.Nc)), dim3(kBlock), 0, st, F.m, F.unk, C.m, C.unk);
        hipLaunchKernelGGL(k_mg_pnorm<DIM>, dim3(grid_for(F.m.Nc)), dim3(kBlock), 0, st, F.m, F.unk, C.m, C.unk, F.pn);
        const int gb = (C.m.Nc + MgGal<DIM>::CELLS - 1) / MgGal<DIM>::CELLS;
        const dim3 gg(gb > 8192 ? 8192 : gb);
        if (l == 0)
            hipLaunchKernelGGL((k_mg_galerkin<DIM, double>), gg, dim3(kBlock), 0, st, F.m, set.amat, F.unk, F.pn, C.m,
                               C.unk, C.A, C.dinv);
        else
            hipLaunchKernelGGL((k_mg_galerkin<DIM, float>), gg, dim3(kBlock), 0, st, F.m, F.A, F.unk, F.pn, C.m, C.unk,
                               C.A, C.dinv);
    }
    const MgLevel& Lc = w.lev[w.L - 1];
    hipLaunchKernelGGL(k_mg_zero_flag, dim3(1), dim3(64), 0, st, w.flag);
    if (w.L == 1)      // the mesh is its own coarsest level: the FP64 matrix (plain form)
        hipLaunchKernelGGL((k_mg_dense<DIM, double>), dim3(1), dim3(256), 0, st, Lc.m, set.amat, Lc.unk, w.dense);
    else
        hipLaunchKernelGGL((k_mg_dense<DIM, float>), dim3(1), dim3(256), 0, st, Lc.m, Lc.A, Lc.unk, w.dense);
    hipLaunchKernelGGL(k_mg_invert, dim3(1), dim3(256), 0, st, w.dense, Lc.m.Nc, w.inv, w.flag);
    return hipGetLastError();
}

hipError_t mg_setup(const MeshDev& m, MgWork& w, const SetDev& set, hipStream_t st) {
    if (!w.usable) return hipErrorNotSupported;
    return m.dim == 2 ? mg_setup_dim<2>(w, set, st) : mg_setup_dim<3>(w, set, st);
}

// One V-cycle on level 0: rhs lev[0].b, result lev[0].y.
template <int DIM>
static void mg_cycle_dim(MgWork& w, hipStream_t st) {
    for (int l = 0; l + 1 < w.L; ++l) {
        MgLevel& F = w.lev[l];
        MgLevel& C = w.lev[l + 1];
        hipLaunchKernelGGL(k_mg_scale, dim3(grid_for(F.m.Nc)), dim3(kBlock), 0, st, F.m.Nc, F.dinv, F.b, F.x);
        // the level's residual goes to y (its cycle result is written only later)
        if (l == 0)
            hipLaunchKernelGGL((k_mg_resid<DIM, true>), dim3(grid_for(F.m.Nc)), dim3(kBlock), 0, st, F.m, F.A, F.unk,
                               F.x, F.b, F.y);
        else
            hipLaunchKernelGGL((k_mg_resid<DIM, false>), dim3(grid_for(F.m.Nc)), dim3(kBlock), 0, st, F.m, F.A, F.unk,
                               F.x, F.b, F.y);
        hipLaunchKernelGGL(k_mg_average<DIM>, dim3(grid_for(C.m.Nc)), dim3(kBlock), 0, st, F.m, F.y, C.m, C.b);
    }
    const MgLevel& Lc = w.lev[w.L - 1];
    hipLaunchKernelGGL(k_mg_coarse_solve, dim3(1), dim3(256), 0, st, w.inv, Lc.m.Nc, Lc.unk, Lc.b, Lc.y);
    for (int l = w.L - 2; l >= 0; --l) {
        MgLevel& F = w.lev[l];
        MgLevel& C = w.lev[l + 1];
        hipLaunchKernelGGL(k_mg_prolong<DIM>, dim3(grid_for(F.m.Nc)), dim3(kBlock), 0, st, F.m, F.unk, F.pn, F.x,
                           C.m, C.unk, C.y);
        if (l == 0)
            hipLaunchKernelGGL((k_mg_smooth<DIM, true>), dim3(grid_for(F.m.Nc)), dim3(kBlock), 0, st, F.m, F.A, F.unk,
                               F.dinv, F.b, F.x, F.y);
        else
            hipLaunchKernelGGL((k_mg_smooth<DIM, false>), dim3(grid_for(F.m.Nc)), dim3(kBlock), 0, st, F.m, F.A,
                               F.unk, F.dinv, F.b, F.x, F.y);
    }
}

static void mg_cycle(const MeshDev& m, MgWork& w, hipStream_t st) {
    if (m.dim == 2)
        mg_cycle_dim<2>(w, st);
    else
        mg_cycle_dim<3>(w, st);
}

// ---------------------------------------------------------------------------
// Outer Bi-CGSTAB (FP64)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void mg_parts(double (&q)[4], int nq, double* part) {
    __shared__ double lds[4][kBlock / 64];
    block_sum<4>(q, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < nq; ++k) part[k * kMgParts + blockIdx.x] = q[k];
}

// r = b - A x, rhat = r (restart = 0 keeps rhat); partials r.r, b.b, rhat.r
template <int DIM>
__global__ void k_mgo_resid(MeshDev m, const double* __restrict__ A, const uint8_t* __restrict__ unk,
                            const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ r,
                            double* __restrict__ rhat, int set_rhat, double* part) {
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (unk[c]) v = b[c] - mg_spmv64<DIM>(m, A, c, [&](int j) { return x[j]; });
        r[c] = v;
        if (set_rhat) rhat[c] = v;
        q[0] += v * v;
        q[1] += b[c] * b[c];
        q[2] += (set_rhat ? v : rhat[c]) * v;
    }
    mg_parts(q, 3, part);
}

// p = r + beta (p - omega v); the cycle's FP32 right-hand side b0 = p
__global__ void k_mgo_p(int N, const uint8_t* __restrict__ unk, const double* __restrict__ r, double* __restrict__ p,
                        const double* __restrict__ v, double beta, double omega, float* __restrict__ b0) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        const double pv = unk[c] ? r[c] + beta * (p[c] - omega * v[c]) : 0.0;
        p[c] = pv;
        b0[c] = (float)pv;
    }
}

// z = (double) y0 (the preconditioned direction), w = A z; partials rhat.w
// (or t.s, t.t with s given)
template <int DIM>
__global__ void k_mgo_apply(MeshDev m, const double* __restrict__ A, const uint8_t* __restrict__ unk,
                            const float* __restrict__ y0, double* __restrict__ z, double* __restrict__ wv,
                            const double* __restrict__ rhat, const double* __restrict__ s, double* part) {
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (unk[c]) v = mg_spmv64<DIM>(m, A, c, [&](int j) { return (double)y0[j]; });
        z[c] = (double)y0[c];
        wv[c] = v;
        if (s) {
            q[0] += v * s[c];
            q[1] += v * v;
        } else {
            q[0] += rhat[c] * v;
        }
    }
    mg_parts(q, s ? 2 : 1, part);
}

// s = r - alpha v; b0 = s
__global__ void k_mgo_s(int N, const double* __restrict__ r, const double* __restrict__ v, double alpha,
                        double* __restrict__ s, float* __restrict__ b0) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        const double sv = r[c] - alpha * v[c];
        s[c] = sv;
        b0[c] = (float)sv;
    }
}

// x += alpha ph + omega sh; r = s - omega t; partials r.r, rhat.r
__global__ void k_mgo_xr(int N, double* __restrict__ x, const double* __restrict__ ph, const double* __restrict__ sh,
                         const double* __restrict__ s, const double* __restrict__ t, double alpha, double omega,
                         double* __restrict__ r, const double* __restrict__ rhat, double* part) {
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        x[c] = x[c] + alpha * ph[c] + omega * sh[c];
        const double rv = s[c] - omega * t[c];
        r[c] = rv;
        q[0] += rv * rv;
        q[1] += rhat[c] * rv;
    }
    mg_parts(q, 2, part);
}

// totals of nq partial rows over nblk blocks, in block order
__global__ void k_mgo_reduce(const double* __restrict__ part, int nblk, int nq, double* __restrict__ tot) {
    __shared__ double lds[4][kBlock / 64];
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nq; ++k)
        for (int b = threadIdx.x; b < nblk; b += blockDim.x) q[k] += part[k * kMgParts + b];
    block_sum<4>(q, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) tot[k] = q[k];
}

static hipError_t totals(MgWork& w, int nblk, int nq, hipStream_t st, double* out) {
    hipLaunchKernelGGL(k_mgo_reduce, dim3(1), dim3(kBlock), 0, st, w.part, nblk, nq, w.tot);
    hipError_t e = hipMemcpyAsync(w.host, w.tot, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess)
        for (int k = 0; k < 4; ++k) out[k] = w.host[k];
    return e;
}

// Right-preconditioned Bi-CGSTAB on the set's FP64 matrix from x (FP64
// vectors of the workspace); b: effective right-hand side.
template <int DIM>
static hipError_t mg_bicgstab_dim(const MeshDev& m, MgWork& w, const SetDev& set, const MgVecs& V, double tol,
                                  int max_iter, hipStream_t st, MgResult* out) {
    const int N = m.Nc;
    const int g = (N + kBlock - 1) / kBlock > kMgParts ? kMgParts : (N + kBlock - 1) / kBlock;
    const double* A = set.amat;
    const uint8_t* unk = set.unknown;
    float* b0 = w.lev[0].b;
    const float* y0 = w.lev[0].y;
    double t4[4];
    if (!w.usable) return hipErrorNotSupported;
    hipError_t e = mg_setup_dim<DIM>(w, set, st);
    if (e != hipSuccess) return e;
    int flag = 0;
    if ((e = hipMemcpyAsync(&flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mgo_resid<DIM>, dim3(g), dim3(kBlock), 0, st, m, A, unk, V.b, V.x, V.r, V.rhat, 1, w.part);
    if ((e = totals(w, g, 3, st, t4)) != hipSuccess) return e;
    *out = MgResult{};
    out->coarse_singular = flag;
    const double bb = t4[1];
    out->bnorm = sqrt(bb);
    if (bb == 0.0) {
        out->converged = 1;
        return hipSuccess;
    }
    const double tol2 = tol * tol * bb;
    double rr = t4[0];
    int iters = 0, restarts = 0;
    while (rr > tol2 && iters < max_iter) {
        // (re)start: rhat = r (set by the residual kernel), rho = alpha = omega = 1, p = v = 0
        double rho = 1.0, alpha = 1.0, omega = 1.0, rho_new = t4[2];
        hipLaunchKernelGGL(k_mgo_p, dim3(g), dim3(kBlock), 0, st, N, unk, V.r, V.p, V.v, 0.0, 0.0, b0);
        bool first = true, restart = false;
        while (iters < max_iter) {
            if (!first) {
                if (!(fabs(rho_new) > 1e-300)) {
                    restart = true;
                    break;
                }
                const double beta = (rho_new / rho) * (alpha / omega);
                hipLaunchKernelGGL(k_mgo_p, dim3(g), dim3(kBlock), 0, st, N, unk, V.r, V.p, V.v, beta, omega, b0);
            }
            first = false;
            mg_cycle(m, w, st);
            hipLaunchKernelGGL(k_mgo_apply<DIM>, dim3(g), dim3(kBlock), 0, st, m, A, unk, y0, V.ph, V.v, V.rhat,
                               (const double*)nullptr, w.part);
            if ((e = totals(w, g, 1, st, t4)) != hipSuccess) return e;
            const double rv = t4[0];
            if (!(fabs(rv) > 0.0) || !std::isfinite(rv)) {
                restart = true;
                break;
            }
            alpha = rho_new / rv;
            hipLaunchKernelGGL(k_mgo_s, dim3(g), dim3(kBlock), 0, st, N, V.r, V.v, alpha, V.s, b0);
            mg_cycle(m, w, st);
            hipLaunchKernelGGL(k_mgo_apply<DIM>, dim3(g), dim3(kBlock), 0, st, m, A, unk, y0, V.sh, V.t, V.rhat,
                               V.s, w.part);
            if ((e = totals(w, g, 2, st, t4)) != hipSuccess) return e;
            omega = t4[1] > 0.0 ? t4[0] / t4[1] : 0.0;
            hipLaunchKernelGGL(k_mgo_xr, dim3(g), dim3(kBlock), 0, st, N, V.x, V.ph, V.sh, V.s, V.t, alpha, omega,
                               V.r, V.rhat, w.part);
            if ((e = totals(w, g, 2, st, t4)) != hipSuccess) return e;
            rho = rho_new;
            rr = t4[0];
            rho_new = t4[1];
            ++iters;
            if (rr <= tol2) break;
            if (omega == 0.0 || !std::isfinite(rr)) {
                restart = true;
                break;
            }
        }
        // confirm with the true residual (and restart from it if needed)
        hipLaunchKernelGGL(k_mgo_resid<DIM>, dim3(g), dim3(kBlock), 0, st, m, A, unk, V.b, V.x, V.r, V.rhat, 1,
                           w.part);
        if ((e = totals(w, g, 3, st, t4)) != hipSuccess) return e;
        rr = t4[0];
        if (restart || rr > tol2) ++restarts;
        if (restart && restarts > 50) break;
    }
    out->iterations = iters;
    out->restarts = restarts;
    out->rel = sqrt(rr / bb);
    out->converged = rr <= tol2 ? 1 : 0;
    return hipSuccess;
}

hipError_t mg_bicgstab(const MeshDev& m, MgWork& w, const SetDev& set, const MgVecs& V, double tol, int max_iter,
                       hipStream_t st, MgResult* out) {
    return m.dim == 2 ? mg_bicgstab_dim<2>(m, w, set, V, tol, max_iter, st, out)
                      : mg_bicgstab_dim<3>(m, w, set, V, tol, max_iter, st, out);
}

// One V-cycle of the set's preconditioner on in (FP64 [Nc], read at unknown
// cells) into out (FP64 [Nc], zero at other cells).
__global__ void k_mg_in(int N, const uint8_t* __restrict__ unk, const double* __restrict__ in, float* __restrict__ b0) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x)
        b0[c] = unk[c] ? (float)in[c] : 0.0f;
}
__global__ void k_mg_out(int N, const float* __restrict__ y0, double* __restrict__ out) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) out[c] = (double)y0[c];
}

hipError_t mg_apply(const MeshDev& m, MgWork& w, const SetDev& set, const double* in, double* out, int* levels,
                    hipStream_t st) {
    hipError_t e = mg_setup(m, w, set, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mg_in, dim3(grid_for(m.Nc)), dim3(kBlock), 0, st, m.Nc, set.unknown, in, w.lev[0].b);
    mg_cycle(m, w, st);
    hipLaunchKernelGGL(k_mg_out, dim3(grid_for(m.Nc)), dim3(kBlock), 0, st, m.Nc, w.lev[0].y, out);
    *levels = w.L;
    return hipGetLastError();
}

}  // namespace mcd
