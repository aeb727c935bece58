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
// Launches per cycle: one per level on the way down (pre-smoothing from zero,
// residual and restriction fused), two per level on the way up
// (prolongation, smoothing), and one workgroup for the levels of at most
// kMgTailCells cells, where separate launches would cost more than the work.
//
// Outer solver: Bi-CGSTAB with FP64 vectors, right-preconditioned (v = A
// M^-1 p, t = A M^-1 s, x += alpha M^-1 p + omega M^-1 s), its products with
// the FP64 matrix or (mixed precision) with the FP32 copy in difference form;
// inner products from per-block partial sums added in a fixed order; stopping
// on ||r|| <= tol ||b|| confirmed by the true residual with the FP64 matrix,
// from which a run that has not met the tolerance restarts (refinement).
#include "common.h"

#include <cmath>

namespace mcd {

constexpr int kMgMaxLevels = 16;
constexpr int kMgMaxCoarse = 64;
constexpr float kMgOmega = 0.8f;
constexpr int kMgParts = 1024;          // outer-solver blocks (partial sums)
constexpr int kMgTailCells = 512;       // levels this small run inside one workgroup
constexpr int kMgMaxTail = 8;           // at most this many levels in that workgroup
constexpr int kMgTailBlock = 1024;

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
    int tail = 0;                // first level of the one-workgroup tail of the cycle
    bool nt = true;              // level-0 and outer matrices streamed (they exceed the last-level cache)
    bool usable = false;         // the coarsest level has at most kMgMaxCoarse cells
    MgLevel lev[kMgMaxLevels];
    double* dense = nullptr;     // [Nc][Nc] coarsest matrix (FP64)
    float* inv = nullptr;        // [Nc][Nc] its inverse
    double* part = nullptr;      // [4][kMgParts] partial sums of the outer solver
    double* host = nullptr;      // [8] totals, pinned host memory written by the reducing kernel
    double* host_dev = nullptr;  // the same memory as the device sees it
    hipEvent_t ev = nullptr;     // completion of the reducing kernel
    struct MgScal* scal = nullptr;  // scalars of the outer iteration (device)
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

// One level as the cycle kernels see it.
struct MgLv {
    int n[3];
    int per[3];
    int Nc;
    int diff;                    // level 0: FP32 copy of the PPE matrix in difference form
    size_t mps;                  // plane stride of A
    const float* A;
    const uint8_t* unk;
    const float* dinv;
    const float* pn;
    float* x;
    float* y;
    float* b;
};

__device__ __forceinline__ void mg_ijk(const int* n, int c, int ijk[3]) {
    ijk[0] = c % n[0];
    const int r = c / n[0];
    ijk[1] = r % n[1];
    ijk[2] = r / n[1];
}

__device__ __forceinline__ int mg_at(const int* n, const int* ijk) { return ijk[0] + n[0] * (ijk[1] + n[1] * ijk[2]); }

// Cell j at stencil slot s of cell ijk (periodic axes wrapped), without
// branches: j is always a valid index (self when the slot lies outside a
// non-periodic mesh) and the return value says whether the slot is a
// neighbour, so that every load of a row can be issued at once.
template <int DIM>
__device__ __forceinline__ bool mg_nbs(const int* n, const int* per, const int* ijk, int s, int self, int& j) {
    int idx = 0, stride = 1;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int v = ijk[a] + (a == 0 ? s % 3 : (a == 1 ? (s / 3) % 3 : s / 9)) - 1;
        const bool lo = v < 0, hi = v >= n[a];
        v = lo ? v + n[a] : (hi ? v - n[a] : v);
        ok = ok && (!(lo || hi) || per[a] != 0);
        idx += v * stride;
        stride *= n[a];
    }
    j = ok ? idx : self;
    return ok;
}

// (A v)_c of a level operator, v given by val(j) and vc = v_c: the plain form
// sum_s a_s v_j, or on level 0 the difference form sum_(s != centre) a_s
// (v_j - v_c) + a_centre v_c (the centre slot holds the row sum).  STREAM:
// non-temporal matrix loads (level 0, read once per pass from HBM); coarse
// levels stay in cache between the passes of a cycle.
template <int DIM, bool STREAM, typename V>
__device__ __forceinline__ float mg_av(const MgLv& L, int c, const int* ijk, float vc, V val) {
    constexpr int S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    const bool diff = L.diff != 0;
    bool inner = ijk[0] > 0 && ijk[0] < L.n[0] - 1 && ijk[1] > 0 && ijk[1] < L.n[1] - 1;
    if (DIM == 3) inner = inner && ijk[2] > 0 && ijk[2] < L.n[2] - 1;
    float acc = 0.0f;
    if (inner) {       // constant offsets: every load of the row can be issued at once
        const int sy = L.n[0], sz = L.n[0] * L.n[1];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float* pa = L.A + (size_t)s * L.mps + c;
            const float a = STREAM ? ld_stream(pa) : *pa;
            if (s == CEN) {
                acc += a * vc;
            } else {
                const float v = val(c + (s % 3 - 1) + ((s / 3) % 3 - 1) * sy + (DIM == 3 ? (s / 9 - 1) * sz : 0));
                acc += diff ? a * (v - vc) : a * v;
            }
        }
        return acc;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const float* pa = L.A + (size_t)s * L.mps + c;
        const float a = STREAM ? ld_stream(pa) : *pa;
        if (s == CEN) {
            acc += a * vc;
            continue;
        }
        int j;
        const bool ok = mg_nbs<DIM>(L.n, L.per, ijk, s, c, j);
        const float v = val(j);
        const float term = diff ? a * (v - vc) : a * v;
        acc += ok ? term : 0.0f;
    }
    return acc;
}

// (A x)_c of the FP64 PPE matrix (plain form, planes at stride m.mps).
template <int DIM, bool NT, typename F>
__device__ __forceinline__ double mg_spmv64(const MeshDev& m, const double* __restrict__ A, int c, F val) {
    constexpr int S = Dims<DIM>::S;
    int ijk[3];
    cell_ijk(m, c, ijk);
    double acc = 0.0;
    if (mg_interior<DIM>(m, ijk)) {
#pragma unroll
        for (int s = 0; s < S; ++s) acc += ld_mat<NT>(A + (size_t)s * m.mps + c) * val(c + mg_off<DIM>(m, s));
        return acc;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const double a = ld_mat<NT>(A + (size_t)s * m.mps + c);
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

// Per-axis prolongation weight: a fine cell at offset o from child c of
// coarse cell I (q = c + o + 1 in 0..3) lies in coarse cell I +
// floor((c + o) / 2) (weight 3/4) and takes 1/4 from that cell's neighbour
// on its side; e in 0..2 is the coarse offset + 1.
__device__ __forceinline__ double mg_w1(int q, int e) {
    const int big = (q + 1) >> 1;
    const int small = big + ((q & 1) ? -1 : 1);
    return e == big ? 0.75 : (e == small ? 0.25 : 0.0);
}

// row[e] = sum_s a[s] prod_a w(c_a + o_a(s) + 1, e_a): the 3^d row of a
// child (parity c[]) contracted with the per-axis prolongation weights one
// axis at a time.
template <int DIM>
__device__ __forceinline__ void mg_contract(const double* a, const int* c, double* row) {
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

// A_c = R A_f P, accumulated in FP64.  One thread per child i of a coarse
// cell I, the 2^d children of I in consecutive lanes.  Row i of A_f P is
// sum_s a_s(i) P[j_s] with P[j][K] = pn[j] w(j, K) over the coarse cells K
// of j that lie inside the mesh and are unknown; all of them lie in the 3^d
// block around I.  Since pn[j] = 0 at fine cells that are not unknown, the
// child contracts a'_s = a_s(i) pn[j_s] (0 for a slot outside the mesh) with
// the separable weights w, and the coarse cells outside the mesh or not
// unknown are dropped from the sum afterwards (a factor of K alone).  The
// children's rows are added across their lanes and scaled by 2^-d (R).
template <int DIM, typename TA>
__global__ __launch_bounds__(kBlock) void k_mg_galerkin(MeshDev mf, const TA* __restrict__ Af,
                                                        const uint8_t* __restrict__ unk_f,
                                                        const float* __restrict__ pn, MeshDev mc,
                                                        const uint8_t* __restrict__ unk_c, float* __restrict__ Ac,
                                                        float* __restrict__ dinv_c) {
    constexpr int S = Dims<DIM>::S, CEN = Dims<DIM>::CEN, CH = 1 << DIM;
    const int total = mc.Nc * CH;        // the grid is a multiple of CH threads: a cell's lanes share a pass
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        const int I = t / CH, ch = t % CH;
        int ic[3] = {0, 0, 0};
        mg_ijk(mc.n, I, ic);
        int f[3] = {0, 0, 0};
        bool in = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            f[a] = 2 * ic[a] + ((ch >> a) & 1);
            in = in && f[a] < mf.n[a];
        }
        const bool cu = unk_c[I] != 0;
        double row[S];
#pragma unroll
        for (int s = 0; s < S; ++s) row[s] = 0.0;
        if (cu && in) {
            const int i = mg_at(mf.n, f);
            if (unk_f[i]) {
                double a[S];
                bool inner = f[0] > 0 && f[0] < mf.n[0] - 1 && f[1] > 0 && f[1] < mf.n[1] - 1;
                if (DIM == 3) inner = inner && f[2] > 0 && f[2] < mf.n[2] - 1;
                if (inner) {
                    const int sy = mf.n[0], sz = mf.n[0] * mf.n[1];
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        a[s] = (double)Af[(size_t)s * mf.mps + i] *
                               (double)pn[i + (s % 3 - 1) + ((s / 3) % 3 - 1) * sy + (DIM == 3 ? (s / 9 - 1) * sz : 0)];
                } else {
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        int j;
                        const bool ok = mg_nbs<DIM>(mf.n, mf.periodic, f, s, i, j);
                        const double v = (double)Af[(size_t)s * mf.mps + i] * (double)pn[j];
                        a[s] = ok ? v : 0.0;
                    }
                }
                const int par[3] = {ch & 1, (ch >> 1) & 1, (ch >> 2) & 1};
                mg_contract<DIM>(a, par, row);
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            row[s] += __shfl_xor(row[s], 1);
            row[s] += __shfl_xor(row[s], 2);
            if (DIM == 3) row[s] += __shfl_xor(row[s], 4);
        }
        // lane ch writes the slots s = ch (mod 2^d)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s % CH != ch) continue;
            int K;
            const bool okn = mg_nbs<DIM>(mc.n, mc.periodic, ic, s, I, K);
            const bool ok = cu && okn && unk_c[K] != 0;
            const double v = ok ? row[s] * (1.0 / (double)CH) : 0.0;
            Ac[(size_t)s * mc.mps + I] = (float)v;
            if (s == CEN) dinv_c[I] = (cu && v != 0.0 && isfinite(v)) ? (float)(1.0 / v) : 0.0f;
        }
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
// coarsest matrix, one block of kMgTailBlock threads, in LDS.  Per column k:
// wave 0 finds the pivot row (largest |M[r][k]|, r >= k, the lowest r on
// ties) by a butterfly; the pivot row p, divided by the pivot, becomes row k
// and the old row k moves to p; then every other row r subtracts M[r][k]
// times the new row k.  flag = 1 when a pivot vanishes.
__global__ __launch_bounds__(kMgTailBlock) void k_mg_invert(const double* __restrict__ D, int N,
                                                            float* __restrict__ inv, int* flag) {
    constexpr int RG = kMgTailBlock / (2 * kMgMaxCoarse);     // row groups
    __shared__ double M[kMgMaxCoarse][2 * kMgMaxCoarse + 1];
    __shared__ double prow[2 * kMgMaxCoarse], orow[2 * kMgMaxCoarse], fac[kMgMaxCoarse];
    __shared__ int piv;
    const int W = 2 * N, tid = threadIdx.x;
    const int col = tid % (2 * kMgMaxCoarse), r0 = tid / (2 * kMgMaxCoarse);
    if (col < W)
        for (int r = r0; r < N; r += RG) M[r][col] = col < N ? D[r * N + col] : (col - N == r ? 1.0 : 0.0);
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        if (tid < 64) {
            double v = (tid >= k && tid < N) ? fabs(M[tid][k]) : -1.0;
            int idx = tid;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double ov = __shfl_xor(v, o);
                const int oi = __shfl_xor(idx, o);
                if (ov > v || (ov == v && oi < idx)) {
                    v = ov;
                    idx = oi;
                }
            }
            if (tid == 0) {
                piv = idx;
                if (!(v > 0.0)) *flag = 1;
            }
        }
        __syncthreads();
        const int p = piv;
        const double d = M[p][k];
        const double id = d != 0.0 ? 1.0 / d : 0.0;
        if (tid < W) {
            prow[tid] = M[p][tid] * id;
            orow[tid] = M[k][tid];
        } else if (tid >= 2 * kMgMaxCoarse && tid < 2 * kMgMaxCoarse + N) {
            const int r = tid - 2 * kMgMaxCoarse;
            fac[r] = r == k ? 0.0 : (r == p ? M[k][k] : M[r][k]);
        }
        __syncthreads();
        if (col < W)
            for (int r = r0; r < N; r += RG) {
                if (r == k)
                    M[r][col] = prow[col];
                else
                    M[r][col] = (r == p ? orow[col] : M[r][col]) - fac[r] * prow[col];
            }
        __syncthreads();
    }
    for (int e = tid; e < N * N; e += blockDim.x) inv[e] = (float)M[e / N][N + e % N];
}

// ---------------------------------------------------------------------------
// Cycle kernels (FP32)
// ---------------------------------------------------------------------------

// Down-leg of level F: x = w D^-1 b, r = b - A x at unknown cells (0
// elsewhere), coarse right-hand side = the mean of the children's r.  Item t
// is child t % 2^d of coarse cell t / 2^d; the children of one coarse cell
// sit in consecutive lanes and add their residuals across them.  x_j of the
// neighbours is formed from b and D^-1 on the fly, so the level needs no
// separate pre-smoothing pass.
template <int DIM, bool STREAM>
__device__ __forceinline__ void mg_down_at(const MgLv& F, const MgLv& C, int t) {
    constexpr int CH = 1 << DIM;
    const int I = t / CH, ch = t % CH;
    int ic[3] = {0, 0, 0};
    mg_ijk(C.n, I, ic);
    int f[3] = {0, 0, 0};
    bool in = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        f[a] = 2 * ic[a] + ((ch >> a) & 1);
        in = in && f[a] < F.n[a];
    }
    float r = 0.0f;
    if (in) {
        const int c = mg_at(F.n, f);
        const float bc = F.b[c];
        const float xc = kMgOmega * F.dinv[c] * bc;
        F.x[c] = xc;
        if (F.unk[c])
            r = bc - mg_av<DIM, STREAM>(F, c, f, xc, [&](int j) { return kMgOmega * F.dinv[j] * F.b[j]; });
    }
    r += __shfl_xor(r, 1);
    r += __shfl_xor(r, 2);
    if (DIM == 3) r += __shfl_xor(r, 4);
    if (ch == 0) C.b[I] = r * (1.0f / (float)CH);
}

// Up-leg, first half: x_j += P y_c at unknown fine cells (y_c is 0 at coarse
// cells that are not unknown, so only the mesh edges need a test).
template <int DIM>
__device__ __forceinline__ void mg_prolong_at(const MgLv& F, const MgLv& C, int j) {
    if (!F.unk[j]) return;
    int fj[3] = {0, 0, 0};
    mg_ijk(F.n, j, fj);
    float add = 0.0f;
#pragma unroll
    for (int corner = 0; corner < (1 << DIM); ++corner) {
        int k[3] = {0, 0, 0};
        float wt = 1.0f;
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int far = (corner >> a) & 1;
            int v = (fj[a] >> 1) + (far ? ((fj[a] & 1) ? 1 : -1) : 0);
            const bool lo = v < 0, hi = v >= C.n[a];
            ok = ok && (!(lo || hi) || C.per[a] != 0);
            k[a] = lo ? v + C.n[a] : (hi ? v - C.n[a] : v);      // in range either way
            wt *= far ? 0.25f : 0.75f;
        }
        const float yk = C.y[mg_at(C.n, k)];
        add += ok ? wt * yk : 0.0f;
    }
    F.x[j] += add * F.pn[j];
}

// Up-leg, second half: y = x + w D^-1 (b - A x) at unknown cells, 0 elsewhere.
template <int DIM, bool STREAM>
__device__ __forceinline__ void mg_smooth_at(const MgLv& F, int c) {
    float y = 0.0f;
    if (F.unk[c]) {
        int ijk[3] = {0, 0, 0};
        mg_ijk(F.n, c, ijk);
        const float xc = F.x[c];
        const float* x = F.x;
        y = xc + kMgOmega * F.dinv[c] * (F.b[c] - mg_av<DIM, STREAM>(F, c, ijk, xc, [&](int j) { return x[j]; }));
    }
    F.y[c] = y;
}

// Down-leg over bricks of 64 x 2 x 2 (3D) or 64 x 4 (2D) fine cells, one
// per block (grid: bricks along x, y, z), one cell per thread so that the
// matrix planes stream in whole rows; the residuals meet in LDS and the
// brick's coarse cells add their children there, in child order.
template <int DIM>
struct MgBrick {
    static constexpr int BX = 64, BY = DIM == 3 ? 2 : 4, BZ = DIM == 3 ? 2 : 1;
};

template <int DIM, bool STREAM>
__global__ __launch_bounds__(kBlock) void k_mg_down(MgLv F, MgLv C) {
    constexpr int BX = MgBrick<DIM>::BX, BY = MgBrick<DIM>::BY, BZ = MgBrick<DIM>::BZ, CH = 1 << DIM;
    static_assert(BX * BY * BZ == kBlock, "one fine cell per thread");
    __shared__ float rs[BZ][BY][BX];
    const int tx = threadIdx.x % BX, ty = (threadIdx.x / BX) % BY, tz = threadIdx.x / (BX * BY);
    const int f[3] = {(int)blockIdx.x * BX + tx, (int)blockIdx.y * BY + ty, DIM == 3 ? (int)blockIdx.z * BZ + tz : 0};
    const bool in = f[0] < F.n[0] && f[1] < F.n[1] && (DIM == 2 || f[2] < F.n[2]);
    float r = 0.0f;
    if (in) {
        const int c = mg_at(F.n, f);
        const float bc = F.b[c];
        const float xc = kMgOmega * F.dinv[c] * bc;
        F.x[c] = xc;
        if (F.unk[c])
            r = bc - mg_av<DIM, STREAM>(F, c, f, xc, [&](int j) { return kMgOmega * F.dinv[j] * F.b[j]; });
    }
    rs[tz][ty][tx] = r;
    __syncthreads();
    constexpr int CX = BX / 2, CY = BY / 2, CZ = DIM == 3 ? BZ / 2 : 1;
    if (threadIdx.x < CX * CY * CZ) {
        const int cx = threadIdx.x % CX, cy = (threadIdx.x / CX) % CY, cz = threadIdx.x / (CX * CY);
        const int I[3] = {(int)blockIdx.x * CX + cx, (int)blockIdx.y * CY + cy, DIM == 3 ? (int)blockIdx.z * CZ + cz : 0};
        if (I[0] < C.n[0] && I[1] < C.n[1] && (DIM == 2 || I[2] < C.n[2])) {
            float sum = 0.0f;
#pragma unroll
            for (int ch = 0; ch < CH; ++ch)
                sum += rs[DIM == 3 ? 2 * cz + ((ch >> 2) & 1) : 0][2 * cy + ((ch >> 1) & 1)][2 * cx + (ch & 1)];
            C.b[mg_at(C.n, I)] = sum * (1.0f / (float)CH);
        }
    }
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_mg_prolong(MgLv F, MgLv C) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < F.Nc; j += gridDim.x * blockDim.x)
        mg_prolong_at<DIM>(F, C, j);
}

template <int DIM, bool STREAM>
__global__ __launch_bounds__(kBlock) void k_mg_smooth(MgLv F) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < F.Nc; c += gridDim.x * blockDim.x)
        mg_smooth_at<DIM, STREAM>(F, c);
}

// The coarse end of the cycle in one workgroup: down-legs of levels
// l[0] .. l[nl - 2], the coarsest level l[nl - 1] solved with its dense
// inverse (y = inv b, 0 at cells that are not unknown), then the up-legs back
// to l[0].  Every phase ends at a barrier of the workgroup, which orders its
// global stores before the next phase's loads.
struct MgTail {
    int nl;
    const float* inv;
    MgLv l[kMgMaxTail];
};

template <int DIM>
__global__ __launch_bounds__(kMgTailBlock) void k_mg_tail(MgTail T) {
    constexpr int CH = 1 << DIM;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int l = 0; l + 1 < T.nl; ++l) {
        const int total = T.l[l + 1].Nc * CH;
        for (int t = tid; t < total; t += nt) mg_down_at<DIM, false>(T.l[l], T.l[l + 1], t);
        __syncthreads();
    }
    {
        const MgLv& Lc = T.l[T.nl - 1];
        const int N = Lc.Nc;                 // <= kMgMaxCoarse: 16 lanes per row
        const int r = tid >> 4, q = tid & 15;
        float acc = 0.0f;
        if (r < N)
            for (int k = q; k < N; k += 16) acc += T.inv[r * N + k] * Lc.b[k];
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) acc += __shfl_xor(acc, o);
        if (r < N && q == 0) Lc.y[r] = Lc.unk[r] ? acc : 0.0f;
    }
    __syncthreads();
    for (int l = T.nl - 2; l >= 0; --l) {
        for (int j = tid; j < T.l[l].Nc; j += nt) mg_prolong_at<DIM>(T.l[l], T.l[l + 1], j);
        __syncthreads();
        for (int c = tid; c < T.l[l].Nc; c += nt) mg_smooth_at<DIM, false>(T.l[l], c);
        __syncthreads();
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
    // the FP64 and FP32 matrices of level 0 stay in the last-level cache when
    // they fit there with room for the vectors; larger ones are streamed
    w->nt = (size_t)S * m.Nc * (sizeof(double) + sizeof(float)) > (kCacheFitBytes * 5) / 6;
    // the tail: the smallest levels, at most kMgMaxTail of them
    w->tail = w->L - 1;
    while (w->tail > 0 && w->lev[w->tail - 1].m.Nc <= kMgTailCells && w->L - (w->tail - 1) <= kMgMaxTail) --w->tail;
    const int Nc = w->usable ? w->lev[w->L - 1].m.Nc : 1;
    if (e == hipSuccess) e = hipMalloc((void**)&w->dense, (size_t)Nc * Nc * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&w->inv, (size_t)Nc * Nc * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&w->part, 4 * kMgParts * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&w->flag, sizeof(int));
    if (e == hipSuccess) e = hipHostMalloc((void**)&w->host, 8 * sizeof(double), hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&w->host_dev, w->host, 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc((void**)&w->scal, 64);
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

    if (w->flag) (void)hipFree(w->flag);
    if (w->host) (void)hipHostFree(w->host);
    if (w->ev) (void)hipEventDestroy(w->ev);
    if (w->scal) (void)hipFree(w->scal);
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
        const int gb = ((C.m.Nc << DIM) + kBlock - 1) / kBlock;
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
    hipLaunchKernelGGL(k_mg_invert, dim3(1), dim3(kMgTailBlock), 0, st, w.dense, Lc.m.Nc, w.inv, w.flag);
    return hipGetLastError();
}

hipError_t mg_setup(const MeshDev& m, MgWork& w, const SetDev& set, hipStream_t st) {
    if (!w.usable) return hipErrorNotSupported;
    return m.dim == 2 ? mg_setup_dim<2>(w, set, st) : mg_setup_dim<3>(w, set, st);
}

static MgLv mg_lv(const MgLevel& L, int level) {
    MgLv v{};
    for (int a = 0; a < 3; ++a) {
        v.n[a] = a < L.m.dim ? L.m.n[a] : 1;
        v.per[a] = a < L.m.dim ? L.m.periodic[a] : 0;
    }
    v.Nc = L.m.Nc;
    v.diff = level == 0 ? 1 : 0;
    v.mps = L.m.mps;
    v.A = L.A;
    v.unk = L.unk;
    v.dinv = L.dinv;
    v.pn = L.pn;
    v.x = L.x;
    v.y = L.y;
    v.b = L.b;
    return v;
}

// One V-cycle on level 0: rhs lev[0].b, result lev[0].y.  Levels above the
// tail take one down-leg launch each and two up-leg launches (prolongation,
// smoothing); the tail runs in one launch.
template <int DIM>
static void mg_cycle_dim(MgWork& w, hipStream_t st) {
    const int ts = w.tail;
    for (int l = 0; l < ts; ++l) {
        const MgLv F = mg_lv(w.lev[l], l), C = mg_lv(w.lev[l + 1], l + 1);
        const dim3 g((F.n[0] + MgBrick<DIM>::BX - 1) / MgBrick<DIM>::BX, (F.n[1] + MgBrick<DIM>::BY - 1) / MgBrick<DIM>::BY,
                     (F.n[2] + MgBrick<DIM>::BZ - 1) / MgBrick<DIM>::BZ);
        if (l == 0 && w.nt)
            hipLaunchKernelGGL((k_mg_down<DIM, true>), g, dim3(kBlock), 0, st, F, C);
        else
            hipLaunchKernelGGL((k_mg_down<DIM, false>), g, dim3(kBlock), 0, st, F, C);
    }
    MgTail T{};
    T.nl = w.L - ts;
    T.inv = w.inv;
    for (int k = 0; k < T.nl; ++k) T.l[k] = mg_lv(w.lev[ts + k], ts + k);
    hipLaunchKernelGGL(k_mg_tail<DIM>, dim3(1), dim3(kMgTailBlock), 0, st, T);
    for (int l = ts - 1; l >= 0; --l) {
        const MgLv F = mg_lv(w.lev[l], l), C = mg_lv(w.lev[l + 1], l + 1);
        const dim3 g(grid_for(F.Nc));
        hipLaunchKernelGGL(k_mg_prolong<DIM>, g, dim3(kBlock), 0, st, F, C);
        if (l == 0 && w.nt)
            hipLaunchKernelGGL((k_mg_smooth<DIM, true>), g, dim3(kBlock), 0, st, F);
        else
            hipLaunchKernelGGL((k_mg_smooth<DIM, false>), g, dim3(kBlock), 0, st, F);
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
template <int DIM, bool NT>
__global__ void k_mgo_resid(MeshDev m, const double* __restrict__ A, const uint8_t* __restrict__ unk,
                            const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ r,
                            double* __restrict__ rhat, int set_rhat, double* part) {
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (unk[c]) v = b[c] - mg_spmv64<DIM, NT>(m, A, c, [&](int j) { return x[j]; });
        r[c] = v;
        if (set_rhat) rhat[c] = v;
        q[0] += v * v;
        q[1] += b[c] * b[c];
        q[2] += (set_rhat ? v : rhat[c]) * v;
    }
    mg_parts(q, 3, part);
}

// Scalars of the outer iteration, kept on the device so that an iteration
// needs one host synchronisation (after its last reduction) instead of three;
// each is formed by the same IEEE operations the host would use.
struct MgScal {
    double rho, alpha, omega, rho_new;
    int flag;                    // rhat.v vanished or is not finite: x and r were left as they were
};

__global__ void k_mgo_restart(MgScal* sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->rho = 1.0;
        sc->alpha = 1.0;
        sc->omega = 1.0;
        sc->flag = 0;
    }
}

// p = r + beta (p - omega v), beta = (rho_new / rho) (alpha / omega) (0 on
// the first iteration after a (re)start, with omega 0); the cycle's FP32
// right-hand side b0 = p
__global__ void k_mgo_p(int N, const uint8_t* __restrict__ unk, const double* __restrict__ r, double* __restrict__ p,
                        const double* __restrict__ v, const MgScal* __restrict__ sc, int first,
                        float* __restrict__ b0) {
    const double beta = first ? 0.0 : (sc->rho_new / sc->rho) * (sc->alpha / sc->omega);
    const double omega = first ? 0.0 : sc->omega;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        const double pv = unk[c] ? r[c] + beta * (p[c] - omega * v[c]) : 0.0;
        p[c] = pv;
        b0[c] = (float)pv;
    }
}

// z = (double) y0 (the preconditioned direction), w = A z; partials rhat.w
// (or t.s, t.t with s given).  F32: A z from the FP32 copy of the matrix in
// difference form, sum a_j (z_j - z_c) + rowsum z_c, formed in FP64.
template <int DIM, bool NT, bool F32>
__global__ void k_mgo_apply(MeshDev m, const double* __restrict__ A, const float* __restrict__ A32,
                            const uint8_t* __restrict__ unk, const float* __restrict__ y0, double* __restrict__ z,
                            double* __restrict__ wv, const double* __restrict__ rhat, const double* __restrict__ s,
                            double* part) {
    constexpr int S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        double v = 0.0;
        const double zc = (double)y0[c];
        if (unk[c]) {
            if constexpr (F32) {
                int ijk[3];
                cell_ijk(m, c, ijk);
                if (mg_interior<DIM>(m, ijk)) {
#pragma unroll
                    for (int sl = 0; sl < S; ++sl) {
                        const double a = (double)ld_mat<NT>(A32 + (size_t)sl * m.mps + c);
                        v += sl == CEN ? a * zc : a * ((double)y0[c + mg_off<DIM>(m, sl)] - zc);
                    }
                } else {
#pragma unroll
                    for (int sl = 0; sl < S; ++sl) {
                        const double a = (double)ld_mat<NT>(A32 + (size_t)sl * m.mps + c);
                        if (sl == CEN) {
                            v += a * zc;
                            continue;
                        }
                        int j;
                        double sh[3];
                        if (!neighbour<DIM>(m, ijk, sl, j, sh)) continue;
                        v += a * ((double)y0[j] - zc);
                    }
                }
            } else {
                v = mg_spmv64<DIM, NT>(m, A, c, [&](int j) { return (double)y0[j]; });
            }
        }
        z[c] = zc;
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
__global__ void k_mgo_s(int N, const double* __restrict__ r, const double* __restrict__ v,
                        const MgScal* __restrict__ sc, double* __restrict__ s, float* __restrict__ b0) {
    const double alpha = sc->alpha;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        const double sv = r[c] - alpha * v[c];
        s[c] = sv;
        b0[c] = (float)sv;
    }
}

// x += alpha ph + omega sh; r = s - omega t; partials r.r, rhat.r (nothing
// changes when the iteration broke down)
__global__ void k_mgo_xr(int N, double* __restrict__ x, const double* __restrict__ ph, const double* __restrict__ sh,
                         const double* __restrict__ s, const double* __restrict__ t, const MgScal* __restrict__ sc,
                         double* __restrict__ r, const double* __restrict__ rhat, double* part) {
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    const double alpha = sc->alpha, omega = sc->omega;
    if (!sc->flag)
        for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
            x[c] = x[c] + alpha * ph[c] + omega * sh[c];
            const double rv = s[c] - omega * t[c];
            r[c] = rv;
            q[0] += rv * rv;
            q[1] += rhat[c] * rv;
        }
    mg_parts(q, 2, part);
}

// Totals of nq partial rows over nblk blocks, in block order, and what the
// iteration makes of them:
//   kResid  r.r, b.b, rhat.r -> rho_new = rhat.r; host {r.r, b.b, rhat.r, the
//           right-hand side's non-finite flag, the coarsest matrix's singular flag}
//   kAlpha  rhat.v -> alpha = rho_new / rhat.v (flag when 0 or not finite)
//   kOmega  t.s, t.t -> omega = t.s / t.t (0 when t.t = 0)
//   kNext   r.r, rhat.r -> rho = rho_new, rho_new = rhat.r;
//           host {r.r, rho_new, omega, flag}
enum { kResid = 0, kAlpha = 1, kOmega = 2, kNext = 3 };

__global__ void k_mgo_reduce(const double* __restrict__ part, int nblk, int nq, int mode, MgScal* sc,
                             double* __restrict__ host, const int* __restrict__ bad,
                             const int* __restrict__ cflag) {
    __shared__ double lds[4][kBlock / 64];
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nq; ++k)
        for (int b = threadIdx.x; b < nblk; b += blockDim.x) q[k] += part[k * kMgParts + b];
    block_sum<4>(q, lds);
    if (threadIdx.x != 0) return;
    if (mode == kResid) {
        sc->rho_new = q[2];
        host[0] = q[0];
        host[1] = q[1];
        host[2] = q[2];
        host[3] = bad ? (double)*bad : 0.0;        // non-finite right-hand side
        host[4] = cflag ? (double)*cflag : 0.0;    // singular coarsest matrix
    } else if (mode == kAlpha) {
        const double rv = q[0];
        const bool bad = !(fabs(rv) > 0.0) || !isfinite(rv);
        sc->flag = bad ? 1 : 0;
        sc->alpha = bad ? 0.0 : sc->rho_new / rv;
    } else if (mode == kOmega) {
        sc->omega = q[1] > 0.0 ? q[0] / q[1] : 0.0;
    } else {
        if (!sc->flag) {
            sc->rho = sc->rho_new;
            sc->rho_new = q[1];
        }
        host[0] = q[0];
        host[1] = sc->rho_new;
        host[2] = sc->omega;
        host[3] = (double)sc->flag;
    }
}

// Reduction in mode `mode`; with `wait`, the host waits for it (polling an
// event, which wakes it sooner than a blocking stream synchronisation) and
// reads the five values its mode leaves in pinned host memory (bad: the
// right-hand side's device flag, reported by kResid).
static hipError_t totals(MgWork& w, int nblk, int nq, int mode, hipStream_t st, bool wait, double* out,
                         const int* bad = nullptr) {
    hipLaunchKernelGGL(k_mgo_reduce, dim3(1), dim3(kBlock), 0, st, w.part, nblk, nq, mode, w.scal, w.host_dev, bad,
                       mode == kResid ? w.flag : nullptr);
    if (!wait) return hipGetLastError();
    hipError_t e = hipEventRecord(w.ev, st);
    if (e == hipSuccess)
        while ((e = hipEventQuery(w.ev)) == hipErrorNotReady) {
        }
    if (e == hipSuccess) {
        const volatile double* h = w.host;
        for (int k = 0; k < 5; ++k) out[k] = h[k];
    }
    return e;
}

// Right-preconditioned Bi-CGSTAB on the set's FP64 matrix from x (FP64
// vectors of the workspace); b: effective right-hand side.
template <int DIM>
static hipError_t mg_bicgstab_dim(const MeshDev& m, MgWork& w, const SetDev& set, const MgVecs& V, double tol,
                                  int max_iter, bool f32_products, const int* bad, hipStream_t st, MgResult* out) {
    const int N = m.Nc;
    const int g = (N + kBlock - 1) / kBlock > kMgParts ? kMgParts : (N + kBlock - 1) / kBlock;
    const double* A = set.amat;
    const uint8_t* unk = set.unknown;
    float* b0 = w.lev[0].b;
    const float* y0 = w.lev[0].y;
    double t4[5];                  // totals of the last reduction waited for
    if (!w.usable) return hipErrorNotSupported;
    auto resid = [&]() {
        if (w.nt)
            hipLaunchKernelGGL((k_mgo_resid<DIM, true>), dim3(g), dim3(kBlock), 0, st, m, A, unk, V.b, V.x, V.r,
                               V.rhat, 1, w.part);
        else
            hipLaunchKernelGGL((k_mgo_resid<DIM, false>), dim3(g), dim3(kBlock), 0, st, m, A, unk, V.b, V.x, V.r,
                               V.rhat, 1, w.part);
    };
    const float* A32 = set.amat32;
    auto apply = [&](double* z, double* wv, const double* sv) {
        if (f32_products) {
            if (w.nt)
                hipLaunchKernelGGL((k_mgo_apply<DIM, true, true>), dim3(g), dim3(kBlock), 0, st, m, A, A32, unk, y0, z,
                                   wv, V.rhat, sv, w.part);
            else
                hipLaunchKernelGGL((k_mgo_apply<DIM, false, true>), dim3(g), dim3(kBlock), 0, st, m, A, A32, unk, y0,
                                   z, wv, V.rhat, sv, w.part);
        } else if (w.nt) {
            hipLaunchKernelGGL((k_mgo_apply<DIM, true, false>), dim3(g), dim3(kBlock), 0, st, m, A, A32, unk, y0, z,
                               wv, V.rhat, sv, w.part);
        } else {
            hipLaunchKernelGGL((k_mgo_apply<DIM, false, false>), dim3(g), dim3(kBlock), 0, st, m, A, A32, unk, y0, z,
                               wv, V.rhat, sv, w.part);
        }
    };
    hipError_t e = mg_setup_dim<DIM>(w, set, st);
    if (e != hipSuccess) return e;
    // the right-hand side's check and the coarsest matrix's flag come back with
    // the first residual's totals (one host wait for the three)
    resid();
    if ((e = totals(w, g, 3, kResid, st, true, t4, bad)) != hipSuccess) return e;
    *out = MgResult{};
    out->coarse_singular = t4[4] != 0.0 ? 1 : 0;
    if (t4[3] != 0.0) {            // non-finite right-hand side: nothing is solved
        out->bad = 1;
        return hipSuccess;
    }
    const double bb = t4[1];
    out->bnorm = sqrt(bb);
    if (bb == 0.0) {
        out->converged = 1;
        return hipSuccess;
    }
    const double tol2 = tol * tol * bb;
    double rr = t4[0], rho_new = t4[2];
    int iters = 0, restarts = 0;
    while (rr > tol2 && iters < max_iter) {
        // (re)start: rhat = r (set by the residual kernel), rho = alpha = omega = 1, p = v = 0
        hipLaunchKernelGGL(k_mgo_restart, dim3(1), dim3(64), 0, st, w.scal);
        bool first = true, restart = false;
        while (iters < max_iter) {
            if (!first && !(fabs(rho_new) > 1e-300)) {
                restart = true;
                break;
            }
            hipLaunchKernelGGL(k_mgo_p, dim3(g), dim3(kBlock), 0, st, N, unk, V.r, V.p, V.v, w.scal, first ? 1 : 0,
                               b0);
            first = false;
            mg_cycle(m, w, st);
            apply(V.ph, V.v, nullptr);
            if ((e = totals(w, g, 1, kAlpha, st, false, nullptr)) != hipSuccess) return e;
            hipLaunchKernelGGL(k_mgo_s, dim3(g), dim3(kBlock), 0, st, N, V.r, V.v, w.scal, V.s, b0);
            mg_cycle(m, w, st);
            apply(V.sh, V.t, V.s);
            if ((e = totals(w, g, 2, kOmega, st, false, nullptr)) != hipSuccess) return e;
            hipLaunchKernelGGL(k_mgo_xr, dim3(g), dim3(kBlock), 0, st, N, V.x, V.ph, V.sh, V.s, V.t, w.scal, V.r,
                               V.rhat, w.part);
            if ((e = totals(w, g, 2, kNext, st, true, t4)) != hipSuccess) return e;
            if (t4[3] != 0.0) {          // rhat.v broke down: x unchanged, restart from its residual
                restart = true;
                break;
            }
            rr = t4[0];
            rho_new = t4[1];
            const double omega = t4[2];
            ++iters;
            if (rr <= tol2) break;
            if (omega == 0.0 || !std::isfinite(rr)) {
                restart = true;
                break;
            }
        }
        // confirm with the true residual (and restart from it if needed)
        resid();
        if ((e = totals(w, g, 3, kResid, st, true, t4)) != hipSuccess) return e;
        rr = t4[0];
        rho_new = t4[2];
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
                       bool f32_products, const int* bad, hipStream_t st, MgResult* out) {
    return m.dim == 2 ? mg_bicgstab_dim<2>(m, w, set, V, tol, max_iter, f32_products, bad, st, out)
                      : mg_bicgstab_dim<3>(m, w, set, V, tol, max_iter, f32_products, bad, st, out);
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
