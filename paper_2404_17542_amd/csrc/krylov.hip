// Bi-CGSTAB for the PPE (Sec. 3.3) on the offset-plane matrix.
//
// One iteration is two fused kernels (T = double or float for vectors and
// matrix; every inner product is accumulated in double):
//   P-stage:  omega = (t.s)/(t.t);  rho' = rhat.s - omega rhat.t;
//             beta = (rho'/rho)(alpha/omega);
//             r = s - omega t;  x += alpha p + omega s;
//             p' = r + beta (p - omega v);  v' = A p'
//             (p' at the stencil neighbours is formed on the fly from s, t,
//             p, v, so p' and v' need no grid-wide barrier); dots rhat.v', r.r
//   S-stage:  alpha = rho'/(rhat.v');  s = r - alpha v';  t = A s
//             (s at the neighbours formed on the fly); dots t.s, t.t,
//             rhat.s, rhat.t
// rho' uses rhat.r_new = rhat.s - omega rhat.t, which is what lets the x/r
// update fuse into the next SpMV.  The last block of each kernel (ticket
// counter) reduces the per-block partial sums in a fixed order, so results
// are run-to-run deterministic, and computes the scalars of the next stage.
// Vectors are zero at non-unknown cells; matrix rows/columns of non-unknown
// cells are zero.
#include <hip/hip_ext.h>

#include <cmath>
#include <mutex>
#include <type_traits>

#include "common.h"

namespace mcd {

struct KState {
    double rho, alpha, omega;
    double bb, rr, rr0, rv;
    double tol2;
    double rho_prev;   // rho of the previous iteration (kept by the P-stage)
    double rho_res;    // rhat.r of a replaced residual (resume P-stage)
    double delta2;     // > 0: also stop when r.r <= delta2 * rr_max (residual replacement due)
    double rr_max;     // largest r.r since the recursion started or its residual was replaced
    int done;          // 0 running, 1 recurrence below the stop threshold, 2 breakdown
    int iter;
    int pad[2];
};

// P-stage modes: a normal iteration; the first iteration after an (re)start
// (r = p = s); resuming after the residual was replaced by a recomputed one
// (r given, x already current, beta from the replaced rho).
enum { P_NORMAL = 0, P_FIRST = 1, P_RESUME = 2 };

// Launch shape of the stage kernels: blocks of 512 threads, at most 512 of
// them (16 waves per CU on 256 CUs; by default exactly min(512, tiles));
// per-block partial sums of one stage are reduced by every block of the next
// stage in a fixed order, so no grid barrier, fence or atomic is needed and
// every block derives bitwise the same scalars.  The block count and the 3D
// brick depth are run-time parameters (chosen by the autotuner).
constexpr int kKBlock = 512;
constexpr int kKGrid = 512;
constexpr int kDefaultDepth = 8;

template <typename T, typename TA = T>
struct KVec {
    T *x, *r, *rhat, *s, *t, *p[2], *v[2];
    const TA* A;     // [S][Nc]; TA = float for an FP32-stored matrix with FP64 vectors
    const T* b;
    // set for the set's own FP64 operator: its unknown flags; the stage
    // kernels then form the centre from the row's other slots
    const uint8_t* unk = nullptr;
};

struct KBufs {
    double* part[3];     // [NQ][cap] partials of init / P / S stages
    KState* st[3];       // state written by block 0 of init/finish, P, S
    int nblk;            // blocks (= partials) of the stage kernels in use
    int cap;             // partials capacity per quantity
    int ntx;             // tiles per row
    int nty;             // tile rows per plane (3D bricks)
    int ntiles;          // tiles (2D) or bricks (3D) of the mesh
    int tpb;             // tiles or bricks per block
    int tz;              // planes per brick (3D)
    int nt;              // matrix loads non-temporal (the iteration's data exceed the last-level cache)
};


// Sum of A[s][c] * val(j) over the stencil slots of cell c.  Interior cells
// use constant slot offsets; cells on the mesh edge take the general path.
template <int DIM, typename T, typename TA, typename F>
__device__ __forceinline__ T spmv_row(const MeshDev& m, const TA* __restrict__ A, int c, F val) {
    // An FP32-stored matrix is in difference form (centre slot = row sum):
    // sum_j a_j (x_j - x_c) + rowsum x_c.  FP64 matrices use the plain form.
    constexpr bool DIFF = sizeof(TA) < sizeof(double);
    constexpr int S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    int ijk[3];
    cell_ijk(m, c, ijk);
    bool interior = ijk[0] > 0 && ijk[0] < m.n[0] - 1 && ijk[1] > 0 && ijk[1] < m.n[1] - 1;
    if (DIM == 3) interior = interior && ijk[2] > 0 && ijk[2] < m.n[2] - 1;
    const T xc = DIFF ? val(c) : T(0);
    T acc = 0;
    if (interior) {
        const int n0 = m.n[0], n01 = m.n[0] * m.n[1];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int off = (s % 3 - 1) + (DIM > 1 ? ((s / 3) % 3 - 1) * n0 : 0) + (DIM > 2 ? (s / 9 - 1) * n01 : 0);
            const T a = (T)A[(size_t)s * m.mps + c];
            if (DIFF)
                acc += s == CEN ? a * xc : a * (val(c + off) - xc);
            else
                acc += a * val(c + off);
        }
        return acc;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const T a = (T)A[(size_t)s * m.mps + c];
        int j;
        double sh[3];
        if (!neighbour<DIM>(m, ijk, s, j, sh)) continue;
        if (DIFF)
            acc += s == CEN ? a * xc : a * (val(j) - xc);
        else
            acc += a * val(j);
    }
    return acc;
}

// Block sum of NQ values; result broadcast to every thread.
template <int NQ>
__device__ __forceinline__ void block_sum_all(double (&v)[NQ]) {
    __shared__ double lds[NQ][kKBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) lds[q][wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kKBlock / 64; ++w) s += lds[q][w];
        v[q] = s;
    }
    __syncthreads();
}

// Every block reduces the NQ x nblk partials of the previous stage in the
// same fixed order (thread t sums partials t, t + 512, ...; then a fixed
// block tree), so all blocks obtain bitwise the same totals.
template <int NQ>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, const KBufs& K, double (&tot)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < K.nblk; b += kKBlock) s += part[q * K.cap + b];
        tot[q] = s;
    }
    block_sum_all<NQ>(tot);
}

template <int NQ>
__device__ __forceinline__ void write_partials(double (&v)[NQ], double* part, const KBufs& K) {
    block_sum_all<NQ>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[q * K.cap + blockIdx.x] = v[q];
    }
}

// One block: reduce the init partials into the state the first P-stage
// reads.  done tests r.r against tol2 * bb; the recursion that follows stops
// at tol2_next * bb (tighter after a recurrence that converged while the
// true residual did not).
__global__ __launch_bounds__(kKBlock) void k_kfinish(KBufs K, int with_bb, double tol2, int keep_iter, double delta2,
                                                     double tol2_next) {
    double tot[2];
    reduce_partials<2>(K.part[0], K, tot);
    if (threadIdx.x == 0) {
        KState* S = K.st[2];
        if (with_bb) S->bb = tot[1];
        if (!keep_iter) S->iter = 0;
        S->rr = tot[0];
        S->rr0 = tot[0];
        S->rr_max = tot[0];
        S->delta2 = delta2;
        S->rho = tot[0];
        S->alpha = 1.0;
        S->omega = 1.0;
        S->done = (tot[0] <= tol2 * S->bb) ? 1 : 0;
        S->tol2 = tol2_next;
    }
}

// beta, omega and the new rho of a P-stage; false (and done = 2 written by
// the leader) on breakdown.
template <int MODE>
__device__ __forceinline__ bool p_scalars(const KState* in, const KBufs& K, bool leader, double& omega, double& beta,
                                          double& rho_new) {
    omega = 1.0;
    beta = 0.0;
    rho_new = in->rho;
    if (MODE == P_FIRST) return true;
    if (MODE == P_NORMAL) {
        double tot[4];
        reduce_partials<4>(K.part[2], K, tot);   // t.s, t.t, rhat.s, rhat.t
        omega = tot[0] / tot[1];
        rho_new = tot[2] - omega * tot[3];
        beta = (rho_new / in->rho) * (in->alpha / omega);
        if (tot[1] > 0.0 && isfinite(omega) && isfinite(beta) && omega != 0.0 && fabs(rho_new) >= 1e-30 * in->rr0)
            return true;
    } else {
        omega = in->omega;
        rho_new = in->rho_res;
        beta = (rho_new / in->rho_prev) * (in->alpha / omega);
        if (isfinite(beta) && omega != 0.0 && fabs(rho_new) >= 1e-30 * in->rr0) return true;
    }
    if (leader) {
        *K.st[1] = *in;
        K.st[1]->done = 2;
    }
    return false;
}

// ---------------------------------------------------------------------------
// 2D stage kernels on LDS tiles.  A block of 512 threads owns a 64 x 8 tile
// of cells; the operand of the stencil product (x, p' or s) is formed once
// per tile-plus-halo cell (66 x 10) into LDS, coalesced along rows, and the
// 9-point product then reads LDS only.  The owner of a tile cell also does
// that cell's element-wise updates in the same pass.
// ---------------------------------------------------------------------------

constexpr int TX = 64, TY = 8, HX = TX + 2, HY = TY + 2, NH = HX * HY;
static_assert(TX * TY == kKBlock, "one tile cell per thread");

// cell index of mesh position (gx, gy) with periodic wrap; -1 outside
__device__ __forceinline__ int halo_cell(const MeshDev& m, int gx, int gy) {
    if (gx < 0) {
        if (!m.periodic[0]) return -1;
        gx += m.n[0];
    } else if (gx >= m.n[0]) {
        if (!m.periodic[0]) return -1;
        gx -= m.n[0];
    }
    if (gy < 0) {
        if (!m.periodic[1]) return -1;
        gy += m.n[1];
    } else if (gy >= m.n[1]) {
        if (!m.periodic[1]) return -1;
        gy -= m.n[1];
    }
    return gx + m.n[0] * gy;
}

// Row of cell c (2D): the 9 planes, or (CF: the set's own FP64 operator,
// whose slots keep the weights of known value neighbours, the operands being
// zero there) the 8 off-centre planes, complete_row9 then forming the centre
// as minus their sum in slot order (the sum the weight build forms).
template <bool NT, bool CF, typename TA>
__device__ __forceinline__ void load_row9(const TA* __restrict__ A, size_t mps, int c, TA (&a)[9]) {
    static_assert(!CF || sizeof(TA) == sizeof(double), "centre formed for FP64 matrices only");
#pragma unroll
    for (int s = 0; s < 9; ++s) a[s] = (CF && s == 4) ? TA(0) : ld_mat<NT>(A + (size_t)s * mps + c);
}

template <bool CF, typename TA>
__device__ __forceinline__ void complete_row9(TA (&a)[9]) {
    if constexpr (CF) {
        TA sum = 0;
#pragma unroll
        for (int s = 0; s < 9; ++s)
            if (s != 4) sum += a[s];
        a[4] = -sum;
    }
}

template <bool NT, bool CF, typename T, typename TA>
__device__ __forceinline__ T stencil_lds(const TA* __restrict__ A, size_t mps, int c, const T* lds, int lx, int ly) {
    T acc = 0;
    if constexpr (CF) {
        TA a[9];
        load_row9<NT, true>(A, mps, c, a);
        complete_row9<true>(a);
#pragma unroll
        for (int s = 0; s < 9; ++s) acc += (T)a[s] * lds[(ly + s / 3) * HX + (lx + s % 3)];
    } else if constexpr (sizeof(TA) < sizeof(double)) {
        // FP32-stored matrix in difference form (centre slot = row sum)
        const T xc = lds[(ly + 1) * HX + lx + 1];
#pragma unroll
        for (int s = 0; s < 9; ++s) {
            const T a = (T)ld_mat<NT>(A + (size_t)s * mps + c);
            acc += s == 4 ? a * xc : a * (lds[(ly + s / 3) * HX + (lx + s % 3)] - xc);
        }
    } else {
#pragma unroll
        for (int s = 0; s < 9; ++s) acc += (T)ld_mat<NT>(A + (size_t)s * mps + c) * lds[(ly + s / 3) * HX + (lx + s % 3)];
    }
    return acc;
}

// Tiles of a block: a contiguous run [first, first + count) of the row-major
// tile order, so consecutive tiles of a block share halo rows and the blocks
// an XCD receives cover one contiguous band of the mesh.  Each block walks
// its run from a different starting tile (rotated by 13 tiles per block):
// when runs are whole rows of tiles, blocks that all started at the same
// column would read addresses a power of two apart at the same time, which
// the HBM channel interleave maps onto the same channels.
struct TileRun {
    int first, count, rot;
};

__device__ __forceinline__ TileRun tiles_of(const KBufs& K) {
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int first = lb * K.tpb;
    int count = K.ntiles - first;
    count = count < 0 ? 0 : (count > K.tpb ? K.tpb : count);
    return TileRun{first, count, count > 1 ? (lb * 13) % count : 0};
}

// The k-th tile a block processes (0 <= k < count).
__device__ __forceinline__ int run_tile(const TileRun& r, int k) {
    const int q = k + r.rot;
    return r.first + (q >= r.count ? q - r.count : q);
}

__device__ __forceinline__ void tile_origin(const KBufs& K, int tile, int& tx0, int& ty0) {
    tx0 = (tile % K.ntx) * TX;
    ty0 = (tile / K.ntx) * TY;
}

template <typename T, typename TA, bool NT, bool CF>
__global__ __launch_bounds__(kKBlock) void k_t2_init(MeshDev m, KVec<T, TA> V, KBufs K) {
    __shared__ T xl[NH];
    const T* __restrict__ xp = V.x;
    const T* __restrict__ bp = V.b;
    const TA* __restrict__ A = V.A;
    T* __restrict__ sp = V.s;
    T* __restrict__ rh = V.rhat;
    const TileRun run = tiles_of(K);
    double a0 = 0.0, a1 = 0.0;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    for (int k = 0; k < run.count; ++k) {
        int tx0, ty0;
        tile_origin(K, run_tile(run, k), tx0, ty0);
        for (int e = threadIdx.x; e < NH; e += kKBlock) {
            const int j = halo_cell(m, tx0 + e % HX - 1, ty0 + e / HX - 1);
            xl[e] = j >= 0 ? xp[j] : T(0);
        }
        __syncthreads();
        const int gx = tx0 + lx, gy = ty0 + ly;
        if (gx < m.n[0] && gy < m.n[1]) {
            const int c = gx + m.n[0] * gy;
            const T ax = stencil_lds<NT, CF, T, TA>(A, m.mps, c, xl, lx, ly);
            const T bc = bp[c];
            const T r = bc - ax;
            sp[c] = r;
            rh[c] = r;
            a0 += (double)r * (double)r;
            a1 += (double)bc * (double)bc;
        }
        __syncthreads();
    }
    double v[2] = {a0, a1};
    write_partials<2>(v, K.part[0], K);
}

// LDS-only block barrier: waits for this wave's LDS traffic, not for its
// outstanding global loads (the stage kernels never read in one thread what
// another thread of the block wrote to global memory in the same kernel).
__device__ __forceinline__ void sync_lds() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// block_sum_all with LDS-only barriers (same arithmetic and order)
template <int NQ>
__device__ __forceinline__ void block_sum_lds(double (&v)[NQ]) {
    __shared__ double lds[NQ][kKBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double sq = wave_sum(v[q]);
        if (lane == 0) lds[q][wid] = sq;
    }
    sync_lds();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double sq = 0.0;
#pragma unroll
        for (int w = 0; w < kKBlock / 64; ++w) sq += lds[q][w];
        v[q] = sq;
    }
    sync_lds();
}

// This block's partials of a stage (one per thread; kKGrid <= kKBlock).
template <int NQ>
__device__ __forceinline__ void load_partials(const double* __restrict__ part, const KBufs& K, double (&q)[NQ]) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) q[k] = (int)threadIdx.x < K.nblk ? part[k * K.cap + threadIdx.x] : 0.0;
}

template <int NQ>
__device__ __forceinline__ void store_partials(double (&v)[NQ], double* part, const KBufs& K) {
    block_sum_lds<NQ>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[q * K.cap + blockIdx.x] = v[q];
    }
}

// Operands of one halo element of a P-stage tile.
template <typename T>
struct HaloP {
    int j;
    bool own;
    T s, t, p, v, x;
};

template <typename T, int MODE>
__device__ __forceinline__ void load_halo_p(const MeshDev& m, int tx0, int ty0, int e, const T* __restrict__ sp, const T* __restrict__ tp,
                                            const T* __restrict__ po, const T* __restrict__ vo,
                                            const T* __restrict__ rp, const T* __restrict__ xp, HaloP<T>& h) {
    const int hx = e % HX, hy = e / HX;
    const int gx = tx0 + hx - 1, gy = ty0 + hy - 1;
    h.j = halo_cell(m, gx, gy);
    h.own = hx >= 1 && hx <= TX && hy >= 1 && hy <= TY && gx < m.n[0] && gy < m.n[1];
    if (h.j < 0) return;
    if (MODE == P_FIRST) {
        h.s = sp[h.j];
    } else if (MODE == P_RESUME) {
        h.s = rp[h.j];               // the replaced residual
        h.p = po[h.j];
        h.v = vo[h.j];
    } else {
        h.s = sp[h.j];
        h.t = tp[h.j];
        h.p = po[h.j];
        h.v = vo[h.j];
        if (h.own) h.x = xp[h.j];
    }
}

// P-stage (2D).  Every load the first tile needs (state, the S-stage
// partials, the halo operands, the matrix row, rhat) is issued before the
// block reduction, and the next tile's halo operands while the current tile
// is formed, so that the memory latencies overlap.
template <typename T, typename TA, int MODE, bool NT, bool CF>
__global__ __launch_bounds__(kKBlock) void k_t2_P(MeshDev m, KVec<T, TA> V, int par, KBufs K) {
    __shared__ T pl[NH];
    const KState* __restrict__ in = K.st[2];
    const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
    const T* __restrict__ sp = V.s;
    const T* __restrict__ tp = V.t;
    const T* __restrict__ po = V.p[par];
    const T* __restrict__ vo = V.v[par];
    const T* __restrict__ rh = V.rhat;
    const TA* __restrict__ A = V.A;
    T* __restrict__ pn = V.p[par ^ 1];
    T* __restrict__ vn = V.v[par ^ 1];
    T* __restrict__ rp = V.r;
    T* __restrict__ xp = V.x;
    const TileRun run = tiles_of(K);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int e0 = threadIdx.x, e1 = threadIdx.x + kKBlock;
    const bool has1 = e1 < NH;
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    if (MODE == P_NORMAL) load_partials<4>(K.part[2], K, q);   // t.s, t.t, rhat.s, rhat.t
    HaloP<T> h0{-1, false, 0, 0, 0, 0, 0}, h1{-1, false, 0, 0, 0, 0, 0};
    int tx0n = 0, ty0n = 0, c = -1;
    TA a[9];
    T rhc = 0;
    if (run.count > 0) {
        tile_origin(K, run_tile(run, 0), tx0n, ty0n);
        load_halo_p<T, MODE>(m, tx0n, ty0n, e0, sp, tp, po, vo, rp, xp, h0);
        if (has1) load_halo_p<T, MODE>(m, tx0n, ty0n, e1, sp, tp, po, vo, rp, xp, h1);
    }
    if (in->done) {
        if (leader) *K.st[1] = *in;
        return;
    }
    double omega = 1.0, beta = 0.0, rho_new = in->rho;
    bool ok = true;
    if (MODE == P_NORMAL) {
        block_sum_lds<4>(q);
        omega = q[0] / q[1];
        rho_new = q[2] - omega * q[3];
        beta = (rho_new / in->rho) * (in->alpha / omega);
        ok = q[1] > 0.0 && isfinite(omega) && isfinite(beta) && omega != 0.0 && fabs(rho_new) >= 1e-30 * in->rr0;
    } else if (MODE == P_RESUME) {
        omega = in->omega;
        rho_new = in->rho_res;
        beta = (rho_new / in->rho_prev) * (in->alpha / omega);
        ok = isfinite(beta) && omega != 0.0 && fabs(rho_new) >= 1e-30 * in->rr0;
    }
    if (!ok) {
        if (leader) {
            *K.st[1] = *in;
            K.st[1]->done = 2;
        }
        return;
    }
    const T ta = (T)in->alpha, tw = (T)omega, tb = (T)beta;
    double a0 = 0.0, a1 = 0.0;
    for (int k = 0; k < run.count; ++k) {
        const int tx0 = tx0n, ty0 = ty0n;
        {
            const int gxo = tx0 + lx, gyo = ty0 + ly;
            c = (gxo < m.n[0] && gyo < m.n[1]) ? gxo + m.n[0] * gyo : -1;
            if (c >= 0) {
                load_row9<NT, CF>(A, m.mps, c, a);
                rhc = rh[c];
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const HaloP<T>& h = u == 0 ? h0 : h1;
            const int e = u == 0 ? e0 : e1;
            if (u == 1 && !has1) break;
            T pv = 0;
            if (h.j >= 0) {
                T rj;
                if (MODE == P_FIRST) {
                    rj = h.s;
                    pv = rj;
                } else if (MODE == P_RESUME) {
                    rj = h.s;
                    pv = rj + tb * (h.p - tw * h.v);
                } else {
                    rj = h.s - tw * h.t;
                    pv = rj + tb * (h.p - tw * h.v);
                }
                if (h.own) {
                    if (MODE != P_RESUME) rp[h.j] = rj;
                    pn[h.j] = pv;
                    if (MODE == P_NORMAL) xp[h.j] = h.x + ta * h.p + tw * h.s;
                    a1 += (double)rj * (double)rj;
                }
            }
            pl[e] = pv;
        }
        if (k + 1 < run.count) {
            tile_origin(K, run_tile(run, k + 1), tx0n, ty0n);
            load_halo_p<T, MODE>(m, tx0n, ty0n, e0, sp, tp, po, vo, rp, xp, h0);
            if (has1) load_halo_p<T, MODE>(m, tx0n, ty0n, e1, sp, tp, po, vo, rp, xp, h1);
        }
        sync_lds();
        if (c >= 0) {
            T av = 0;
            complete_row9<CF>(a);
            if constexpr (sizeof(TA) < sizeof(double)) {
                const T xc = pl[(ly + 1) * HX + lx + 1];
#pragma unroll
                for (int s = 0; s < 9; ++s)
                    av += s == 4 ? (T)a[s] * xc : (T)a[s] * (pl[(ly + s / 3) * HX + (lx + s % 3)] - xc);
            } else {
#pragma unroll
                for (int s = 0; s < 9; ++s) av += (T)a[s] * pl[(ly + s / 3) * HX + (lx + s % 3)];
            }
            vn[c] = av;
            a0 += (double)rhc * (double)av;
        }
        sync_lds();
    }
    double acc[2] = {a0, a1};
    store_partials<2>(acc, K.part[1], K);
    if (leader) {
        *K.st[1] = *in;
        K.st[1]->rho_prev = in->rho;
        K.st[1]->rho = rho_new;
        K.st[1]->omega = omega;
    }
}

// S-stage (2D), load-first like the P-stage.
template <typename T, typename TA, bool NT, bool CF>
__global__ __launch_bounds__(kKBlock) void k_t2_S(MeshDev m, KVec<T, TA> V, int par, KBufs K) {
    __shared__ T sl[NH];
    const KState* __restrict__ in = K.st[1];
    const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
    const T* __restrict__ rp = V.r;
    const T* __restrict__ vn = V.v[par ^ 1];
    const T* __restrict__ rh = V.rhat;
    const TA* __restrict__ A = V.A;
    T* __restrict__ sp = V.s;
    T* __restrict__ tp = V.t;
    const TileRun run = tiles_of(K);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int e0 = threadIdx.x, e1 = threadIdx.x + kKBlock;
    const bool has1 = e1 < NH;
    double tot[2];
    load_partials<2>(K.part[1], K, tot);           // rhat.v, r.r
    int j0 = -1, j1 = -1, tx0n = 0, ty0n = 0, c = -1;
    T r0 = 0, v0 = 0, r1 = 0, v1 = 0, rhc = 0;
    TA a[9];
    if (run.count > 0) {
        tile_origin(K, run_tile(run, 0), tx0n, ty0n);
        j0 = halo_cell(m, tx0n + e0 % HX - 1, ty0n + e0 / HX - 1);
        if (j0 >= 0) {
            r0 = rp[j0];
            v0 = vn[j0];
        }
        if (has1) {
            j1 = halo_cell(m, tx0n + e1 % HX - 1, ty0n + e1 / HX - 1);
            if (j1 >= 0) {
                r1 = rp[j1];
                v1 = vn[j1];
            }
        }
        const int gxo = tx0n + lx, gyo = ty0n + ly;
        c = (gxo < m.n[0] && gyo < m.n[1]) ? gxo + m.n[0] * gyo : -1;
        if (c >= 0) {
            load_row9<NT, CF>(A, m.mps, c, a);
            rhc = rh[c];
        }
    }
    if (in->done) {
        if (leader) *K.st[2] = *in;
        return;
    }
    block_sum_lds<2>(tot);
    const double alpha = in->rho / tot[0];
    int done = 0;
    if (tot[1] <= fmax(in->tol2 * in->bb, in->delta2 * in->rr_max)) {
        done = 1;                                // x already holds the iterate of this residual
    } else if (!(tot[0] != 0.0) || !isfinite(alpha)) {
        done = 2;
    }
    if (done) {
        if (leader) {
            *K.st[2] = *in;
            K.st[2]->rv = tot[0];
            K.st[2]->rr = tot[1];
            K.st[2]->done = done;
        }
        return;
    }
    const T ta = (T)alpha;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int k = 0; k < run.count; ++k) {
        const int tx0 = tx0n, ty0 = ty0n;
        if (k > 0) {
            const int gxo = tx0 + lx, gyo = ty0 + ly;
            c = (gxo < m.n[0] && gyo < m.n[1]) ? gxo + m.n[0] * gyo : -1;
            if (c >= 0) {
                load_row9<NT, CF>(A, m.mps, c, a);
                rhc = rh[c];
            }
        }
        {
            const int hx = e0 % HX, hy = e0 / HX, gx = tx0 + hx - 1, gy = ty0 + hy - 1;
            T sv = 0;
            if (j0 >= 0) {
                sv = r0 - ta * v0;
                if (hx >= 1 && hx <= TX && hy >= 1 && hy <= TY && gx < m.n[0] && gy < m.n[1]) sp[j0] = sv;
            }
            sl[e0] = sv;
        }
        if (has1) {
            const int hx = e1 % HX, hy = e1 / HX, gx = tx0 + hx - 1, gy = ty0 + hy - 1;
            T sv = 0;
            if (j1 >= 0) {
                sv = r1 - ta * v1;
                if (hx >= 1 && hx <= TX && hy >= 1 && hy <= TY && gx < m.n[0] && gy < m.n[1]) sp[j1] = sv;
            }
            sl[e1] = sv;
        }
        if (k + 1 < run.count) {
            tile_origin(K, run_tile(run, k + 1), tx0n, ty0n);
            j0 = halo_cell(m, tx0n + e0 % HX - 1, ty0n + e0 / HX - 1);
            if (j0 >= 0) {
                r0 = rp[j0];
                v0 = vn[j0];
            }
            if (has1) {
                j1 = halo_cell(m, tx0n + e1 % HX - 1, ty0n + e1 / HX - 1);
                if (j1 >= 0) {
                    r1 = rp[j1];
                    v1 = vn[j1];
                }
            }
        }
        sync_lds();
        if (c >= 0) {
            T tcv = 0;
            complete_row9<CF>(a);
            if constexpr (sizeof(TA) < sizeof(double)) {
                const T xc = sl[(ly + 1) * HX + lx + 1];
#pragma unroll
                for (int s = 0; s < 9; ++s)
                    tcv += s == 4 ? (T)a[s] * xc : (T)a[s] * (sl[(ly + s / 3) * HX + (lx + s % 3)] - xc);
            } else {
#pragma unroll
                for (int s = 0; s < 9; ++s) tcv += (T)a[s] * sl[(ly + s / 3) * HX + (lx + s % 3)];
            }
            const T sc = sl[(ly + 1) * HX + lx + 1];
            tp[c] = tcv;
            const double r = (double)rhc;
            a0 += (double)tcv * (double)sc;
            a1 += (double)tcv * (double)tcv;
            a2 += r * (double)sc;
            a3 += r * (double)tcv;
        }
        sync_lds();
    }
    double acc[4] = {a0, a1, a2, a3};
    store_partials<4>(acc, K.part[2], K);
    if (leader) {
        *K.st[2] = *in;
        K.st[2]->rv = tot[0];
        K.st[2]->rr = tot[1];
        K.st[2]->rr_max = fmax(in->rr_max, tot[1]);
        K.st[2]->alpha = alpha;
        K.st[2]->iter = in->iter + 1;
    }
}

// ---------------------------------------------------------------------------
// 3D stage kernels (2.5D).  A block of 512 threads owns a 64 x 8 column of
// cells and marches it over K.tz planes (a brick).  The operand of the
// 27-point product is formed once per plane of the brick plus one halo
// plane below and above, into a ring of three (66 x 10) planes in LDS, so the
// product reads LDS only; the owner of a cell does its element-wise updates
// when its plane is formed.
// ---------------------------------------------------------------------------

// cell index of mesh position (gx, gy, gz) with periodic wrap; -1 outside
__device__ __forceinline__ int halo_cell3(const MeshDev& m, int gx, int gy, int gz) {
    if (gz < 0) {
        if (!m.periodic[2]) return -1;
        gz += m.n[2];
    } else if (gz >= m.n[2]) {
        if (!m.periodic[2]) return -1;
        gz -= m.n[2];
    }
    const int j = halo_cell(m, gx, gy);
    return j < 0 ? -1 : j + m.n[0] * m.n[1] * gz;
}

__device__ __forceinline__ void brick_origin(const KBufs& K, int brick, int& tx0, int& ty0, int& tz0) {
    tx0 = (brick % K.ntx) * TX;
    ty0 = ((brick / K.ntx) % K.nty) * TY;
    tz0 = (brick / (K.ntx * K.nty)) * K.tz;
}

// Matrix rows of the 3D stage kernels.  Rows of cells that are not unknown
// are 27 zeros (+0.0) in every FP64 matrix, and their 26 off-centre planes
// are not read; what tells them apart is fetched one plane ahead, so the
// test adds no latency:
// - CF (the set's own FP64 operator): the cell's unknown flag.  The row's
//   slots also keep the weights of its known value neighbours (operands are
//   zero there), so the centre is minus the sum of the other 26 slots, in
//   slot order (the sum the weight build forms and stores), and the centre
//   plane is not read either.
// - other FP64 matrices (the Jacobi-scaled copy): the centre.  The centre of
//   an unknown row is never +0.0: it is -sum of the row's value weights, a
//   sum that starts at +0.0 and so is never -0.0, times its reciprocal
//   (about 1), times 1 (not finite), or the -0.0 kept.
// - FP32 matrices (difference form: the centre holds the row sum, zero for
//   most rows): every plane is read.
template <typename TA>
struct RowSkip {
    static constexpr bool on = sizeof(TA) == sizeof(double);
};

template <typename TA, bool NT, bool CF>
struct RowLoad {
    static_assert(!CF || sizeof(TA) == sizeof(double), "centre formed for FP64 matrices only");
    const TA* __restrict__ A;
    size_t mps;
    const uint8_t* __restrict__ unk;
    TA cen;          // centre of the next row (FP64, not CF)
    uint8_t u;       // unknown flag of the next row (CF)

    // row of cell c into a; false for a row of zeros
    __device__ __forceinline__ bool load(int c, TA (&a)[27]) {
        bool nz = true;
        if constexpr (CF)
            nz = u != 0;
        else if constexpr (RowSkip<TA>::on)
            nz = __double_as_longlong((double)cen) != 0;
        if (!nz) {
#pragma unroll
            for (int s = 0; s < 27; ++s) a[s] = TA(0);
            return false;
        }
#pragma unroll
        for (int s = 0; s < 27; ++s) {
            if (s == 13)
                a[s] = CF ? TA(0) : (RowSkip<TA>::on ? cen : ld_mat<NT>(A + (size_t)s * mps + c));
            else
                a[s] = ld_mat<NT>(A + (size_t)s * mps + c);
        }
        return true;
    }
    // fetches what the row of cell cn is told apart by
    __device__ __forceinline__ void ahead(int cn) {
        if constexpr (CF)
            u = unk[cn];
        else if constexpr (RowSkip<TA>::on)
            cen = ld_mat<NT>(A + (size_t)13 * mps + cn);
    }
    // completes a loaded row before its product
    __device__ __forceinline__ void complete(TA (&a)[27]) {
        if constexpr (CF) {
            TA sum = 0;
#pragma unroll
            for (int s = 0; s < 27; ++s)
                if (s != 13) sum += a[s];
            a[13] = -sum;
        }
    }
};

// 27-point product of a preloaded row with the ring planes (slots of planes
// z-1, z, z+1).
template <typename T, typename TA>
__device__ __forceinline__ T stencil3_lds(const TA (&a)[27], const T (*ring)[NH], int s0, int s1, int s2, int lx,
                                          int ly) {
    const int sl[3] = {s0, s1, s2};
    T acc = 0;
    if constexpr (sizeof(TA) < sizeof(double)) {
        const T xc = ring[s1][(ly + 1) * HX + lx + 1];
#pragma unroll
        for (int s = 0; s < 27; ++s) {
            const T v = ring[sl[s / 9]][(ly + (s / 3) % 3) * HX + (lx + s % 3)];
            acc += s == 13 ? (T)a[s] * xc : (T)a[s] * (v - xc);
        }
    } else {
#pragma unroll
        for (int s = 0; s < 27; ++s) acc += (T)a[s] * ring[sl[s / 9]][(ly + (s / 3) % 3) * HX + (lx + s % 3)];
    }
    return acc;
}

// Marches the bricks of this block: form(gz, slot, own_plane) fills a ring
// slot with the operand of plane gz (doing the owners' updates when
// own_plane); pre(c, cn) issues the loads of output cell c (matrix row)
// before the next plane is formed, so that they overlap, and those that the
// row of cell cn (the next plane of the brick, -1 after the last) depends
// on; pre(-1, c) at the start of a brick fetches them for its first plane;
// out(c, s0, s1, s2) consumes the product at cell c.  Barriers are LDS-only.
template <typename T, typename FORM, typename PRE, typename OUT>
__device__ __forceinline__ void march_bricks(const MeshDev& m, const KBufs& K, FORM form, PRE pre, OUT out) {
    const TileRun run = tiles_of(K);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int n01 = m.n[0] * m.n[1];
    for (int k = 0; k < run.count; ++k) {
        int tx0, ty0, tz0;
        brick_origin(K, run_tile(run, k), tx0, ty0, tz0);
        const int tz1 = min(tz0 + K.tz, m.n[2]);
        const int gx = tx0 + lx, gy = ty0 + ly;
        const bool inside = gx < m.n[0] && gy < m.n[1];
        if (inside) pre(-1, gx + m.n[0] * (gy + m.n[1] * tz0));
        form(tx0, ty0, tz0 - 1, 0, false);
        form(tx0, ty0, tz0, 1, true);
        for (int z = tz0; z < tz1; ++z) {
            const int c = gx + m.n[0] * (gy + m.n[1] * z);
            if (inside) pre(c, z + 1 < tz1 ? c + n01 : -1);
            form(tx0, ty0, z + 1, (z - tz0 + 2) % 3, z + 1 < tz1);
            sync_lds();
            if (inside) out(c, (z - tz0) % 3, (z - tz0 + 1) % 3, (z - tz0 + 2) % 3);
            sync_lds();
        }
    }
}

template <typename T, typename TA, bool NT, bool CF>
__global__ __launch_bounds__(kKBlock) void k_t3_init(MeshDev m, KVec<T, TA> V, KBufs K) {
    __shared__ T ring[3][NH];
    const T* __restrict__ xp = V.x;
    const T* __restrict__ bp = V.b;
    const TA* __restrict__ A = V.A;
    T* __restrict__ sp = V.s;
    T* __restrict__ rh = V.rhat;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    double a0 = 0.0, a1 = 0.0;
    TA a[27];
    RowLoad<TA, NT, CF> rows{A, m.mps, V.unk, TA(0), 0};
    T bcv = 0;
    march_bricks<T>(
        m, K,
        [&](int tx0, int ty0, int gz, int slot, bool) {
            for (int e = threadIdx.x; e < NH; e += kKBlock) {
                const int j = halo_cell3(m, tx0 + e % HX - 1, ty0 + e / HX - 1, gz);
                ring[slot][e] = j >= 0 ? xp[j] : T(0);
            }
        },
        [&](int c, int cn) {
            if (c >= 0) {
                rows.load(c, a);
                bcv = bp[c];
            }
            if (cn >= 0) rows.ahead(cn);
        },
        [&](int c, int s0, int s1, int s2) {
            rows.complete(a);
            const T ax = stencil3_lds<T, TA>(a, ring, s0, s1, s2, lx, ly);
            const T bc = bcv;
            const T r = bc - ax;
            sp[c] = r;
            rh[c] = r;
            a0 += (double)r * (double)r;
            a1 += (double)bc * (double)bc;
        });
    double v[2] = {a0, a1};
    write_partials<2>(v, K.part[0], K);
}

template <typename T, typename TA, int MODE, bool NT, bool CF>
__global__ __launch_bounds__(kKBlock) void k_t3_P(MeshDev m, KVec<T, TA> V, int par, KBufs K) {
    __shared__ T ring[3][NH];
    const KState* __restrict__ in = K.st[2];
    const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
    if (in->done) {
        if (leader) *K.st[1] = *in;
        return;
    }
    double omega, beta, rho_new;
    if (!p_scalars<MODE>(in, K, leader, omega, beta, rho_new)) return;
    const T ta = (T)in->alpha, tw = (T)omega, tb = (T)beta;
    const T* __restrict__ sp = V.s;
    const T* __restrict__ tp = V.t;
    const T* __restrict__ po = V.p[par];
    const T* __restrict__ vo = V.v[par];
    const T* __restrict__ rh = V.rhat;
    const TA* __restrict__ A = V.A;
    T* __restrict__ pn = V.p[par ^ 1];
    T* __restrict__ vn = V.v[par ^ 1];
    T* __restrict__ rp = V.r;
    T* __restrict__ xp = V.x;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    double a0 = 0.0, a1 = 0.0;
    TA a[27];
    RowLoad<TA, NT, CF> rows{A, m.mps, V.unk, TA(0), 0};
    T rhc = 0;
    march_bricks<T>(
        m, K,
        [&](int tx0, int ty0, int gz, int slot, bool own_plane) {
            for (int e = threadIdx.x; e < NH; e += kKBlock) {
                const int hx = e % HX, hy = e / HX;
                const int gx = tx0 + hx - 1, gy = ty0 + hy - 1;
                const int j = halo_cell3(m, gx, gy, gz);
                T pv = 0;
                if (j >= 0) {
                    T rj, sj = 0, poj = 0;
                    if (MODE == P_FIRST) {
                        rj = sp[j];
                        pv = rj;
                    } else if (MODE == P_RESUME) {
                        rj = rp[j];
                        poj = po[j];
                        pv = rj + tb * (poj - tw * vo[j]);
                    } else {
                        sj = sp[j];
                        const T tj = tp[j];
                        poj = po[j];
                        const T voj = vo[j];
                        rj = sj - tw * tj;
                        pv = rj + tb * (poj - tw * voj);
                    }
                    if (own_plane && hx >= 1 && hx <= TX && hy >= 1 && hy <= TY && gx < m.n[0] && gy < m.n[1]) {
                        if (MODE != P_RESUME) rp[j] = rj;
                        pn[j] = pv;
                        if (MODE == P_NORMAL) xp[j] = xp[j] + ta * poj + tw * sj;
                        a1 += (double)rj * (double)rj;
                    }
                }
                ring[slot][e] = pv;
            }
        },
        [&](int c, int cn) {
            if (c >= 0) {
                // r-hat is +0.0 wherever the row is zero
                rhc = rows.load(c, a) ? rh[c] : T(0);
            }
            if (cn >= 0) rows.ahead(cn);
        },
        [&](int c, int s0, int s1, int s2) {
            rows.complete(a);
            const T av = stencil3_lds<T, TA>(a, ring, s0, s1, s2, lx, ly);
            vn[c] = av;
            a0 += (double)rhc * (double)av;
        });
    double acc[2] = {a0, a1};
    write_partials<2>(acc, K.part[1], K);
    if (leader) {
        *K.st[1] = *in;
        K.st[1]->rho_prev = in->rho;
        K.st[1]->rho = rho_new;
        K.st[1]->omega = omega;
    }
}

template <typename T, typename TA, bool NT, bool CF>
__global__ __launch_bounds__(kKBlock) void k_t3_S(MeshDev m, KVec<T, TA> V, int par, KBufs K) {
    __shared__ T ring[3][NH];
    const KState* __restrict__ in = K.st[1];
    const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
    if (in->done) {
        if (leader) *K.st[2] = *in;
        return;
    }
    double tot[2];
    reduce_partials<2>(K.part[1], K, tot);       // rhat.v, r.r
    const double alpha = in->rho / tot[0];
    int done = 0;
    if (tot[1] <= fmax(in->tol2 * in->bb, in->delta2 * in->rr_max)) {
        done = 1;
    } else if (!(tot[0] != 0.0) || !isfinite(alpha)) {
        done = 2;
    }
    if (done) {
        if (leader) {
            *K.st[2] = *in;
            K.st[2]->rv = tot[0];
            K.st[2]->rr = tot[1];
            K.st[2]->done = done;
        }
        return;
    }
    const T ta = (T)alpha;
    const T* __restrict__ rp = V.r;
    const T* __restrict__ vn = V.v[par ^ 1];
    const T* __restrict__ rh = V.rhat;
    const TA* __restrict__ A = V.A;
    T* __restrict__ sp = V.s;
    T* __restrict__ tp = V.t;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    TA a[27];
    RowLoad<TA, NT, CF> rows{A, m.mps, V.unk, TA(0), 0};
    T rhc = 0;
    march_bricks<T>(
        m, K,
        [&](int tx0, int ty0, int gz, int slot, bool own_plane) {
            for (int e = threadIdx.x; e < NH; e += kKBlock) {
                const int hx = e % HX, hy = e / HX;
                const int gx = tx0 + hx - 1, gy = ty0 + hy - 1;
                const int j = halo_cell3(m, gx, gy, gz);
                T sv = 0;
                if (j >= 0) {
                    sv = rp[j] - ta * vn[j];
                    if (own_plane && hx >= 1 && hx <= TX && hy >= 1 && hy <= TY && gx < m.n[0] && gy < m.n[1])
                        sp[j] = sv;
                }
                ring[slot][e] = sv;
            }
        },
        [&](int c, int cn) {
            if (c >= 0) {
                // r-hat is +0.0 wherever the row is zero
                rhc = rows.load(c, a) ? rh[c] : T(0);
            }
            if (cn >= 0) rows.ahead(cn);
        },
        [&](int c, int s0, int s1, int s2) {
            rows.complete(a);
            const T tcv = stencil3_lds<T, TA>(a, ring, s0, s1, s2, lx, ly);
            const T sc = ring[s1][(ly + 1) * HX + lx + 1];
            tp[c] = tcv;
            const double r = (double)rhc;
            a0 += (double)tcv * (double)sc;
            a1 += (double)tcv * (double)tcv;
            a2 += r * (double)sc;
            a3 += r * (double)tcv;
        });
    double acc[4] = {a0, a1, a2, a3};
    write_partials<4>(acc, K.part[2], K);
    if (leader) {
        *K.st[2] = *in;
        K.st[2]->rv = tot[0];
        K.st[2]->rr = tot[1];
        K.st[2]->rr_max = fmax(in->rr_max, tot[1]);
        K.st[2]->alpha = alpha;
        K.st[2]->iter = in->iter + 1;
    }
}

// b_eff of unknown row c: rhs - (Dirichlet columns) g - (Neumann rows) f.
// Only known value neighbours (the row's kmask, from the weight build) and
// Neumann rows move to the right-hand side; they are visited in slot order,
// and the weights of the other slots are not read.
template <int DIM>
__device__ __forceinline__ double beff_row(const MeshDev& m, const SetDev& st, int c, const double* __restrict__ rhs,
                                           const double* __restrict__ g, const double* __restrict__ fneu,
                                           double irs2) {
    constexpr int NB = Dims<DIM>::NB, S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    double acc = rhs[c];
    const uint32_t km = st.kmask[c], nm = st.nmask[c];
    uint32_t todo = km | (fneu ? nm & ((1u << S) - 1u) & ~(1u << CEN) : 0u);
    if (todo) {
        int ijk[3];
        cell_ijk(m, c, ijk);
        while (todo) {
            const int s = __ffs(todo) - 1;
            todo &= todo - 1u;
            const bool known = ((km >> s) & 1u) != 0, n = fneu && ((nm >> s) & 1u);
            int j;
            double sh[3];
            neighbour_or_self<DIM>(m, ijk, s, c, j, sh);
            double ph[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) ph[q] = ld_stream(st.phi + ((size_t)q * (S + 1) + s) * m.mps + c);
            const double lc = diag2<DIM>(ph) * irs2;
            if (known) acc -= lc * g[j];
            if (n) acc -= lc * fneu[j];
        }
    }
    if (fneu && ((nm >> S) & 1u)) {
        double ph[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) ph[q] = ld_stream(st.phi + ((size_t)q * (S + 1) + S) * m.mps + c);
        acc -= diag2<DIM>(ph) * irs2 * fneu[c];
    }
    return acc;
}

// b_eff = rhs - (Dirichlet columns) g - (Neumann rows) f at unknown rows; x0.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_ppe_rhs(MeshDev m, SetDev st, const double* __restrict__ rhs,
                                                    const double* __restrict__ g, const double* __restrict__ fneu,
                                                    int caller_guess, double* __restrict__ beff,
                                                    double* __restrict__ x0, int* bad) {
    const double irs2 = 1.0 / (st.rs * st.rs);
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        if (!st.unknown[c]) {
            beff[c] = 0.0;
            x0[c] = 0.0;
            continue;
        }
        const double acc = beff_row<DIM>(m, st, c, rhs, g, fneu, irs2);
        if (!isfinite(acc)) atomicAdd(bad, 1);
        beff[c] = acc;
        x0[c] = caller_guess ? g[c] : 0.0;
    }
}

// r = b_eff - A x at unknown rows (0 elsewhere), with per-block partial sums
// of r.r and b_eff.b_eff.  x is zero at non-unknown cells.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_ppe_resid(MeshDev m, const double* __restrict__ A,
                                                      const uint8_t* __restrict__ unknown,
                                                      const double* __restrict__ beff, const double* __restrict__ x,
                                                      double* __restrict__ r, double* __restrict__ part) {
    __shared__ double lds[2][kBlock / 64];
    double rr = 0.0, bb = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (unknown[c]) {
            v = beff[c] - spmv_row<DIM, double, double>(m, A, c, [&](int j) { return x[j]; });
            rr += v * v;
            bb += beff[c] * beff[c];
        }
        r[c] = v;
    }
    double q[2] = {rr, bb};
    block_sum<2>(q, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = q[0];
        part[2 * blockIdx.x + 1] = q[1];
    }
}

// Sums the partials in block order (one block).
__global__ void k_resid_finish(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    __shared__ double lds[2][kBlock / 64];
    double q[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        q[0] += part[2 * b];
        q[1] += part[2 * b + 1];
    }
    block_sum<2>(q, lds);
    if (threadIdx.x == 0) {
        out[0] = sqrt(q[0]);
        out[1] = sqrt(q[1]);
    }
}

// r = b_eff - A p at unknown rows (0 elsewhere) in one pass, b_eff formed per
// row instead of staged: the same arithmetic, grid and per-thread order as
// k_ppe_rhs followed by k_ppe_resid (so the same bits), with the partials,
// the counter of non-finite rows and nothing else in the caller's scratch.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_ppe_resid_fused(MeshDev m, SetDev st, const double* __restrict__ rhs,
                                                            const double* __restrict__ p,
                                                            const double* __restrict__ fneu, double* __restrict__ r,
                                                            double* __restrict__ part, int* bad) {
    __shared__ double lds[2][kBlock / 64];
    const double irs2 = 1.0 / (st.rs * st.rs);
    double rr = 0.0, bb = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (st.unknown[c]) {
            const double be = beff_row<DIM>(m, st, c, rhs, p, fneu, irs2);
            if (!isfinite(be)) atomicAdd(bad, 1);
            v = be - spmv_row<DIM, double, double>(m, st.amat, c,
                                                   [&](int j) { return st.unknown[j] ? p[j] : 0.0; });
            rr += v * v;
            bb += be * be;
        }
        r[c] = v;
    }
    double q[2] = {rr, bb};
    block_sum<2>(q, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = q[0];
        part[2 * blockIdx.x + 1] = q[1];
    }
}

__global__ void k_zero_int(int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// Residual replacement (FP32-stored matrix, FP64 vectors): r = b_eff - A64 x
// with the FP64 matrix at unknown rows (0 elsewhere); partials of rhat.r and
// r.r.  Launched with the stage grid so that the partials match its
// reduction.
template <int DIM>
__global__ __launch_bounds__(kKBlock) void k_true_replace(MeshDev m, const double* __restrict__ A64,
                                                          const uint8_t* __restrict__ unknown,
                                                          const double* __restrict__ beff, KVec<double, float> V,
                                                          KBufs K) {
    const double* __restrict__ x = V.x;
    const double* __restrict__ rh = V.rhat;
    double* __restrict__ r = V.r;
    double a0 = 0.0, a1 = 0.0;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    for (int c = lb * kKBlock + threadIdx.x; c < m.Nc; c += gridDim.x * kKBlock) {
        double v = 0.0;
        if (unknown[c]) v = beff[c] - spmv_row<DIM, double, double>(m, A64, c, [&](int j) { return x[j]; });
        r[c] = v;
        a0 += rh[c] * v;
        a1 += v * v;
    }
    double acc[2] = {a0, a1};
    write_partials<2>(acc, K.part[0], K);
}

// One block: the state a resume P-stage reads; done = 1 when the replaced
// residual already meets the tolerance.
__global__ __launch_bounds__(kKBlock) void k_replace_finish(KBufs K, double tol2, double tol2_next, double delta2_next) {
    double tot[2];
    reduce_partials<2>(K.part[0], K, tot);
    if (threadIdx.x == 0) {
        KState* S = K.st[2];
        S->rho_res = tot[0];
        S->rr = tot[1];
        S->rr_max = tot[1];
        S->done = tot[1] <= tol2 * S->bb ? 1 : 0;
        S->tol2 = tol2_next;
        S->delta2 = delta2_next;
    }
}

// x := 0 (a zero right-hand side has the zero solution).
template <typename T>
__global__ void k_zero(int Nc, T* __restrict__ x) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x) x[c] = T(0);
}

// p := x at unknown cells.
__global__ void k_writeback(int Nc, const uint8_t* __restrict__ unknown, const double* __restrict__ x,
                            double* __restrict__ p) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x)
        if (unknown[c]) p[c] = x[c];
}

// Mixed precision helpers: b32 = r64 * scale; x32 = 0;  x64 += d32 / scale.
__global__ void k_to32(int Nc, const double* __restrict__ r, double scale, float* __restrict__ b32,
                       float* __restrict__ x32) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x) {
        b32[c] = (float)(r[c] * scale);
        x32[c] = 0.0f;
    }
}
__global__ void k_refine(int Nc, const float* __restrict__ d, double inv_scale, double* __restrict__ x) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x)
        x[c] = x[c] + (double)d[c] * inv_scale;
}

// Jacobi (diagonal) right preconditioning of Bi-CGSTAB (Sec. 3.3 names the
// solver; the preconditioner is the comparator of the learned guess).  With
// D = diag(A), Bi-CGSTAB on (A D^-1) y = b followed by x = D^-1 y performs the
// iterations of right-preconditioned Bi-CGSTAB (v = A D^-1 p, t = A D^-1 s)
// and its residual b - (A D^-1) y is b - A x, so the stopping rule is
// unchanged.  The column scaling is done once per solve.
//
// dinv := 1/diag at unknown rows (1 where the diagonal is zero or not
// finite, and at known rows); x := D x (the initial guess in y).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_jacobi_diag(MeshDev m, const double* __restrict__ A,
                                                        const uint8_t* __restrict__ unknown,
                                                        double* __restrict__ dinv, double* __restrict__ x) {
    constexpr int CEN = Dims<DIM>::CEN;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const double d = unknown[c] ? A[(size_t)CEN * m.mps + c] : 0.0;
        const bool ok = d != 0.0 && isfinite(d);
        dinv[c] = ok ? 1.0 / d : 1.0;
        if (ok) x[c] = x[c] * d;
    }
}

// J[s][c] = A[s][c] dinv[j(c, s)] (FP64; like A, it keeps the weights of
// known value neighbours, scaled by 1), and its FP32 copy over the unknown
// columns in difference form (centre slot = row sum of the scaled row), as
// the MLS build stores A.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_jacobi_matrix(MeshDev m, const double* __restrict__ A,
                                                          const uint8_t* __restrict__ unknown,
                                                          const double* __restrict__ dinv, double* __restrict__ J,
                                                          float* __restrict__ J32) {
    constexpr int S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    const size_t P = m.mps;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        int ijk[3];
        cell_ijk(m, c, ijk);
        double off_sum = 0.0, diag = 0.0;
        for (int s = 0; s < S; ++s) {
            const double a = A[(size_t)s * P + c];
            // a zero keeps its sign: the centre of an unknown row is never
            // +0.0, here as in A (the stage kernels skip rows whose centre is)
            double v = a == 0.0 ? a : 0.0;
            bool col = false;      // an unknown column
            int j;
            double sh[3];
            if (a != 0.0 && neighbour<DIM>(m, ijk, s, j, sh)) {
                v = a * dinv[j];
                col = unknown[j] != 0;
            }
            J[(size_t)s * P + c] = v;
            if (s == CEN) {
                diag = v;
            } else {
                const double v32 = col ? v : 0.0;
                J32[(size_t)s * P + c] = (float)v32;
                off_sum += v32;
            }
        }
        J32[(size_t)CEN * P + c] = (float)(diag + off_sum);
    }
}

// x := D^-1 y at unknown rows.
__global__ void k_jacobi_unscale(int Nc, const uint8_t* __restrict__ unknown, const double* __restrict__ dinv,
                                 double* __restrict__ x) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x)
        if (unknown[c]) x[c] = x[c] * dinv[c];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct GraphEntry {
    const void* A;
    int fp32;
    hipGraphExec_t exec;
};

struct KrylovWork {
    int Nc;
    KBufs kb64, kb32;      // partials and stage states of the FP64 and FP32 solves
    KState* host;          // pinned [2]
    hipEvent_t ev[2];
    hipEvent_t join;       // orders the solve stream after the caller's stream
    hipStream_t st;        // solve stream (default priority, owned)
    KVec<double> v64;
    KVec<float> v32;
    double* beff;
    float* b32;
    double* xsave;         // iterate before a refinement step
    double* dinv;          // [Nc] inverse diagonal (Jacobi)
    double* jac64;         // [S][mps] column-scaled matrix A D^-1 (Jacobi)
    float* jac32;          // [S][mps] its FP32 copy in difference form
    int* bad_host;         // pinned
    // replayed chunks of kGraphIters iterations (per operator and precision)
    static constexpr int kGraphIters = 16;
    static constexpr int kStallIters = 2000;   // see run_iterations
    static constexpr int kMaxGraphs = 16;
    GraphEntry graphs[kMaxGraphs];
    int ngraphs = 0;
    int use_graphs = 1;
    int grid_req = kKGrid;   // block count asked for (the shape clips it to the tiles)
    // optional timing of the stage kernels: start/stop events stamped by the
    // kernel dispatch itself (hipExtLaunchKernelGGL)
    int profile = 0;
    static constexpr int kProf = 4096;
    hipEvent_t pev[kProf][4];
    int pidx[kProf];       // global iteration index of the recorded launch pair
    int pa32[kProf];       // 1 when the recorded pair read the FP32 copy of the matrix
    int np = 0;
    double ms[2] = {0.0, 0.0};   // accumulated P, S milliseconds of working launches
    long long cnt[2] = {0, 0};
    double ms32[2] = {0.0, 0.0};   // the part of them that read the FP32 matrix
    long long cnt32[2] = {0, 0};
    MgWork* mg = nullptr;          // multigrid hierarchy (MCD_PRECOND_MG)
};

template <int DIM, typename T, typename TA, bool NT, bool CF>
static void enqueue_stages(const MeshDev& m, const KVec<T, TA>& V, const KBufs& K, int par, int mode, hipStream_t st,
                           hipEvent_t e0, hipEvent_t e1, hipEvent_t e2, hipEvent_t e3) {
    const dim3 G(K.nblk), B(kKBlock);
    if constexpr (DIM == 2) {
        if (mode == P_FIRST)
            hipExtLaunchKernelGGL((k_t2_P<T, TA, P_FIRST, NT, CF>), G, B, 0, st, e0, e1, 0, m, V, par, K);
        else if (mode == P_RESUME)
            hipExtLaunchKernelGGL((k_t2_P<T, TA, P_RESUME, NT, CF>), G, B, 0, st, e0, e1, 0, m, V, par, K);
        else
            hipExtLaunchKernelGGL((k_t2_P<T, TA, P_NORMAL, NT, CF>), G, B, 0, st, e0, e1, 0, m, V, par, K);
        hipExtLaunchKernelGGL((k_t2_S<T, TA, NT, CF>), G, B, 0, st, e2, e3, 0, m, V, par, K);
    } else {
        if (mode == P_FIRST)
            hipExtLaunchKernelGGL((k_t3_P<T, TA, P_FIRST, NT, CF>), G, B, 0, st, e0, e1, 0, m, V, par, K);
        else if (mode == P_RESUME)
            hipExtLaunchKernelGGL((k_t3_P<T, TA, P_RESUME, NT, CF>), G, B, 0, st, e0, e1, 0, m, V, par, K);
        else
            hipExtLaunchKernelGGL((k_t3_P<T, TA, P_NORMAL, NT, CF>), G, B, 0, st, e0, e1, 0, m, V, par, K);
        hipExtLaunchKernelGGL((k_t3_S<T, TA, NT, CF>), G, B, 0, st, e2, e3, 0, m, V, par, K);
    }
}

// Enqueues one Bi-CGSTAB iteration (P-stage in `mode`, then S-stage) with
// operand parity par.
template <int DIM, typename T, typename TA, bool NT>
static void enqueue_iteration_nt(const MeshDev& m, const KVec<T, TA>& V, const KBufs& K, int par, int mode,
                                 hipStream_t st, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2, hipEvent_t e3) {
    if constexpr (sizeof(TA) == sizeof(double)) {
        if (V.unk) {
            enqueue_stages<DIM, T, TA, NT, true>(m, V, K, par, mode, st, e0, e1, e2, e3);
            return;
        }
    }
    enqueue_stages<DIM, T, TA, NT, false>(m, V, K, par, mode, st, e0, e1, e2, e3);
}

template <int DIM, typename T, typename TA>
static void enqueue_iteration(const MeshDev& m, const KVec<T, TA>& V, const KBufs& K, int par, int mode,
                              hipStream_t st, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2, hipEvent_t e3) {
    if (K.nt)
        enqueue_iteration_nt<DIM, T, TA, true>(m, V, K, par, mode, st, e0, e1, e2, e3);
    else
        enqueue_iteration_nt<DIM, T, TA, false>(m, V, K, par, mode, st, e0, e1, e2, e3);
}

// Graph of kGraphIters non-first iterations starting at parity 1 (an even
// count, so every replay starts and ends at parity 1).
template <int DIM, typename T, typename TA>
static hipError_t chunk_graph(const MeshDev& m, KrylovWork& w, const KVec<T, TA>& V, const KBufs& K,
                              hipGraphExec_t* out) {
    // key: the matrix, the precision and whether the centre is formed
    const int fp32 = (sizeof(T) == 4 ? 1 : 0) | (V.unk ? 2 : 0);
    for (int i = 0; i < w.ngraphs; ++i)
        if (w.graphs[i].A == (const void*)V.A && w.graphs[i].fp32 == fp32) {
            *out = w.graphs[i].exec;
            return hipSuccess;
        }
    if (w.ngraphs == KrylovWork::kMaxGraphs) return hipErrorNotSupported;
    hipError_t e = hipStreamBeginCapture(w.st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    int par = 1;
    for (int q = 0; q < KrylovWork::kGraphIters; ++q) {
        enqueue_iteration<DIM, T, TA>(m, V, K, par, P_NORMAL, w.st, nullptr, nullptr, nullptr, nullptr);
        par ^= 1;
    }
    hipGraph_t g;
    if ((e = hipStreamEndCapture(w.st, &g)) != hipSuccess) return e;
    hipGraphExec_t ex;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    w.graphs[w.ngraphs++] = GraphEntry{(const void*)V.A, fp32, ex};
    *out = ex;
    return hipSuccess;
}

// Runs up to `budget` iterations; the first one's P-stage is in mode0 with
// parity par0 (the P-stage of iteration k always has parity k % 2).
template <int DIM, typename T, typename TA>
static hipError_t run_iterations(const MeshDev& m, KrylovWork& w, const KVec<T, TA>& V, const KBufs& K, int iter0,
                                 int budget, int check_every, hipStream_t st, int* iters_out, int* done_out,
                                 int mode0 = P_FIRST, double* rr_out = nullptr) {
    // Pipelined chunks: chunk q+1 is enqueued before chunk q's state is
    // examined, so the GPU never waits for the host.  Stage kernels return at
    // once when the state they read says done.  Without kernel timing, full
    // chunks are replays of a captured graph.
    int par = iter0 & 1;
    bool first = true, stalled = false;
    double rr_mark = 0.0;
    int it_mark = -1;
    int chunk = 0, last = -1, launched = 0;
    hipError_t e = hipSuccess;
    hipGraphExec_t graph = nullptr;
    const bool timing = w.profile == 1;
    if (!timing && w.use_graphs) {
        if ((e = chunk_graph<DIM, T, TA>(m, w, V, K, &graph)) != hipSuccess) graph = nullptr;
    }
    w.np = 0;
    while (budget > 0) {
        int n = budget < check_every ? budget : check_every;
        const bool replay = graph && !first && par == 1 && budget >= KrylovWork::kGraphIters;
        if (replay) {
            n = KrylovWork::kGraphIters;
            if ((e = hipGraphLaunch(graph, st)) != hipSuccess) return e;
            launched += n;
        } else {
            // with a graph, single iterations only bridge to parity 1 or finish a short budget
            if (graph && n > 1) n = 1;
            for (int q = 0; q < n; ++q) {
                const bool rec = timing && w.np < KrylovWork::kProf;
                hipEvent_t* ev = rec ? w.pev[w.np] : nullptr;
                if (rec) {
                    w.pidx[w.np] = iter0 + launched;
                    w.pa32[w.np] = sizeof(TA) < sizeof(double) ? 1 : 0;
                }
                enqueue_iteration<DIM, T, TA>(m, V, K, par, first ? mode0 : P_NORMAL, st, ev ? ev[0] : nullptr,
                                          ev ? ev[1] : nullptr,
                                          ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
                if (rec) ++w.np;
                ++launched;
                first = false;
                par ^= 1;
            }
        }
        budget -= n;
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(&w.host[chunk & 1], K.st[2], sizeof(KState), hipMemcpyDeviceToHost, st)) !=
            hipSuccess)
            return e;
        if ((e = hipEventRecord(w.ev[chunk & 1], st)) != hipSuccess) return e;
        last = chunk;
        if (chunk > 0) {
            if ((e = hipEventSynchronize(w.ev[(chunk - 1) & 1])) != hipSuccess) return e;
            const KState& q = w.host[(chunk - 1) & 1];
            if (q.done) break;
            // stagnation: no tenfold drop of the recurrence residual within
            // kStallIters iterations ends the run so that the caller restarts
            if (q.rr < 0.01 * rr_mark || it_mark < 0) {
                rr_mark = q.rr;
                it_mark = q.iter;
            } else if (q.iter - it_mark > KrylovWork::kStallIters) {
                stalled = true;
                break;
            }
        }
        ++chunk;
    }
    if (last < 0) {
        *iters_out = iter0;
        *done_out = 0;
        return hipSuccess;
    }
    if ((e = hipEventSynchronize(w.ev[last & 1])) != hipSuccess) return e;
    *iters_out = w.host[last & 1].iter;
    *done_out = w.host[last & 1].done;
    if (stalled && *done_out == 0) *done_out = 3;
    if (rr_out) *rr_out = w.host[last & 1].rr;
    // stage kernels that ran before convergence did work; later ones returned at once
    for (int k = 0; k < w.np; ++k) {
        if (w.pidx[k] >= *iters_out) continue;
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, w.pev[k][0], w.pev[k][1]) == hipSuccess &&
            hipEventElapsedTime(&b, w.pev[k][2], w.pev[k][3]) == hipSuccess) {
            w.ms[0] += a;
            w.ms[1] += b;
            w.cnt[0] += 1;
            w.cnt[1] += 1;
            if (w.pa32[k]) {
                w.ms32[0] += a;
                w.ms32[1] += b;
                w.cnt32[0] += 1;
                w.cnt32[1] += 1;
            }
        }
    }
    w.np = 0;
    return hipSuccess;
}

// r = b - A x, rhat = r and the state the next P-stage starts from;
// synchronises and returns that state.
template <int DIM, typename T, typename TA>
static hipError_t kinit(const MeshDev& m, KrylovWork& w, const KVec<T, TA>& V, const KBufs& K, int with_bb, double tol2,
                        hipStream_t st, KState* out, double delta2 = 0.0, double tol2_next = -1.0) {
    {
        auto go = [&](auto nt_c, auto cf_c) {
            constexpr bool NT = decltype(nt_c)::value, CF = decltype(cf_c)::value;
            if constexpr (DIM == 2)
                hipLaunchKernelGGL((k_t2_init<T, TA, NT, CF>), dim3(K.nblk), dim3(kKBlock), 0, st, m, V, K);
            else
                hipLaunchKernelGGL((k_t3_init<T, TA, NT, CF>), dim3(K.nblk), dim3(kKBlock), 0, st, m, V, K);
        };
        using Tr = std::true_type;
        using Fa = std::false_type;
        if constexpr (sizeof(TA) == sizeof(double)) {
            const bool cf = V.unk != nullptr;
            if (K.nt)
                cf ? go(Tr{}, Tr{}) : go(Tr{}, Fa{});
            else
                cf ? go(Fa{}, Tr{}) : go(Fa{}, Fa{});
        } else {
            K.nt ? go(Tr{}, Fa{}) : go(Fa{}, Fa{});
        }
    }
    hipLaunchKernelGGL(k_kfinish, dim3(1), dim3(kKBlock), 0, st, K, with_bb, tol2, with_bb ? 0 : 1, delta2,
                       tol2_next < 0.0 ? tol2 : tol2_next);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&w.host[0], K.st[2], sizeof(KState), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    *out = w.host[0];
    return hipSuccess;
}

// Bi-CGSTAB with restarts from the true residual; returns iterations,
// restarts, ||r||/||b|| of the final true residual.
template <int DIM, typename T, typename TA>
static hipError_t bicgstab(const MeshDev& m, KrylovWork& w, const KVec<T, TA>& V, const KBufs& K, double tol,
                           int max_iter, int check_every, hipStream_t st, int* iters, int* restarts, double* rel,
                           int* conv, bool confirm = true) {
    KState h;
    hipError_t e = kinit<DIM, T, TA>(m, w, V, K, 1, tol * tol, st, &h);
    if (e != hipSuccess) return e;
    *restarts = 0;
    *iters = 0;
    const double bb = h.bb;
    if (bb == 0.0) {
        const int gz = (m.Nc + kBlock - 1) / kBlock > 8192 ? 8192 : (m.Nc + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_zero<T>, dim3(gz), dim3(kBlock), 0, st, m.Nc, V.x);
        *rel = 0.0;
        *conv = 1;
        return hipGetLastError();
    }
    int idle = 0;
    double tight = 1.0;
    while (!h.done && h.iter < max_iter) {
        const int before = h.iter;
        int it = 0, done = 0;
        if ((e = run_iterations<DIM, T, TA>(m, w, V, K, h.iter, max_iter - h.iter, check_every, st, &it, &done)) !=
            hipSuccess)
            return e;
        if (!confirm) {
            // inner solve of the refinement: the FP64 outer residual is the check
            h = w.host[0];
            h.iter = it;
            h.done = done == 1 ? 1 : 0;
            h.rr = 0.0;
            break;
        }
        // confirm with the true residual; restart from it if needed, with the
        // recurrence held to a tighter threshold when it had claimed convergence
        const double next = done == 1 ? tight * 0.25 : tight;
        if ((e = kinit<DIM, T, TA>(m, w, V, K, 0, tol * tol, st, &h, 0.0, tol * tol * next)) != hipSuccess) return e;
        if (!h.done) {
            *restarts += 1;
            tight = next > 1e-6 ? next : 1e-6;
        }
        // a restart that makes no progress (a non-finite iterate, or the
        // recurrence and the true residual straddling the tolerance) ends
        // the solve unconverged instead of looping
        idle = h.iter == before ? idle + 1 : 0;
        if (idle >= 2 || !std::isfinite(h.rr)) break;
    }
    *iters = h.iter;
    *rel = bb > 0 ? sqrt(h.rr / bb) : 0.0;
    *conv = h.done == 1 || bb == 0.0;
    return hipSuccess;
}

template <int DIM>
static hipError_t solve_dim(const MeshDev& m, const SetDev& set, KrylovWork& w, const double* rhs,
                            const double* fneu, double* p, const SolveParams& sp, SolveOut* out, int* bad,
                            hipStream_t st) {
    const int g = (m.Nc + kBlock - 1) / kBlock > 8192 ? 8192 : (m.Nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_ppe_rhs<DIM>, dim3(g), dim3(kBlock), 0, st, m, set, rhs, p, fneu, sp.caller_guess, w.beff,
                       w.v64.x, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    *out = SolveOut{};
    // the multigrid solve reads the non-finite flag back with its first
    // totals; the other forms check it here
    if (sp.precond != MCD_PRECOND_MG) {
        if ((e = hipMemcpyAsync(w.bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        if (*w.bad_host) {                      // caller reports the non-finite input
            out->bad = 1;
            return hipSuccess;
        }
    }
    // the operator the Krylov iterations see: A, or A D^-1 with Jacobi
    const double* A64 = set.amat;
    const float* A32 = set.amat32;
    if (sp.precond == MCD_PRECOND_MG) {
        // Bi-CGSTAB with FP64 vectors right-preconditioned by one FP32 V-cycle,
        // products with the FP64 matrix or (FP32_MATRIX) its FP32 copy; p[1]
        // and v[1] hold the preconditioned directions
        const MgVecs mv{w.v64.x, w.v64.r, w.v64.rhat, w.v64.p[0], w.v64.v[0], w.v64.s, w.v64.t, w.v64.p[1],
                        w.v64.v[1], w.beff};
        MgResult res;
        if ((e = mg_bicgstab(m, *w.mg, set, mv, sp.tol, sp.max_iter, sp.precision == MCD_PREC_FP32_MATRIX, bad, st,
                             &res)) != hipSuccess)
            return e;
        if (res.bad) {                          // caller reports the non-finite input
            out->bad = 1;
            return hipSuccess;
        }
        out->iterations = res.iterations;
        out->restarts = res.restarts;
        out->converged = res.converged;
        out->rel = res.rel;
        out->bnorm = res.bnorm;
        hipLaunchKernelGGL(k_writeback, dim3(g), dim3(kBlock), 0, st, m.Nc, set.unknown, w.v64.x, p);
        return hipGetLastError();
    }
    const bool jacobi = sp.precond == MCD_PRECOND_JACOBI;
    if (jacobi) {
        hipLaunchKernelGGL(k_jacobi_diag<DIM>, dim3(g), dim3(kBlock), 0, st, m, set.amat, set.unknown, w.dinv,
                           w.v64.x);
        hipLaunchKernelGGL(k_jacobi_matrix<DIM>, dim3(g), dim3(kBlock), 0, st, m, set.amat, set.unknown, w.dinv,
                           w.jac64, w.jac32);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        A64 = w.jac64;
        A32 = w.jac32;
    }
    KVec<double> V = w.v64;
    V.A = A64;
    V.b = w.beff;
    if (!jacobi) V.unk = set.unknown;
    const int check = sp.check_every > 0 ? sp.check_every : 8;
    if (sp.precision == MCD_PREC_FP64) {
        int it = 0, rst = 0, conv = 0;
        double rel = 0.0;
        if ((e = bicgstab<DIM, double, double>(m, w, V, w.kb64, sp.tol, sp.max_iter, check, st, &it, &rst, &rel, &conv)) !=
            hipSuccess)
            return e;
        out->iterations = it;
        out->restarts = rst;
        out->converged = conv;
        out->rel = rel;
        out->bnorm = sqrt(w.host[0].bb);
    } else if (sp.precision == MCD_PREC_FP32_MATRIX) {
        // FP64 Bi-CGSTAB whose stage products read the FP32-stored matrix
        // (half the matrix bytes; products and all vectors in FP64), with
        // residual replacement: when the recursive residual has fallen by
        // inner_tol below its largest value since the last replacement (or
        // to the tolerance), r := b - A64 x is recomputed with the FP64
        // matrix and the recursion resumes from it with its Krylov space
        // kept.  Convergence is only declared on that FP64 residual.  A
        // breakdown restarts from the FP64 residual; more than max_outer
        // replacements, two rounds without an iteration, or an FP64 residual
        // 100x above the best one seen hand over to plain FP64 Bi-CGSTAB
        // from the current iterate.
        KVec<double, float> VM;
        VM.x = V.x;
        VM.r = V.r;
        VM.rhat = V.rhat;
        VM.s = V.s;
        VM.t = V.t;
        VM.p[0] = V.p[0];
        VM.p[1] = V.p[1];
        VM.v[0] = V.v[0];
        VM.v[1] = V.v[1];
        VM.A = A32;
        VM.b = w.beff;
        const double tol2 = sp.tol * sp.tol, delta2 = sp.inner_tol * sp.inner_tol;
        KState h;
        if ((e = kinit<DIM, double, double>(m, w, V, w.kb64, 1, tol2, st, &h, delta2)) != hipSuccess) return e;
        const double bb = h.bb;
        if (bb == 0.0) {             // zero right-hand side: the zero solution
            hipLaunchKernelGGL(k_zero<double>, dim3(g), dim3(kBlock), 0, st, m.Nc, V.x);
            h.done = 1;
            h.rr = 0.0;
        }
        int mode = P_FIRST, repl = 0, idle = 0, restarts = 0, fallback = 0;
        double rr_best = h.rr, tight = 1.0;
        bool fp64_phase = false;
        while (!h.done && h.iter < sp.max_iter) {
            const int before = h.iter;
            int it = 0, done = 0;
            double rr_rec = 0.0;
            if (fp64_phase) {
                if ((e = run_iterations<DIM, double, double>(m, w, V, w.kb64, h.iter, sp.max_iter - h.iter, check, st,
                                                             &it, &done, mode, &rr_rec)) != hipSuccess)
                    return e;
            } else if ((e = run_iterations<DIM, double, float>(m, w, VM, w.kb64, h.iter, sp.max_iter - h.iter, check,
                                                               st, &it, &done, mode, &rr_rec)) != hipSuccess) {
                return e;
            }
            if (done == 0) {          // iteration budget spent
                h.iter = it;
                break;
            }
            hipLaunchKernelGGL(k_true_replace<DIM>, dim3(w.kb64.nblk), dim3(kKBlock), 0, st, m, A64,
                               set.unknown, w.beff, VM, w.kb64);
            // a recurrence that reached the tolerance without the FP64 residual
            // doing so continues to a tighter one
            if (done == 1 && rr_rec <= tol2 * tight * bb) tight = tight * 0.25 > 1e-6 ? tight * 0.25 : 1e-6;
            // the FP64 phase needs no further replacements before the tolerance
            const bool tail = fp64_phase || rr_rec <= sp.fp64_below * sp.fp64_below * bb;
            hipLaunchKernelGGL(k_replace_finish, dim3(1), dim3(kKBlock), 0, st, w.kb64, tol2, tol2 * tight,
                               tail ? 0.0 : delta2);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(&w.host[0], w.kb64.st[2], sizeof(KState), hipMemcpyDeviceToHost, st)) !=
                hipSuccess)
                return e;
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
            h = w.host[0];
            ++repl;
            if (h.done) break;
            rr_best = fmin(rr_best, h.rr);
            idle = h.iter == before ? idle + 1 : 0;
            // no progress, too many replacements, or a recursion that has
            // drifted away (FP64 residual 100x above its best): plain FP64
            if (idle >= 2 || repl > sp.max_outer || !std::isfinite(h.rr) || h.rr > 1e4 * rr_best) {
                fallback = 1;
                break;
            }
            // close to the tolerance the products switch to the FP64 matrix (the
            // vectors are FP64 already, so the recursion just goes on)
            if (tail) fp64_phase = true;
            if (done >= 2) {          // breakdown or stagnation: new recursion from the FP64 residual
                if ((e = kinit<DIM, double, double>(m, w, V, w.kb64, 0, tol2, st, &h, delta2, tol2 * tight)) !=
                    hipSuccess)
                    return e;
                ++restarts;
                mode = P_FIRST;
            } else {
                mode = P_RESUME;
            }
        }
        int total = h.iter;
        bool conv = h.done == 1 || bb == 0.0;
        double rr = h.rr;
        if (fallback && !conv && total < sp.max_iter) {
            if (!std::isfinite(h.rr))      // a non-finite iterate: start over from zero
                hipLaunchKernelGGL(k_ppe_rhs<DIM>, dim3(g), dim3(kBlock), 0, st, m, set, rhs, p, fneu, 0, w.beff,
                                   w.v64.x, bad);
            int it = 0, rst = 0, c64 = 0;
            double rel = 0.0;
            if ((e = bicgstab<DIM, double, double>(m, w, V, w.kb64, sp.tol, sp.max_iter - total, check, st, &it, &rst,
                                                   &rel, &c64)) != hipSuccess)
                return e;
            total += it;
            restarts += rst + 1;
            conv = c64 != 0;
            rr = rel * rel * bb;
        }
        out->iterations = total;
        out->restarts = restarts;
        out->refinements = repl;
        out->converged = conv ? 1 : 0;
        out->rel = bb > 0 ? sqrt(rr / bb) : 0.0;
        out->bnorm = sqrt(bb);
    } else {
        // FP64 iterative refinement around an FP32 Bi-CGSTAB (FP64 dots).
        // A correction that does not lower the FP64 true residual is undone
        // and the inner tolerance loosened; after two such rejections the
        // solve finishes with FP64 Bi-CGSTAB from the current iterate, so the
        // tolerance is always met on the FP64 operator.
        KVec<float> V32 = w.v32;
        V32.A = A32;
        KState h;
        if ((e = kinit<DIM, double, double>(m, w, V, w.kb64, 1, sp.tol * sp.tol, st, &h)) != hipSuccess) return e;
        const double bb = h.bb;
        if (bb == 0.0) {             // zero right-hand side: the zero solution
            hipLaunchKernelGGL(k_zero<double>, dim3(g), dim3(kBlock), 0, st, m.Nc, V.x);
            h.done = 1;
            h.rr = 0.0;
        }
        int total = 0, outer = 0, rst_total = 0, rejected = 0, fallback = 0;
        double itol = sp.inner_tol;
        while (!h.done && outer < sp.max_outer && total < sp.max_iter) {
            const double nr = sqrt(h.rr);
            const double rr_old = h.rr;
            if ((e = hipMemcpyAsync(w.xsave, V.x, (size_t)m.Nc * sizeof(double), hipMemcpyDeviceToDevice, st)) !=
                hipSuccess)
                return e;
            hipLaunchKernelGGL(k_to32, dim3(g), dim3(kBlock), 0, st, m.Nc, V.s, 1.0 / nr, (float*)V32.b, V32.x);
            int it = 0, rst = 0, conv = 0;
            double rel = 0.0;
            const int left = sp.max_iter - total;
            const int cap = sp.max_inner > 0 && sp.max_inner < left ? sp.max_inner : left;
            if ((e = bicgstab<DIM, float, float>(m, w, V32, w.kb32, itol, cap, check, st, &it, &rst, &rel, &conv, false)) !=
                hipSuccess)
                return e;
            total += it;
            rst_total += rst;
            hipLaunchKernelGGL(k_refine, dim3(g), dim3(kBlock), 0, st, m.Nc, V32.x, nr, V.x);
            if ((e = kinit<DIM, double, double>(m, w, V, w.kb64, 0, sp.tol * sp.tol, st, &h)) != hipSuccess) return e;
            ++outer;
            if (!(h.rr < rr_old)) {
                if ((e = hipMemcpyAsync(V.x, w.xsave, (size_t)m.Nc * sizeof(double), hipMemcpyDeviceToDevice, st)) !=
                    hipSuccess)
                    return e;
                if ((e = kinit<DIM, double, double>(m, w, V, w.kb64, 0, sp.tol * sp.tol, st, &h)) != hipSuccess) return e;
                itol = itol * 3.0 < 0.5 ? itol * 3.0 : 0.5;
                if (++rejected >= 2) {
                    fallback = 1;
                    break;
                }
            }
        }
        if (fallback && !h.done && total < sp.max_iter) {
            int it = 0, rst = 0, conv = 0;
            double rel = 0.0;
            if ((e = bicgstab<DIM, double, double>(m, w, V, w.kb64, sp.tol, sp.max_iter - total, check, st, &it, &rst, &rel,
                                           &conv)) != hipSuccess)
                return e;
            total += it;
            rst_total += rst + 1;
            h.done = conv ? 1 : 0;
            h.rr = rel * rel * bb;
        }
        out->iterations = total;
        out->restarts = rst_total;
        out->refinements = outer;
        out->converged = h.done == 1 || bb == 0.0;
        out->rel = bb > 0 ? sqrt(h.rr / bb) : 0.0;
        out->bnorm = sqrt(bb);
    }
    if (jacobi) {
        // back to x = D^-1 y; the tolerance is confirmed on A itself (the
        // scaled product differs from A x by rounding), and a miss is finished
        // by unpreconditioned FP64 Bi-CGSTAB within the iteration budget
        hipLaunchKernelGGL(k_jacobi_unscale, dim3(g), dim3(kBlock), 0, st, m.Nc, set.unknown, w.dinv, V.x);
        KVec<double> V0 = V;
        V0.A = set.amat;
        V0.unk = set.unknown;
        if (out->bnorm > 0.0) {
            KState h;
            if ((e = kinit<DIM, double, double>(m, w, V0, w.kb64, 1, sp.tol * sp.tol, st, &h)) != hipSuccess) return e;
            double rel = sqrt(h.rr / h.bb);
            int conv = h.done == 1;
            if (!conv && out->iterations < sp.max_iter) {
                int it = 0, rst = 0;
                if ((e = bicgstab<DIM, double, double>(m, w, V0, w.kb64, sp.tol, sp.max_iter - out->iterations, check,
                                                       st, &it, &rst, &rel, &conv)) != hipSuccess)
                    return e;
                out->iterations += it;
                out->restarts += rst + 1;
            }
            out->rel = rel;
            out->converged = conv ? 1 : 0;
        }
    }
    hipLaunchKernelGGL(k_writeback, dim3(g), dim3(kBlock), 0, st, m.Nc, set.unknown, V.x, p);
    return hipGetLastError();
}

// The solve runs on the workspace's own stream (ordered after the caller's
// stream by an event) so that its chunks can be captured and replayed as
// graphs; it returns after that stream is idle.
hipError_t solve_ppe_impl(const MeshDev& m, const SetDev& set, KrylovWork& w, const double* rhs, const double* fneu,
                          double* p, const SolveParams& sp, SolveOut* out, int* bad, hipStream_t caller) {
    hipError_t e = hipEventRecord(w.join, caller);
    if (e != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(w.st, w.join, 0)) != hipSuccess) return e;
    e = m.dim == 2 ? solve_dim<2>(m, set, w, rhs, fneu, p, sp, out, bad, w.st)
                   : solve_dim<3>(m, set, w, rhs, fneu, p, sp, out, bad, w.st);
    const hipError_t e2 = hipStreamSynchronize(w.st);
    return e != hipSuccess ? e : e2;
}

// The nine vectors of one precision in one allocation, mps elements apart
// (padded, so that the same cell of different vectors is not on one HBM
// channel); x is the allocation's base.
template <typename T>
static hipError_t alloc_vec(KVec<T>& V, size_t mps) {
    T* base = nullptr;
    hipError_t e = hipMalloc((void**)&base, 9 * mps * sizeof(T));
    if (e != hipSuccess) return e;
    if ((e = hipMemset(base, 0, 9 * mps * sizeof(T))) != hipSuccess) {
        (void)hipFree(base);
        return e;
    }
    T** ptrs[9] = {&V.x, &V.r, &V.rhat, &V.s, &V.t, &V.p[0], &V.p[1], &V.v[0], &V.v[1]};
    for (int k = 0; k < 9; ++k) *ptrs[k] = base + k * mps;
    V.A = nullptr;
    V.b = nullptr;
    return hipSuccess;
}

template <typename T>
static void free_vec(KVec<T>& V) {
    if (V.x) (void)hipFree(V.x);
}

// Residual of the PPE at p: r = (rhs - Dirichlet and Neumann columns) - A p
// on unknown rows.  norms = (||r||_2, ||b_eff||_2): runs on the caller's
// stream and returns after it has drained; norms null: only enqueues r.
hipError_t ppe_residual_impl(const MeshDev& m, const SetDev& set, KrylovWork& w, const double* rhs, const double* fneu,
                             const double* p, double* r, double norms[2], int* bad, hipStream_t st) {
    const int g = (m.Nc + kBlock - 1) / kBlock > 8192 ? 8192 : (m.Nc + kBlock - 1) / kBlock;
    const int gr = (m.Nc + kBlock - 1) / kBlock > 2 * kKGrid ? 2 * kKGrid : (m.Nc + kBlock - 1) / kBlock;
    double* part = w.kb64.part[0];     // 4 * cap >= 2 * gr doubles
    double* fin = w.kb64.part[1];
    if (m.dim == 2) {
        hipLaunchKernelGGL(k_ppe_rhs<2>, dim3(g), dim3(kBlock), 0, st, m, set, rhs, p, fneu, 1, w.beff, w.v64.x, bad);
        hipLaunchKernelGGL(k_ppe_resid<2>, dim3(gr), dim3(kBlock), 0, st, m, set.amat, set.unknown, w.beff, w.v64.x,
                           r, part);
    } else {
        hipLaunchKernelGGL(k_ppe_rhs<3>, dim3(g), dim3(kBlock), 0, st, m, set, rhs, p, fneu, 1, w.beff, w.v64.x, bad);
        hipLaunchKernelGGL(k_ppe_resid<3>, dim3(gr), dim3(kBlock), 0, st, m, set.amat, set.unknown, w.beff, w.v64.x,
                           r, part);
    }
    if (!norms) return hipGetLastError();        // r only: nothing to wait for
    hipLaunchKernelGGL(k_resid_finish, dim3(1), dim3(kBlock), 0, st, part, gr, fin);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = hipMemcpyAsync(w.host, fin, 2 * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    const double* h = reinterpret_cast<const double*>(w.host);
    norms[0] = h[0];
    norms[1] = h[1];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Allocation-free residual: its scratch is a file-scope device array (one copy
// per device, kept until the process ends).  The residual's grid is at most
// 2 kKGrid blocks at any mesh size, so the scratch size does not depend on
// the mesh.  Host code uses the per-device address from hipGetSymbolAddress,
// never the array's name.
// ---------------------------------------------------------------------------

constexpr int kNoAllocBlocks = 2 * kKGrid;
struct NoAllocScratch {
    double part[2 * kNoAllocBlocks];   // per-block partial sums of r.r and b.b
    double fin[2];                     // ||r||, ||b_eff||
    int bad;                           // non-finite b_eff rows
};
static __device__ __align__(256) NoAllocScratch scratch;

constexpr int kMaxDevices = 64;
static NoAllocScratch* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

size_t noalloc_scratch_bytes() { return sizeof(NoAllocScratch); }

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<NoAllocScratch*>(ptr);
    return hipSuccess;
}

hipError_t ppe_residual_noalloc_impl(int device, const MeshDev& m, const SetDev& set, const double* rhs,
                                     const double* fneu, const double* p, double* r, double norms[2], int* bad_out,
                                     hipStream_t st) {
    if (device < 0 || device >= kMaxDevices || !g_scratch_ptr[device]) return hipErrorNotInitialized;
    NoAllocScratch* ptr = g_scratch_ptr[device];
    const int gr = (m.Nc + kBlock - 1) / kBlock > kNoAllocBlocks ? kNoAllocBlocks : (m.Nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, &ptr->bad);
    if (m.dim == 2)
        hipLaunchKernelGGL(k_ppe_resid_fused<2>, dim3(gr), dim3(kBlock), 0, st, m, set, rhs, p, fneu, r, ptr->part,
                           &ptr->bad);
    else
        hipLaunchKernelGGL(k_ppe_resid_fused<3>, dim3(gr), dim3(kBlock), 0, st, m, set, rhs, p, fneu, r, ptr->part,
                           &ptr->bad);
    hipLaunchKernelGGL(k_resid_finish, dim3(1), dim3(kBlock), 0, st, ptr->part, gr, ptr->fin);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double h[2];
    if ((e = hipMemcpyAsync(h, ptr->fin, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(bad_out, &ptr->bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    norms[0] = h[0];
    norms[1] = h[1];
    return hipSuccess;
}

// Stage-kernel shape: 64 x 8 tiles (2D) or 64 x 8 x depth bricks (3D), at
// most `grid` (<= kKGrid) blocks, each looping over a contiguous run of
// tiles.  Returns false for a shape outside those limits.
static bool shape_of(const MeshDev& m, int grid, int depth, KBufs& K) {
    if (grid < 1 || grid > kKGrid || (m.dim == 3 && (depth < 1 || depth > m.n[2])) || (m.dim == 2 && depth != 1))
        return false;
    const int ntx = (m.n[0] + TX - 1) / TX, nty = (m.n[1] + TY - 1) / TY;
    const int ntiles = ntx * nty * (m.dim == 3 ? (m.n[2] + depth - 1) / depth : 1);
    const int nblk = ntiles < grid ? ntiles : grid;
    K.nblk = nblk;
    K.ntx = ntx;
    K.nty = nty;
    K.ntiles = ntiles;
    K.tpb = (ntiles + nblk - 1) / nblk;
    K.tz = m.dim == 3 ? depth : 1;
    return true;
}

// Applies a stage-kernel shape to both precisions; captured chunk graphs
// hold the old one, so they are dropped.
hipError_t krylov_set_shape(const MeshDev& m, KrylovWork& w, int grid, int depth) {
    KBufs K = w.kb64;
    if (!shape_of(m, grid, depth, K)) return hipErrorInvalidValue;
    hipError_t e = hipStreamSynchronize(w.st);
    if (e != hipSuccess) return e;
    for (int i = 0; i < w.ngraphs; ++i) (void)hipGraphExecDestroy(w.graphs[i].exec);
    w.ngraphs = 0;
    for (KBufs* Q : {&w.kb64, &w.kb32}) {
        Q->nblk = K.nblk;
        Q->ntx = K.ntx;
        Q->nty = K.nty;
        Q->ntiles = K.ntiles;
        Q->tpb = K.tpb;
        Q->tz = K.tz;
    }
    w.grid_req = grid;
    return hipSuccess;
}

void krylov_get_shape(const KrylovWork& w, int* grid, int* depth, int* blocks) {
    *grid = w.grid_req;
    *depth = w.kb64.tz;
    *blocks = w.kb64.nblk;
}

// b := 1 and x := 0 at unknown rows (0 elsewhere): the timing problem.
__global__ void k_tune_problem(int Nc, const uint8_t* __restrict__ unknown, double* __restrict__ b,
                               double* __restrict__ x) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x) {
        b[c] = unknown[c] ? 1.0 : 0.0;
        x[c] = 0.0;
    }
}

// Times `iters` FP64 iterations (after two untimed ones) of the stage kernels
// in the current shape on the set's operator; *ok = 0 when the recursion
// stopped early (a breakdown would make later launches return at once).
template <int DIM>
static hipError_t time_shape(const MeshDev& m, const SetDev& set, KrylovWork& w, int iters, hipEvent_t t0,
                             hipEvent_t t1, float* ms, int* ok) {
    hipStream_t st = w.st;
    KVec<double> V = w.v64;
    V.A = set.amat;
    V.b = w.beff;
    V.unk = set.unknown;
    const int g = (m.Nc + kBlock - 1) / kBlock > 8192 ? 8192 : (m.Nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_tune_problem, dim3(g), dim3(kBlock), 0, st, m.Nc, set.unknown, w.beff, V.x);
    KState h;
    hipError_t e = kinit<DIM, double, double>(m, w, V, w.kb64, 1, 0.0, st, &h);
    if (e != hipSuccess) return e;
    enqueue_iteration<DIM, double, double>(m, V, w.kb64, 0, P_FIRST, st, nullptr, nullptr, nullptr, nullptr);
    enqueue_iteration<DIM, double, double>(m, V, w.kb64, 1, P_NORMAL, st, nullptr, nullptr, nullptr, nullptr);
    if ((e = hipEventRecord(t0, st)) != hipSuccess) return e;
    for (int q = 0; q < iters; ++q)
        enqueue_iteration<DIM, double, double>(m, V, w.kb64, q & 1, P_NORMAL, st, nullptr, nullptr, nullptr, nullptr);
    if ((e = hipEventRecord(t1, st)) != hipSuccess) return e;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&w.host[0], w.kb64.st[2], sizeof(KState), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if ((e = hipEventElapsedTime(ms, t0, t1)) != hipSuccess) return e;
    *ok = w.host[0].done == 0 && w.host[0].iter == iters + 2;
    return hipSuccess;
}

// Autotuner of the stage-kernel shape: every candidate (block count, and
// brick depth in 3D) is timed on the set's FP64 operator, each twice,
// keeping the faster run; the fastest candidate is applied, unless the
// default shape is within 2 % of it (the default is kept then, so that
// timing noise does not change the shape, and with it the summation order,
// from run to run).  Results: per candidate (grid, depth, us per iteration,
// < 0 when rejected) and the index applied.
hipError_t krylov_autotune(const MeshDev& m, const SetDev& set, KrylovWork& w, int iters, int max_cand,
                           int* n_out, int* grid_out, int* depth_out, double* us_out, int* chosen) {
    static const int grids[] = {128, 256, 384, 512};
    static const int depths3[] = {4, 8, 16};
    const int nd = m.dim == 3 ? 3 : 1;
    int n = 0;
    for (int di = 0; di < nd; ++di) {
        const int depth = m.dim == 3 ? depths3[di] : 1;
        if (m.dim == 3 && depth > m.n[2]) continue;
        int last_nblk = -1;
        for (int grid : grids) {
            KBufs K = w.kb64;
            if (!shape_of(m, grid, depth, K) || K.nblk == last_nblk) continue;    // same effective shape
            last_nblk = K.nblk;
            if (n == max_cand) break;
            grid_out[n] = grid;
            depth_out[n] = depth;
            ++n;
        }
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    const int grid0 = w.grid_req, depth0 = w.kb64.tz;
    // the candidate with the default shape's effective block count and depth
    KBufs K0 = w.kb64;
    (void)shape_of(m, kKGrid, m.dim == 3 ? kDefaultDepth : 1, K0);
    int best = -1, dflt = -1;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        if ((e = krylov_set_shape(m, w, grid_out[i], depth_out[i])) != hipSuccess) break;
        float ms = 0.f, ms2 = 0.f;
        int ok = 0, ok2 = 0;
        e = m.dim == 2 ? time_shape<2>(m, set, w, iters, t0, t1, &ms, &ok) : time_shape<3>(m, set, w, iters, t0, t1, &ms, &ok);
        if (e != hipSuccess) break;
        e = m.dim == 2 ? time_shape<2>(m, set, w, iters, t0, t1, &ms2, &ok2)
                       : time_shape<3>(m, set, w, iters, t0, t1, &ms2, &ok2);
        if (e != hipSuccess) break;
        us_out[i] = ok && ok2 ? 1e3 * (double)fminf(ms, ms2) / iters : -1.0;
        if (us_out[i] > 0 && (best < 0 || us_out[i] < us_out[best])) best = i;
        KBufs Ki = w.kb64;
        (void)shape_of(m, grid_out[i], depth_out[i], Ki);
        if (Ki.nblk == K0.nblk && Ki.tz == K0.tz) dflt = i;
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e != hipSuccess) {
        (void)krylov_set_shape(m, w, grid0, depth0);
        return e;
    }
    if (best >= 0 && dflt >= 0 && us_out[dflt] > 0 && us_out[dflt] <= 1.02 * us_out[best]) best = dflt;
    *n_out = n;
    *chosen = best;
    if (best < 0) return krylov_set_shape(m, w, grid0, depth0);
    return krylov_set_shape(m, w, grid_out[best], depth_out[best]);
}

hipError_t krylov_alloc(const MeshDev& m, KrylovWork** out) {
    KrylovWork* w = new KrylovWork{};
    *out = w;
    const int Nc = m.Nc;
    w->Nc = Nc;
    hipError_t e;
    KBufs K0{};
    (void)shape_of(m, kKGrid, m.dim == 3 ? kDefaultDepth : 1, K0);
    w->grid_req = kKGrid;
    const int cap = kKGrid;
    // the matrix stays in the last-level cache between iterations when it fits
    // there with the Krylov vectors; larger systems stream it
    const size_t S = m.dim == 3 ? 27 : 9;
    for (KBufs* K : {&w->kb64, &w->kb32}) {
        *K = K0;
        K->cap = cap;
        const size_t mat = S * (size_t)Nc * (K == &w->kb64 ? sizeof(double) : sizeof(float));
        K->nt = mat + 10 * (size_t)Nc * sizeof(double) > kCacheFitBytes ? 1 : 0;
        for (int q = 0; q < 3; ++q) {
            if ((e = hipMalloc((void**)&K->part[q], 4 * (size_t)cap * sizeof(double))) != hipSuccess) return e;
            if ((e = hipMemset(K->part[q], 0, 4 * (size_t)cap * sizeof(double))) != hipSuccess) return e;
            if ((e = hipMalloc((void**)&K->st[q], sizeof(KState))) != hipSuccess) return e;
            if ((e = hipMemset(K->st[q], 0, sizeof(KState))) != hipSuccess) return e;
        }
    }
    if ((e = hipHostMalloc((void**)&w->host, 2 * sizeof(KState), hipHostMallocDefault)) != hipSuccess) return e;
    for (int i = 0; i < 2; ++i)
        if ((e = hipEventCreateWithFlags(&w->ev[i], hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = mg_alloc(m, &w->mg)) != hipSuccess) return e;
    if ((e = alloc_vec(w->v64, m.mps)) != hipSuccess) return e;
    if ((e = alloc_vec(w->v32, m.mps)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->beff, (size_t)Nc * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->b32, (size_t)Nc * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->xsave, (size_t)Nc * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->dinv, (size_t)Nc * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->jac64, S * m.mps * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->jac32, S * m.mps * sizeof(float))) != hipSuccess) return e;
    w->v32.b = w->b32;
    if ((e = hipHostMalloc((void**)&w->bad_host, sizeof(int), hipHostMallocDefault)) != hipSuccess) return e;
    if ((e = hipStreamCreateWithFlags(&w->st, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&w->join, hipEventDisableTiming)) != hipSuccess) return e;
    return hipSuccess;
}

bool krylov_mg_usable(const KrylovWork* w) { return mg_usable(w->mg); }

hipError_t krylov_mg_apply(const MeshDev& m, KrylovWork& w, const SetDev& set, const double* in, double* out,
                           int* levels, hipStream_t st) {
    hipError_t e = mg_apply(m, *w.mg, set, in, out, levels, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

hipError_t krylov_profile(KrylovWork* w, int enable) {
    if (enable && !w->profile) {
        for (int k = 0; k < KrylovWork::kProf; ++k)
            for (int q = 0; q < 4; ++q) {
                hipError_t e = hipEventCreate(&w->pev[k][q]);
                if (e != hipSuccess) return e;
            }
        w->profile = 1;
    }
    if (!enable && w->profile) w->profile = 2;   // events stay allocated; recording off
    if (enable) w->profile = 1;
    return hipSuccess;
}

void krylov_profile_read(KrylovWork* w, double* ms_p, long long* n_p, double* ms_s, long long* n_s, double* ms32,
                         long long* n32, int reset) {
    *ms_p = w->ms[0];
    *n_p = w->cnt[0];
    *ms_s = w->ms[1];
    *n_s = w->cnt[1];
    if (ms32 && n32) {
        ms32[0] = w->ms32[0];
        ms32[1] = w->ms32[1];
        n32[0] = w->cnt32[0];
        n32[1] = w->cnt32[1];
    }
    if (reset) {
        w->ms[0] = w->ms[1] = 0.0;
        w->cnt[0] = w->cnt[1] = 0;
        w->ms32[0] = w->ms32[1] = 0.0;
        w->cnt32[0] = w->cnt32[1] = 0;
    }
}

void krylov_free(KrylovWork* w) {
    if (!w) return;
    for (KBufs* K : {&w->kb64, &w->kb32})
        for (int q = 0; q < 3; ++q) {
            if (K->part[q]) (void)hipFree(K->part[q]);
            if (K->st[q]) (void)hipFree(K->st[q]);
        }
    if (w->host) (void)hipHostFree(w->host);
    for (int i = 0; i < 2; ++i)
        if (w->ev[i]) (void)hipEventDestroy(w->ev[i]);
    free_vec(w->v64);
    free_vec(w->v32);
    mg_free(w->mg);
    if (w->beff) (void)hipFree(w->beff);
    if (w->b32) (void)hipFree(w->b32);
    if (w->xsave) (void)hipFree(w->xsave);
    if (w->dinv) (void)hipFree(w->dinv);
    if (w->jac64) (void)hipFree(w->jac64);
    if (w->jac32) (void)hipFree(w->jac32);
    if (w->bad_host) (void)hipHostFree(w->bad_host);
    for (int i = 0; i < w->ngraphs; ++i) (void)hipGraphExecDestroy(w->graphs[i].exec);
    if (w->join) (void)hipEventDestroy(w->join);
    if (w->st) (void)hipStreamDestroy(w->st);
    if (w->profile)
        for (int k = 0; k < KrylovWork::kProf; ++k)
            for (int q = 0; q < 4; ++q) (void)hipEventDestroy(w->pev[k][q]);
    delete w;
}

}  // namespace mcd
