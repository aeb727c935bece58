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
#include "common.h"

namespace mcd {

struct KState {
    double rho, alpha, omega;
    double bb, rr, rr0, rv;
    double ts, tt, rsv, rtv;
    double tol2;
    int done;       // 0 running, 1 recurrence converged, 2 breakdown
    int iter;
    unsigned int ticket;
    int pad;
};

constexpr int kMaxGrid = 2048;

template <typename T>
struct KVec {
    T *x, *r, *rhat, *s, *t, *p[2], *v[2];
    const T* A;      // [S][Nc]
    const T* b;
};

// Sum of A[s][c] * val(j) over the stencil slots of cell c.
template <int DIM, typename T, typename F>
__device__ __forceinline__ T spmv_row(const MeshDev& m, const T* __restrict__ A, int c, F val) {
    constexpr int S = Dims<DIM>::S;
    const size_t Nc = (size_t)m.Nc;
    int ijk[3];
    cell_ijk(m, c, ijk);
    T acc = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const T a = A[(size_t)s * Nc + c];
        if (a == T(0)) continue;
        int j;
        double sh[3];
        if (!neighbour<DIM>(m, ijk, s, j, sh)) continue;
        acc += a * val(j);
    }
    return acc;
}

// Block-reduce NQ partial sums, then the last block reduces all blocks'
// partials (fixed order) into tot[] (valid in thread 0 of the last block).
template <int NQ>
__device__ __forceinline__ bool grid_reduce(double (&v)[NQ], double* part, KState* ks, double (&tot)[NQ]) {
    __shared__ double lds[NQ][kBlock / 64];
    __shared__ bool last;
    block_sum<NQ>(v, lds);
    const int G = gridDim.x;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[q * kMaxGrid + blockIdx.x] = v[q];
        __threadfence();
        const unsigned t = atomicAdd(&ks->ticket, 1u);
        last = (t == (unsigned)(G - 1));
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int b = threadIdx.x; b < G; b += kBlock) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += __builtin_nontemporal_load(&part[q * kMaxGrid + b]);
    }
    __syncthreads();
    block_sum<NQ>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tot[q] = acc[q];
        ks->ticket = 0;
    }
    return true;
}

// r0 = b - A x;  rhat = r0 (stored in s and rhat);  dots: r0.r0 (and b.b).
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_kinit(MeshDev m, KVec<T> V, double* part, KState* ks, int with_bb,
                                                  double tol2) {
    double v[2] = {0.0, 0.0};
    const int G = gridDim.x;
    const int lb = xcd_block(blockIdx.x, G);
    for (int c = lb * blockDim.x + threadIdx.x; c < m.Nc; c += G * blockDim.x) {
        const T* x = V.x;
        const T ax = spmv_row<DIM, T>(m, V.A, c, [&](int j) { return x[j]; });
        const T bc = V.b[c];
        const T r = bc - ax;
        V.s[c] = r;
        V.rhat[c] = r;
        v[0] += (double)r * (double)r;
        v[1] += (double)bc * (double)bc;
    }
    double tot[2];
    if (grid_reduce<2>(v, part, ks, tot) && threadIdx.x == 0) {
        if (with_bb) {
            ks->bb = tot[1];
            ks->tol2 = tol2;
            ks->iter = 0;
        }
        ks->rr = tot[0];
        ks->rr0 = tot[0];
        ks->rho = tot[0];
        ks->alpha = 1.0;
        ks->omega = 1.0;
        ks->done = (tot[0] <= ks->tol2 * ks->bb) ? 1 : 0;
    }
}

template <int DIM, typename T, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_kP(MeshDev m, KVec<T> V, int par, double* part, KState* ks) {
    if (ks->done) return;
    const double alpha = ks->alpha;
    double omega = 1.0, beta = 0.0, rho_new = ks->rho;
    if (!FIRST) {
        omega = ks->ts / ks->tt;
        rho_new = ks->rsv - omega * ks->rtv;
        beta = (rho_new / ks->rho) * (alpha / omega);
    }
    const T ta = (T)alpha, tw = (T)omega, tb = (T)beta;
    const T* __restrict__ s = V.s;
    const T* __restrict__ t = V.t;
    const T* __restrict__ po = V.p[par];
    const T* __restrict__ vo = V.v[par];
    T* __restrict__ pn = V.p[par ^ 1];
    T* __restrict__ vn = V.v[par ^ 1];
    double acc[2] = {0.0, 0.0};
    const int G = gridDim.x;
    const int lb = xcd_block(blockIdx.x, G);
    for (int c = lb * blockDim.x + threadIdx.x; c < m.Nc; c += G * blockDim.x) {
        T pc;
        T rc;
        if (FIRST) {
            rc = s[c];
            pc = rc;
        } else {
            rc = s[c] - tw * t[c];
            V.x[c] = V.x[c] + ta * po[c] + tw * s[c];
            pc = rc + tb * (po[c] - tw * vo[c]);
        }
        V.r[c] = rc;
        pn[c] = pc;
        T av;
        if (FIRST) {
            av = spmv_row<DIM, T>(m, V.A, c, [&](int j) { return s[j]; });
        } else {
            av = spmv_row<DIM, T>(m, V.A, c, [&](int j) {
                return (s[j] - tw * t[j]) + tb * (po[j] - tw * vo[j]);
            });
        }
        vn[c] = av;
        acc[0] += (double)V.rhat[c] * (double)av;
        acc[1] += (double)rc * (double)rc;
    }
    double tot[2];
    if (grid_reduce<2>(acc, part, ks, tot) && threadIdx.x == 0) {
        ks->rv = tot[0];
        ks->rr = tot[1];
        if (!FIRST) {
            ks->omega = omega;
            ks->rho = rho_new;
        }
        if (tot[1] <= ks->tol2 * ks->bb) {
            ks->done = 1;
        } else {
            const double a = rho_new / tot[0];
            const bool bad = !(tot[0] != 0.0) || !isfinite(a) || !isfinite(beta) ||
                             fabs(rho_new) < 1e-30 * ks->rr0;
            if (bad)
                ks->done = 2;
            else
                ks->alpha = a;
        }
    }
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_kS(MeshDev m, KVec<T> V, int par, double* part, KState* ks) {
    if (ks->done) return;
    const T ta = (T)ks->alpha;
    const T* __restrict__ r = V.r;
    const T* __restrict__ vn = V.v[par ^ 1];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int G = gridDim.x;
    const int lb = xcd_block(blockIdx.x, G);
    for (int c = lb * blockDim.x + threadIdx.x; c < m.Nc; c += G * blockDim.x) {
        const T sc = r[c] - ta * vn[c];
        const T tc = spmv_row<DIM, T>(m, V.A, c, [&](int j) { return r[j] - ta * vn[j]; });
        V.s[c] = sc;
        V.t[c] = tc;
        const double rh = (double)V.rhat[c];
        acc[0] += (double)tc * (double)sc;
        acc[1] += (double)tc * (double)tc;
        acc[2] += rh * (double)sc;
        acc[3] += rh * (double)tc;
    }
    double tot[4];
    if (grid_reduce<4>(acc, part, ks, tot) && threadIdx.x == 0) {
        ks->ts = tot[0];
        ks->tt = tot[1];
        ks->rsv = tot[2];
        ks->rtv = tot[3];
        ks->iter += 1;
        if (!(tot[1] > 0.0)) ks->done = 2;
    }
}

// b_eff = rhs - (Dirichlet columns) g - (Neumann rows) f at unknown rows; x0.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_ppe_rhs(MeshDev m, SetDev st, const double* __restrict__ rhs,
                                                    const double* __restrict__ g, const double* __restrict__ fneu,
                                                    int caller_guess, double* __restrict__ beff,
                                                    double* __restrict__ x0, int* bad) {
    constexpr int NB = Dims<DIM>::NB, S = Dims<DIM>::S, CEN = Dims<DIM>::CEN;
    const size_t Nc = (size_t)m.Nc;
    const double irs2 = 1.0 / (st.rs * st.rs);
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        if (!st.unknown[c]) {
            beff[c] = 0.0;
            x0[c] = 0.0;
            continue;
        }
        int ijk[3];
        cell_ijk(m, c, ijk);
        double acc = rhs[c];
        const uint32_t vm = st.vmask[c], nm = st.nmask[c];
        for (int s = 0; s < S; ++s) {
            if (s == CEN) continue;
            const bool v = (vm >> s) & 1u, n = fneu && ((nm >> s) & 1u);
            if (!v && !n) continue;
            int j;
            double sh[3];
            neighbour<DIM>(m, ijk, s, j, sh);
            double ph[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) ph[q] = st.phi[((size_t)q * (S + 1) + s) * Nc + c];
            const double lc = diag2<DIM>(ph) * irs2;
            if (v && !st.unknown[j]) acc -= lc * g[j];
            if (n) acc -= lc * fneu[j];
        }
        if (fneu && ((nm >> S) & 1u)) {
            double ph[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) ph[q] = st.phi[((size_t)q * (S + 1) + S) * Nc + c];
            acc -= diag2<DIM>(ph) * irs2 * fneu[c];
        }
        if (!isfinite(acc)) atomicAdd(bad, 1);
        beff[c] = acc;
        x0[c] = caller_guess ? g[c] : 0.0;
    }
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

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct KrylovWork {
    int Nc;
    int grid;
    double* part;          // [4][kMaxGrid]
    KState* ks;            // device
    KState* ks32;          // device (inner FP32 solve)
    KState* host;          // pinned [2]
    hipEvent_t ev[2];
    KVec<double> v64;
    KVec<float> v32;
    double* beff;
    float* b32;
    int* bad_host;         // pinned
    // optional timing of the stage kernels (events on the solve stream)
    int profile = 0;
    static constexpr int kProf = 4096;
    hipEvent_t pev[kProf][4];
    int pidx[kProf];       // global iteration index of the recorded launch pair
    int np = 0;
    double ms[2] = {0.0, 0.0};   // accumulated P, S milliseconds of working launches
    long long cnt[2] = {0, 0};
};

template <int DIM, typename T>
static hipError_t run_iterations(const MeshDev& m, KrylovWork& w, const KVec<T>& V, KState* ks, int budget,
                                 int check_every, hipStream_t st, int* iters_out, int* done_out) {
    // Pipelined chunks: chunk q+1 is enqueued before chunk q's state is
    // examined, so the GPU never waits for the host.  Kernels of a chunk
    // return at once when the state says done.
    int par = 0;
    bool first = true;
    int chunk = 0, last = -1, launched = 0;
    hipError_t e = hipSuccess;
    const int G = w.grid;
    const int iter0 = w.host[0].iter;   // state before this call (host copy is current)
    w.np = 0;
    while (budget > 0) {
        const int n = budget < check_every ? budget : check_every;
        budget -= n;
        for (int q = 0; q < n; ++q) {
            const bool rec = w.profile == 1 && w.np < KrylovWork::kProf;
            if (rec) {
                w.pidx[w.np] = iter0 + launched;
                (void)hipEventRecord(w.pev[w.np][0], st);
            }
            if (first)
                hipLaunchKernelGGL((k_kP<DIM, T, true>), dim3(G), dim3(kBlock), 0, st, m, V, par, w.part, ks);
            else
                hipLaunchKernelGGL((k_kP<DIM, T, false>), dim3(G), dim3(kBlock), 0, st, m, V, par, w.part, ks);
            if (rec) (void)hipEventRecord(w.pev[w.np][1], st);
            if (rec) (void)hipEventRecord(w.pev[w.np][2], st);
            hipLaunchKernelGGL((k_kS<DIM, T>), dim3(G), dim3(kBlock), 0, st, m, V, par, w.part, ks);
            if (rec) {
                (void)hipEventRecord(w.pev[w.np][3], st);
                ++w.np;
            }
            ++launched;
            first = false;
            par ^= 1;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(&w.host[chunk & 1], ks, sizeof(KState), hipMemcpyDeviceToHost, st)) != hipSuccess)
            return e;
        if ((e = hipEventRecord(w.ev[chunk & 1], st)) != hipSuccess) return e;
        last = chunk;
        if (chunk > 0) {
            if ((e = hipEventSynchronize(w.ev[(chunk - 1) & 1])) != hipSuccess) return e;
            if (w.host[(chunk - 1) & 1].done) break;
        }
        ++chunk;
    }
    if (last < 0) {
        *iters_out = 0;
        *done_out = 0;
        return hipSuccess;
    }
    if ((e = hipEventSynchronize(w.ev[last & 1])) != hipSuccess) return e;
    *iters_out = w.host[last & 1].iter;
    *done_out = w.host[last & 1].done;
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
        }
    }
    w.np = 0;
    return hipSuccess;
}

template <int DIM, typename T>
static hipError_t kinit(const MeshDev& m, KrylovWork& w, const KVec<T>& V, KState* ks, int with_bb, double tol2,
                        hipStream_t st, KState* out) {
    hipLaunchKernelGGL((k_kinit<DIM, T>), dim3(w.grid), dim3(kBlock), 0, st, m, V, w.part, ks, with_bb, tol2);
    hipError_t e = hipMemcpyAsync(&w.host[0], ks, sizeof(KState), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    *out = w.host[0];
    return hipGetLastError();
}

// Plain Bi-CGSTAB with restarts; returns iterations, restarts, rr/bb.
template <int DIM, typename T>
static hipError_t bicgstab(const MeshDev& m, KrylovWork& w, const KVec<T>& V, KState* ks, double tol, int max_iter,
                           int check_every, hipStream_t st, int* iters, int* restarts, double* rel, int* conv) {
    KState h;
    hipError_t e = kinit<DIM, T>(m, w, V, ks, 1, tol * tol, st, &h);
    if (e != hipSuccess) return e;
    *restarts = 0;
    *iters = 0;
    const double bb = h.bb;
    while (!h.done && h.iter < max_iter) {
        int it = 0, done = 0;
        if ((e = run_iterations<DIM, T>(m, w, V, ks, max_iter - h.iter, check_every, st, &it, &done)) != hipSuccess)
            return e;
        // confirm with the true residual; restarts from it if needed
        if ((e = kinit<DIM, T>(m, w, V, ks, 0, tol * tol, st, &h)) != hipSuccess) return e;
        h.iter = it;
        if (!h.done) *restarts += 1;
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
    if ((e = hipMemcpyAsync(w.bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    *out = SolveOut{};
    if (*w.bad_host) return hipSuccess;     // caller reports the non-finite input
    KVec<double> V = w.v64;
    V.A = set.amat;
    V.b = w.beff;
    const int check = sp.check_every > 0 ? sp.check_every : 8;
    if (sp.precision == MCD_PREC_FP64) {
        int it = 0, rst = 0, conv = 0;
        double rel = 0.0;
        if ((e = bicgstab<DIM, double>(m, w, V, w.ks, sp.tol, sp.max_iter, check, st, &it, &rst, &rel, &conv)) !=
            hipSuccess)
            return e;
        out->iterations = it;
        out->restarts = rst;
        out->converged = conv;
        out->rel = rel;
        out->bnorm = sqrt(w.host[0].bb);
    } else {
        // FP64 iterative refinement around an FP32 Bi-CGSTAB (FP64 dots)
        KVec<float> V32 = w.v32;
        V32.A = set.amat32;
        KState h;
        if ((e = kinit<DIM, double>(m, w, V, w.ks, 1, sp.tol * sp.tol, st, &h)) != hipSuccess) return e;
        const double bb = h.bb;
        int total = 0, outer = 0, rst_total = 0;
        while (!h.done && outer < sp.max_outer && total < sp.max_iter) {
            const double nr = sqrt(h.rr);
            hipLaunchKernelGGL(k_to32, dim3(g), dim3(kBlock), 0, st, m.Nc, V.s, 1.0 / nr, (float*)V32.b, V32.x);
            int it = 0, rst = 0, conv = 0;
            double rel = 0.0;
            if ((e = bicgstab<DIM, float>(m, w, V32, w.ks32, sp.inner_tol, sp.max_iter - total, check, st, &it, &rst,
                                          &rel, &conv)) != hipSuccess)
                return e;
            total += it;
            rst_total += rst;
            hipLaunchKernelGGL(k_refine, dim3(g), dim3(kBlock), 0, st, m.Nc, V32.x, nr, V.x);
            if ((e = kinit<DIM, double>(m, w, V, w.ks, 0, sp.tol * sp.tol, st, &h)) != hipSuccess) return e;
            ++outer;
        }
        out->iterations = total;
        out->restarts = rst_total;
        out->refinements = outer;
        out->converged = h.done == 1 || bb == 0.0;
        out->rel = bb > 0 ? sqrt(h.rr / bb) : 0.0;
        out->bnorm = sqrt(bb);
    }
    hipLaunchKernelGGL(k_writeback, dim3(g), dim3(kBlock), 0, st, m.Nc, set.unknown, V.x, p);
    return hipGetLastError();
}

hipError_t solve_ppe_impl(const MeshDev& m, const SetDev& set, KrylovWork& w, const double* rhs, const double* fneu,
                          double* p, const SolveParams& sp, SolveOut* out, int* bad, hipStream_t st) {
    return m.dim == 2 ? solve_dim<2>(m, set, w, rhs, fneu, p, sp, out, bad, st)
                      : solve_dim<3>(m, set, w, rhs, fneu, p, sp, out, bad, st);
}

template <typename T>
static hipError_t alloc_vec(KVec<T>& V, size_t Nc) {
    T** ptrs[9] = {&V.x, &V.r, &V.rhat, &V.s, &V.t, &V.p[0], &V.p[1], &V.v[0], &V.v[1]};
    for (T** q : ptrs) {
        hipError_t e = hipMalloc((void**)q, Nc * sizeof(T));
        if (e != hipSuccess) return e;
        if ((e = hipMemset(*q, 0, Nc * sizeof(T))) != hipSuccess) return e;
    }
    V.A = nullptr;
    V.b = nullptr;
    return hipSuccess;
}

template <typename T>
static void free_vec(KVec<T>& V) {
    T* ptrs[9] = {V.x, V.r, V.rhat, V.s, V.t, V.p[0], V.p[1], V.v[0], V.v[1]};
    for (T* q : ptrs)
        if (q) (void)hipFree(q);
}

hipError_t krylov_alloc(int Nc, KrylovWork** out) {
    KrylovWork* w = new KrylovWork{};
    *out = w;
    w->Nc = Nc;
    int g = (Nc + kBlock - 1) / kBlock;
    w->grid = g > kMaxGrid ? kMaxGrid : (g < 8 ? 8 : (g + 7) / 8 * 8);
    if (w->grid > kMaxGrid) w->grid = kMaxGrid;
    hipError_t e;
    if ((e = hipMalloc((void**)&w->part, 4 * kMaxGrid * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->ks, sizeof(KState))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->ks32, sizeof(KState))) != hipSuccess) return e;
    if ((e = hipMemset(w->ks, 0, sizeof(KState))) != hipSuccess) return e;
    if ((e = hipMemset(w->ks32, 0, sizeof(KState))) != hipSuccess) return e;
    if ((e = hipHostMalloc((void**)&w->host, 2 * sizeof(KState), hipHostMallocDefault)) != hipSuccess) return e;
    for (int i = 0; i < 2; ++i)
        if ((e = hipEventCreateWithFlags(&w->ev[i], hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = alloc_vec(w->v64, Nc)) != hipSuccess) return e;
    if ((e = alloc_vec(w->v32, Nc)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->beff, (size_t)Nc * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&w->b32, (size_t)Nc * sizeof(float))) != hipSuccess) return e;
    w->v32.b = w->b32;
    if ((e = hipHostMalloc((void**)&w->bad_host, sizeof(int), hipHostMallocDefault)) != hipSuccess) return e;
    return hipSuccess;
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

void krylov_profile_read(KrylovWork* w, double* ms_p, long long* n_p, double* ms_s, long long* n_s, int reset) {
    *ms_p = w->ms[0];
    *n_p = w->cnt[0];
    *ms_s = w->ms[1];
    *n_s = w->cnt[1];
    if (reset) {
        w->ms[0] = w->ms[1] = 0.0;
        w->cnt[0] = w->cnt[1] = 0;
    }
}

void krylov_free(KrylovWork* w) {
    if (!w) return;
    if (w->part) (void)hipFree(w->part);
    if (w->ks) (void)hipFree(w->ks);
    if (w->ks32) (void)hipFree(w->ks32);
    if (w->host) (void)hipHostFree(w->host);
    for (int i = 0; i < 2; ++i)
        if (w->ev[i]) (void)hipEventDestroy(w->ev[i]);
    free_vec(w->v64);
    free_vec(w->v32);
    if (w->beff) (void)hipFree(w->beff);
    if (w->b32) (void)hipFree(w->b32);
    if (w->bad_host) (void)hipHostFree(w->bad_host);
    if (w->profile)
        for (int k = 0; k < KrylovWork::kProf; ++k)
            for (int q = 0; q < 4; ++q) (void)hipEventDestroy(w->pev[k][q]);
    delete w;
}

}  // namespace mcd
