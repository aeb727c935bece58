// The PPE on a wider MLS support (Sec. 4, flow past stationary cylinders:
// the original 3x3 stencil against an expanded 9x9 one with r_e = 3.5 l0),
// 2D: the chi_c = 1 quadratic fit of Sec. 3.2 over the (2H+1)^2 block of
// cells around each DP, its Laplacian weights assembled into the PPE over the
// unknown DPs, and a plain Bi-CGSTAB (Sec. 3.3) on that operator.
//
// This is a comparison path, written for any half width H so that the same
// code runs the 3x3 (H = 1) and the 9x9 (H = 4) supports: one thread per DP
// with global gathers (no LDS tiles: an 81-slot row does not fit them), the
// matrix as S = (2H+1)^2 slot planes, and a Bi-CGSTAB whose scalars are
// formed on the host from fixed-order block partial sums after each
// reduction.  The production solver (the fused 3x3 stage kernels) is not
// used here.
#include <cmath>

#include "common.h"

namespace mcd {

namespace {

constexpr int kWBlock = 256;
constexpr int kWGrid = 1024;           // blocks of the reduction kernels (partials per quantity)

__device__ __forceinline__ double wide_weight(double r, double re, int kind) {
    if (r > re) return 0.0;
    if (kind == MCD_WEIGHT_COS2) {
        const double t = cos(M_PI * r / (2.0 * re));
        return t * t;
    }
    return exp(-4.0 * r * r / (re * re));
}

// cell of slot s of the (2H+1)^2 block around (i, j) with the periodic image
// shift of its position; false outside a non-periodic mesh
__device__ __forceinline__ bool wide_nbr(const MeshDev& m, int i, int j, int s, int H, int& c, double sh[2]) {
    const int W = 2 * H + 1;
    int ii = i + s % W - H, jj = j + s / W - H;
    sh[0] = sh[1] = 0.0;
    if (ii < 0 || ii >= m.n[0]) {
        if (!m.periodic[0]) return false;
        const int w = ii < 0 ? -1 : 1;
        ii -= w * m.n[0];
        sh[0] = w * m.length[0];
    }
    if (jj < 0 || jj >= m.n[1]) {
        if (!m.periodic[1]) return false;
        const int w = jj < 0 ? -1 : 1;
        jj -= w * m.n[1];
        sh[1] = w * m.length[1];
    }
    c = ii + m.n[0] * jj;
    return true;
}

// row of slot s for DP c: kind (0 none, 1 value, 2 Neumann), weight and basis row
__device__ __forceinline__ int wide_row(const MeshDev& m, const double* __restrict__ pos, const int8_t* __restrict__ role,
                                        const double* __restrict__ normal, const BcDev& bc, int c, int i, int j, int s,
                                        int H, double re, double rs, int wkind, double& w, double a[5]) {
    const size_t Nc = (size_t)m.Nc;
    int nb;
    double sh[2];
    if (!wide_nbr(m, i, j, s, H, nb, sh)) return 0;
    int kind = row_kind(role[nb], bc);
    const int W = 2 * H + 1;
    if (s == (W * W - 1) / 2 && kind != 2) return 0;      // the DP itself: only its Neumann row
    if (kind == 0) return 0;
    double X[2];
    double r2 = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double d = (pos[q * Nc + nb] + sh[q]) - pos[q * Nc + c];
        r2 += d * d;
        X[q] = d / rs;
    }
    w = wide_weight(sqrt(r2), re, wkind);
    if (kind == 1) {
        basis<2>(X, a);
    } else {
        const double nv[2] = {normal[nb], normal[Nc + nb]};
        basis_normal<2>(X, nv, a);
    }
    return kind;
}

// Laplacian weights per slot (planes lc[S+1][Nc]; slot S is the DP's own
// Neumann row) of every active DP; singular fits get zero weights.
__global__ __launch_bounds__(kWBlock) void k_wide_lap(MeshDev m, const double* __restrict__ pos,
                                                      const int8_t* __restrict__ role, const double* __restrict__ normal,
                                                      BcDev bc, int H, double re, double rs, int wkind,
                                                      double* __restrict__ lc, int* __restrict__ nsing) {
    const int W = 2 * H + 1, S = W * W, CEN = (S - 1) / 2;
    const size_t Nc = (size_t)m.Nc;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        for (int s = 0; s <= S; ++s) lc[(size_t)s * Nc + c] = 0.0;
        if (role[c] == MCD_ROLE_VOID) continue;
        const int i = c % m.n[0], j = c / m.n[0];
        double M[15];
#pragma unroll
        for (int q = 0; q < 15; ++q) M[q] = 0.0;
        int nrows = 0;
        for (int s = 0; s < S; ++s) {
            double w = 0.0, a[5];
            if (!wide_row(m, pos, role, normal, bc, c, i, j, s, H, re, rs, wkind, w, a)) continue;
            if (w > 0.0) ++nrows;
            int q = 0;
#pragma unroll
            for (int r = 0; r < 5; ++r)
#pragma unroll
                for (int k = 0; k <= r; ++k) M[q++] += w * a[r] * a[k];
        }
        // Cholesky M = L L^T (packed lower triangle, in place)
        double tr = 0.0;
#pragma unroll
        for (int r = 0; r < 5; ++r) tr += M[r * (r + 1) / 2 + r];
        bool singular = nrows < 5;
#pragma unroll
        for (int col = 0; col < 5; ++col) {
            double d = M[col * (col + 1) / 2 + col];
#pragma unroll
            for (int k = 0; k < col; ++k) d -= M[col * (col + 1) / 2 + k] * M[col * (col + 1) / 2 + k];
            if (d <= 1e-12 * tr / 5.0) {
                singular = true;
                d = 1.0;
            }
            const double l = sqrt(d);
            M[col * (col + 1) / 2 + col] = l;
#pragma unroll
            for (int r = col + 1; r < 5; ++r) {
                double acc = M[r * (r + 1) / 2 + col];
#pragma unroll
                for (int k = 0; k < col; ++k) acc -= M[r * (r + 1) / 2 + k] * M[col * (col + 1) / 2 + k];
                M[r * (r + 1) / 2 + col] = acc / l;
            }
        }
        if (singular) {
            // zero weights; counted when the DP's PPE row is needed (wall corners
            // with too few rows are not unknowns)
            if (is_unknown(role[c], c, bc)) atomicAdd(nsing, 1);
            continue;
        }
        double centre = 0.0;
        for (int s = 0; s < S; ++s) {
            double w = 0.0, a[5];
            const int kind = wide_row(m, pos, role, normal, bc, c, i, j, s, H, re, rs, wkind, w, a);
            if (!kind) continue;
            double z[5];
#pragma unroll
            for (int r = 0; r < 5; ++r) {
                double acc = w * a[r];
#pragma unroll
                for (int k = 0; k < r; ++k) acc -= M[r * (r + 1) / 2 + k] * z[k];
                z[r] = acc / M[r * (r + 1) / 2 + r];
            }
#pragma unroll
            for (int r = 4; r >= 0; --r) {
                double acc = z[r];
#pragma unroll
                for (int k = r + 1; k < 5; ++k) acc -= M[k * (k + 1) / 2 + r] * z[k];
                z[r] = acc / M[r * (r + 1) / 2 + r];
            }
            const double lap = (z[2] + z[4]) / (rs * rs);
            if (s == CEN) {
                lc[(size_t)S * Nc + c] = lap * rs;          // own Neumann row: coefficient of f_c
            } else if (kind == 2) {
                lc[(size_t)s * Nc + c] = lap * rs;          // coefficient of f_j
            } else {
                lc[(size_t)s * Nc + c] = lap;               // coefficient of (P_j - P_c)
                centre -= lap;
            }
        }
        lc[(size_t)CEN * Nc + c] = centre;
    }
}

// PPE rows over the unknown DPs (Eq. pressure_poisson): sum over value rows
// of L_j (P_j - P_c) + Neumann terms = rhs_c, known columns (Dirichlet,
// pinned) moved to the right side with their values g = p, Neumann data f
// too.  Rows of other DPs are the identity with a zero right side.
__global__ __launch_bounds__(kWBlock) void k_wide_assemble(MeshDev m, const int8_t* __restrict__ role, BcDev bc, int H,
                                                           const double* __restrict__ lc, const double* __restrict__ rhs,
                                                           const double* __restrict__ g, const double* __restrict__ f,
                                                           double* __restrict__ A, double* __restrict__ b,
                                                           uint8_t* __restrict__ unk) {
    const int W = 2 * H + 1, S = W * W, CEN = (S - 1) / 2;
    const size_t Nc = (size_t)m.Nc;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const bool u = is_unknown(role[c], c, bc);
        unk[c] = u ? 1 : 0;
        for (int s = 0; s < S; ++s) A[(size_t)s * Nc + c] = 0.0;
        if (!u) {
            A[(size_t)CEN * Nc + c] = 1.0;
            b[c] = 0.0;
            continue;
        }
        const int i = c % m.n[0], j = c / m.n[0];
        double beff = rhs[c], diag = 0.0;
        for (int s = 0; s < S; ++s) {
            if (s == CEN) continue;
            int nb;
            double sh[2];
            if (!wide_nbr(m, i, j, s, H, nb, sh)) continue;
            const int kind = row_kind(role[nb], bc);
            const double cj = lc[(size_t)s * Nc + c];
            if (kind == 1) {
                diag -= cj;
                if (is_unknown(role[nb], nb, bc))
                    A[(size_t)s * Nc + c] = cj;
                else
                    beff -= cj * g[nb];
            } else if (kind == 2 && f) {
                beff -= cj * f[nb];
            }
        }
        if (f && row_kind(role[c], bc) == 2) beff -= lc[(size_t)S * Nc + c] * f[c];
        A[(size_t)CEN * Nc + c] = diag;
        b[c] = beff;
    }
}

// y = A x over the slot planes
__device__ __forceinline__ double wide_row_product(const MeshDev& m, const double* __restrict__ A,
                                                   const double* __restrict__ x, int c, int H) {
    const int W = 2 * H + 1, S = W * W;
    const size_t Nc = (size_t)m.Nc;
    const int i = c % m.n[0], j = c / m.n[0];
    double acc = 0.0;
    for (int s = 0; s < S; ++s) {
        const double a = A[(size_t)s * Nc + c];
        if (a == 0.0) continue;
        int nb;
        double sh[2];
        if (!wide_nbr(m, i, j, s, H, nb, sh)) continue;
        acc += a * x[nb];
    }
    return acc;
}

template <int NQ>
__device__ __forceinline__ void wide_partials(double (&v)[NQ], double* part) {
    __shared__ double lds[NQ][kWBlock / 64];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double s = wave_sum(v[q]);
        if ((threadIdx.x & 63) == 0) lds[q][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double s = 0.0;
            for (int w = 0; w < kWBlock / 64; ++w) s += lds[q][w];
            part[q * kWGrid + blockIdx.x] = s;
        }
    }
}

// r = b - A x (unknown rows), rhat = r; partials r.r, b.b
__global__ __launch_bounds__(kWBlock) void k_wide_init(MeshDev m, int H, const double* __restrict__ A,
                                                       const double* __restrict__ b, const double* __restrict__ x,
                                                       const uint8_t* __restrict__ unk, double* __restrict__ r,
                                                       double* __restrict__ rhat, double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const double rc = unk[c] ? b[c] - wide_row_product(m, A, x, c, H) : 0.0;
        r[c] = rc;
        rhat[c] = rc;
        v[0] += rc * rc;
        v[1] += unk[c] ? b[c] * b[c] : 0.0;
    }
    wide_partials<2>(v, part);
}

// p = r + beta (p - omega v); v = A p needs p complete, so this is its own pass
__global__ __launch_bounds__(kWBlock) void k_wide_p(int Nc, double beta, double omega, const double* __restrict__ r,
                                                    const double* __restrict__ v, double* __restrict__ p) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x)
        p[c] = r[c] + beta * (p[c] - omega * v[c]);
}

// y = A x on unknown rows (0 elsewhere); partials rhat.y
__global__ __launch_bounds__(kWBlock) void k_wide_spmv_dot(MeshDev m, int H, const double* __restrict__ A,
                                                           const double* __restrict__ x, const uint8_t* __restrict__ unk,
                                                           const double* __restrict__ rhat, double* __restrict__ y,
                                                           double* __restrict__ part) {
    double v[1] = {0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const double yc = unk[c] ? wide_row_product(m, A, x, c, H) : 0.0;
        y[c] = yc;
        v[0] += rhat[c] * yc;
    }
    wide_partials<1>(v, part);
}

// s = r - alpha v
__global__ __launch_bounds__(kWBlock) void k_wide_s(int Nc, double alpha, const double* __restrict__ r,
                                                    const double* __restrict__ v, double* __restrict__ s) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x) s[c] = r[c] - alpha * v[c];
}

// t = A s; partials t.s, t.t
__global__ __launch_bounds__(kWBlock) void k_wide_t(MeshDev m, int H, const double* __restrict__ A,
                                                    const double* __restrict__ s, const uint8_t* __restrict__ unk,
                                                    double* __restrict__ t, double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m.Nc; c += gridDim.x * blockDim.x) {
        const double tc = unk[c] ? wide_row_product(m, A, s, c, H) : 0.0;
        t[c] = tc;
        v[0] += tc * s[c];
        v[1] += tc * tc;
    }
    wide_partials<2>(v, part);
}

// x += alpha p + omega s; r = s - omega t; partials rhat.r, r.r
__global__ __launch_bounds__(kWBlock) void k_wide_xr(int Nc, double alpha, double omega, const double* __restrict__ p,
                                                     const double* __restrict__ s, const double* __restrict__ t,
                                                     const double* __restrict__ rhat, double* __restrict__ x,
                                                     double* __restrict__ r, double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x) {
        x[c] = x[c] + alpha * p[c] + omega * s[c];
        const double rc = s[c] - omega * t[c];
        r[c] = rc;
        v[0] += rhat[c] * rc;
        v[1] += rc * rc;
    }
    wide_partials<2>(v, part);
}

__global__ void k_wide_fill(int n, double v, double* __restrict__ x) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) x[c] = v;
}

// x (all cells) <- p at unknown rows, 0 elsewhere; after the solve p <- x at unknown rows
__global__ void k_wide_gather(int Nc, const uint8_t* __restrict__ unk, const double* __restrict__ p,
                              double* __restrict__ x) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x) x[c] = unk[c] ? p[c] : 0.0;
}
__global__ void k_wide_scatter(int Nc, const uint8_t* __restrict__ unk, const double* __restrict__ x,
                               double* __restrict__ p) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x)
        if (unk[c]) p[c] = x[c];
}

}  // namespace

struct WideWork {
    int H = 0;
    size_t Nc = 0;
    double *lc = nullptr, *A = nullptr, *b = nullptr;
    double *x = nullptr, *r = nullptr, *rhat = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *t = nullptr;
    double* part = nullptr;      // [2][kWGrid]
    double* host = nullptr;      // pinned [2][kWGrid]
    uint8_t* unk = nullptr;
    int* nsing = nullptr;
};

void wide_free(WideWork* w) {
    if (!w) return;
    void* ptrs[] = {w->lc, w->A, w->b, w->x, w->r, w->rhat, w->p, w->v, w->s, w->t, w->part, w->unk, w->nsing};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (w->host) (void)hipHostFree(w->host);
    delete w;
}

static hipError_t wide_alloc(WideWork** out, int H, size_t Nc) {
    WideWork* w = new WideWork();
    w->H = H;
    w->Nc = Nc;
    const size_t S = (size_t)(2 * H + 1) * (2 * H + 1);
    hipError_t e = hipMalloc((void**)&w->lc, (S + 1) * Nc * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&w->A, S * Nc * sizeof(double));
    double** vecs[] = {&w->b, &w->x, &w->r, &w->rhat, &w->p, &w->v, &w->s, &w->t};
    for (double** q : vecs)
        if (e == hipSuccess) e = hipMalloc((void**)q, Nc * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&w->part, 2 * kWGrid * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&w->host, 2 * kWGrid * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&w->unk, Nc);
    if (e == hipSuccess) e = hipMalloc((void**)&w->nsing, sizeof(int));
    if (e != hipSuccess) {
        wide_free(w);
        return e;
    }
    *out = w;
    return hipSuccess;
}

// fixed-order sums of NQ partial arrays (copied to pinned memory)
static hipError_t wide_sums(WideWork& w, int nq, double* out, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(w.host, w.part, (size_t)nq * kWGrid * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int q = 0; q < nq; ++q) {
        double s = 0.0;
        for (int k = 0; k < kWGrid; ++k) s += w.host[q * kWGrid + k];
        out[q] = s;
    }
    return hipSuccess;
}

hipError_t wide_ppe(const MeshDev& m, WideWork** slot, int H, double re, double rs, int wkind, const double* pos,
                    const int8_t* role, const double* normal, const BcDev& bc, const double* rhs, const double* f,
                    double* p, double tol, int max_iter, WideResult* res, hipStream_t st) {
    const size_t Nc = (size_t)m.Nc;
    hipError_t e = hipSuccess;
    if (!*slot || (*slot)->H != H || (*slot)->Nc != Nc) {
        wide_free(*slot);
        *slot = nullptr;
        if ((e = wide_alloc(slot, H, Nc)) != hipSuccess) return e;
    }
    WideWork& w = **slot;
    const int g = kWGrid;
    hipEvent_t ev[3];
    for (int k = 0; k < 3; ++k)
        if ((e = hipEventCreate(&ev[k])) != hipSuccess) return e;
    *res = WideResult{};
    double rho_prev = 1.0;
    e = hipMemsetAsync(w.nsing, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipEventRecord(ev[0], st);
    if (e != hipSuccess) goto done;
    hipLaunchKernelGGL(k_wide_lap, dim3(g), dim3(kWBlock), 0, st, m, pos, role, normal, bc, H, re, rs, wkind, w.lc,
                       w.nsing);
    hipLaunchKernelGGL(k_wide_assemble, dim3(g), dim3(kWBlock), 0, st, m, role, bc, H, w.lc, rhs, p, f, w.A, w.b,
                       w.unk);
    if ((e = hipGetLastError()) != hipSuccess) goto done;
    if ((e = hipEventRecord(ev[1], st)) != hipSuccess) goto done;
    {
        const int n = (int)Nc;
        hipLaunchKernelGGL(k_wide_gather, dim3(g), dim3(kWBlock), 0, st, n, w.unk, p, w.x);
        hipLaunchKernelGGL(k_wide_init, dim3(g), dim3(kWBlock), 0, st, m, H, w.A, w.b, w.x, w.unk, w.r, w.rhat, w.part);
        double sums[2];
        if ((e = wide_sums(w, 2, sums, st)) != hipSuccess) goto done;
        double rr = sums[0];
        const double bb = sums[1];
        const double stop = tol * tol * bb;
        double rho = rr, alpha = 1.0, omega = 1.0;
        hipLaunchKernelGGL(k_wide_fill, dim3(g), dim3(kWBlock), 0, st, n, 0.0, w.p);
        hipLaunchKernelGGL(k_wide_fill, dim3(g), dim3(kWBlock), 0, st, n, 0.0, w.v);
        int it = 0;
        bool conv = rr <= stop;
        while (!conv && it < max_iter) {
            const double beta = it == 0 ? 0.0 : (rho / rho_prev) * (alpha / omega);
            hipLaunchKernelGGL(k_wide_p, dim3(g), dim3(kWBlock), 0, st, n, beta, omega, w.r, w.v, w.p);
            hipLaunchKernelGGL(k_wide_spmv_dot, dim3(g), dim3(kWBlock), 0, st, m, H, w.A, w.p, w.unk, w.rhat, w.v,
                               w.part);
            double rv;
            if ((e = wide_sums(w, 1, &rv, st)) != hipSuccess) goto done;
            alpha = rho / rv;
            hipLaunchKernelGGL(k_wide_s, dim3(g), dim3(kWBlock), 0, st, n, alpha, w.r, w.v, w.s);
            hipLaunchKernelGGL(k_wide_t, dim3(g), dim3(kWBlock), 0, st, m, H, w.A, w.s, w.unk, w.t, w.part);
            double ts[2];
            if ((e = wide_sums(w, 2, ts, st)) != hipSuccess) goto done;
            omega = ts[1] > 0.0 ? ts[0] / ts[1] : 0.0;
            hipLaunchKernelGGL(k_wide_xr, dim3(g), dim3(kWBlock), 0, st, n, alpha, omega, w.p, w.s, w.t, w.rhat, w.x,
                               w.r, w.part);
            double q2[2];
            if ((e = wide_sums(w, 2, q2, st)) != hipSuccess) goto done;
            rho_prev = rho;
            rho = q2[0];
            rr = q2[1];
            ++it;
            if (!std::isfinite(rr) || omega == 0.0 || !std::isfinite(alpha)) break;
            conv = rr <= stop;
        }
        // true residual of the result
        hipLaunchKernelGGL(k_wide_init, dim3(g), dim3(kWBlock), 0, st, m, H, w.A, w.b, w.x, w.unk, w.r, w.rhat,
                           w.part);
        if ((e = wide_sums(w, 2, sums, st)) != hipSuccess) goto done;
        hipLaunchKernelGGL(k_wide_scatter, dim3(g), dim3(kWBlock), 0, st, n, w.unk, w.x, p);
        if ((e = hipEventRecord(ev[2], st)) != hipSuccess) goto done;
        if ((e = hipEventSynchronize(ev[2])) != hipSuccess) goto done;
        res->iterations = it;
        res->true_rel_residual = bb > 0.0 ? sqrt(sums[0] / bb) : 0.0;
        res->converged = res->true_rel_residual <= tol ? 1 : 0;
        float ms0 = 0.f, ms1 = 0.f;
        (void)hipEventElapsedTime(&ms0, ev[0], ev[1]);
        (void)hipEventElapsedTime(&ms1, ev[1], ev[2]);
        res->build_ms = ms0;
        res->solve_ms = ms1;
        int ns = 0;
        if ((e = hipMemcpy(&ns, w.nsing, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess) goto done;
        res->singular = ns;
    }
done:
    for (int k = 0; k < 3; ++k) (void)hipEventDestroy(ev[k]);
    return e;
}

hipError_t wide_lap_planes(const WideWork* w, double* out, hipStream_t st) {
    if (!w) return hipErrorInvalidValue;
    const size_t S = (size_t)(2 * w->H + 1) * (2 * w->H + 1);
    return hipMemcpyAsync(out, w->A, S * w->Nc * sizeof(double), hipMemcpyDeviceToDevice, st);
}

}  // namespace mcd
