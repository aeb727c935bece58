// Internal definitions shared by the libmcd HIP sources (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcd.h"

namespace mcd {

constexpr int kBlock = 256;          // 4 wave64 per block
constexpr int kMaxBodies = MCD_MAX_BODIES;

struct MeshDev {
    int dim;
    int n[3];
    int Nc;
    double origin[3];
    double l0;
    int periodic[3];
    double length[3];   // n[a] * l0
    int walls;
    int wall_id;
    // Element stride between the slot planes of the PPE matrix (and between
    // the Krylov vectors of one precision): Nc rounded up to 64 plus 576, so
    // that planes do not start a power of two apart, which puts the same cell
    // of every plane on the same HBM channel.
    size_t mps;
};

// Stride of the padded planes for a mesh of Nc cells (see MeshDev::mps).
inline size_t padded_plane_stride(size_t Nc) { return (Nc + 63) / 64 * 64 + 576; }

// Load of a matrix entry that is read once per stage launch: non-temporal, so
// that the streamed matrix does not evict the vectors whose tile halos other
// blocks re-read from cache.
template <typename TA>
__device__ __forceinline__ TA ld_stream(const TA* p) {
    return __builtin_nontemporal_load(p);
}

// Load of a matrix entry that iterative solvers read once per iteration:
// non-temporal (NT) when the matrix and vectors of an iteration exceed the
// last-level cache, so that the streamed matrix does not evict the vectors;
// plain otherwise, so that the matrix stays in cache from one iteration to
// the next.
template <bool NT, typename TA>
__device__ __forceinline__ TA ld_mat(const TA* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// The last-level cache (256 MB on the MI355X) holds an iteration's data when
// they stay below this.
constexpr size_t kCacheFitBytes = 192u << 20;

struct BodiesDev {
    int n;
    int id[kMaxBodies];
    double c[kMaxBodies][3];
    double R[kMaxBodies];
    double R2[kMaxBodies];      // R * R computed on the host
    double vel[kMaxBodies][3];
    double dvdt[kMaxBodies][3];
    double om[kMaxBodies][3];   // angular velocity
    double dom[kMaxBodies][3];  // its backward difference over dt
    int rot[kMaxBodies];        // omega or domega non-zero
    int any_rot;
    // discrete SDF bodies (Sec. 2.5); sdf[k] == nullptr: circle/sphere
    const double* sdf[kMaxBodies];
    int sn[kMaxBodies][3];
    double so[kMaxBodies][3];
    double sh[kMaxBodies];
    double cth[kMaxBodies], sth[kMaxBodies];   // 2D posture
    double post[kMaxBodies][9];                // 3D posture R (row-major): x = c + R xi
    double far2[kMaxBodies];
    // 3D closed form over the 3x3x3 nodes: weights of face, edge and corner
    // nodes; D1 = sum w X^2, DX = sum w X^2 Y^2; the diagonal quadratic block
    // is (A - B) I + B 11^T with A = D1 / 4, B = DX / 4
    double s3w[3];
    double s3D1, s3DX, s3A, s3B;
    // chi_c = 1 quadratic MLS over the 3x3 SDF nodes in closed form (the grid
    // is regular and symmetric, so the normal equations decouple):
    // g_q = sum_k sdfc[q][k] (psi_k - psi_centre) with sdfc = w_k p_q(X_k)
    // (exact: X, Y in {-1, 0, 1}), then Phi_X = g_0 / D1, Phi_Y = g_1 / D1,
    // Phi_XY = g_3 / D3 and the (X^2/2, Y^2/2) pair from its 2x2 block
    // [[A, B], [B, A]]; neighbours k in row order without the centre
    double sdfc[5][8];
    double sdfD1, sdfD3, sdfA, sdfB, sdfDet;
};

// psi and grad psi of discrete-SDF body b at the 2D point (x0, x1): the point
// in the body frame, xi = R(-theta)(x - c); the 3x3 nodes around the nearest
// node (kept one node inside the grid); psi = psi_s + p(s).Phi with s the
// offset from that node in units of h; the gradient rotated back.  Beyond
// the far radius: the bounding disc, psi = |x - c| - R.  Every operation is
// rounded on its own (no contraction), in a fixed order, so that the result
// is reproducible bit for bit by a plain evaluation of the same formulas.
__device__ __forceinline__ double sdf_psi(const BodiesDev& B, int b, double x0, double x1, double* g) {
#pragma clang fp contract(off)
    const double d0 = x0 - B.c[b][0], d1 = x1 - B.c[b][1];
    const double r2 = d0 * d0 + d1 * d1;
    if (r2 >= B.far2[b]) {
        const double r = sqrt(r2);
        g[0] = d0 / r;
        g[1] = d1 / r;
        return r - B.R[b];
    }
    const double ct = B.cth[b], st = B.sth[b], h = B.sh[b];
    const double xi0 = ct * d0 + st * d1, xi1 = ct * d1 - st * d0;
    const double q0 = (xi0 - B.so[b][0]) / h, q1 = (xi1 - B.so[b][1]) / h;
    const int n0 = B.sn[b][0], n1 = B.sn[b][1];
    int i = (int)floor(q0 + 0.5), j = (int)floor(q1 + 0.5);
    i = i < 1 ? 1 : (i > n0 - 2 ? n0 - 2 : i);
    j = j < 1 ? 1 : (j > n1 - 2 ? n1 - 2 : j);
    const double s0 = q0 - (double)i, s1 = q1 - (double)j;
    const double* __restrict__ S = B.sdf[b];
    const double ps = S[(size_t)j * n0 + i];
    double gq[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int k = 0;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
            if (di == 0 && dj == 0) continue;
            const double dv = S[(size_t)(j + dj) * n0 + (i + di)] - ps;
#pragma unroll
            for (int q = 0; q < 5; ++q) gq[q] = gq[q] + B.sdfc[q][k] * dv;
            ++k;
        }
    const double P0 = gq[0] / B.sdfD1, P1 = gq[1] / B.sdfD1, P3 = gq[3] / B.sdfD3;
    const double P2 = (B.sdfA * gq[2] - B.sdfB * gq[4]) / B.sdfDet;
    const double P4 = (B.sdfA * gq[4] - B.sdfB * gq[2]) / B.sdfDet;
    const double psi = ps + (s0 * P0 + s1 * P1 + 0.5 * s0 * s0 * P2 + s0 * s1 * P3 + 0.5 * s1 * s1 * P4);
    const double gx = (P0 + s0 * P2 + s1 * P3) / h;
    const double gy = (P1 + s0 * P3 + s1 * P4) / h;
    g[0] = ct * gx - st * gy;
    g[1] = st * gx + ct * gy;
    return psi;
}

// 3D: the same rule over the 3x3x3 nodes, basis (X, Y, Z, X^2/2, Y^2/2,
// Z^2/2, XY, YZ, ZX); on the symmetric support the linear and mixed terms
// decouple (denominators D1 and DX) and the three squares solve
// ((A - B) I + B 11^T) Phi = g, i.e. Phi_q = (g_q - B (g_0 + g_1 + g_2) /
// (A + 2B)) / (A - B).  Node factors w_k p_q(X_k) are exact.
__device__ __forceinline__ double sdf_psi3(const BodiesDev& B, int b, const double* x, double* g) {
#pragma clang fp contract(off)
    const double d0 = x[0] - B.c[b][0], d1 = x[1] - B.c[b][1], d2 = x[2] - B.c[b][2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (r2 >= B.far2[b]) {
        const double r = sqrt(r2);
        g[0] = d0 / r;
        g[1] = d1 / r;
        g[2] = d2 / r;
        return r - B.R[b];
    }
    const double* R = B.post[b];
    const double h = B.sh[b];
    // xi = R^T d
    const double xi0 = R[0] * d0 + R[3] * d1 + R[6] * d2;
    const double xi1 = R[1] * d0 + R[4] * d1 + R[7] * d2;
    const double xi2 = R[2] * d0 + R[5] * d1 + R[8] * d2;
    const double q0 = (xi0 - B.so[b][0]) / h, q1 = (xi1 - B.so[b][1]) / h, q2 = (xi2 - B.so[b][2]) / h;
    const int n0 = B.sn[b][0], n1 = B.sn[b][1], n2 = B.sn[b][2];
    int i = (int)floor(q0 + 0.5), j = (int)floor(q1 + 0.5), l = (int)floor(q2 + 0.5);
    i = i < 1 ? 1 : (i > n0 - 2 ? n0 - 2 : i);
    j = j < 1 ? 1 : (j > n1 - 2 ? n1 - 2 : j);
    l = l < 1 ? 1 : (l > n2 - 2 ? n2 - 2 : l);
    const double s0 = q0 - (double)i, s1 = q1 - (double)j, s2 = q2 - (double)l;
    const double* __restrict__ S = B.sdf[b];
    const size_t n01 = (size_t)n0 * n1;
    const double ps = S[(size_t)l * n01 + (size_t)j * n0 + i];
    double gq[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk)
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
            for (int di = -1; di <= 1; ++di) {
                const int nz = (di != 0) + (dj != 0) + (dk != 0);
                if (nz == 0) continue;
                const double w = B.s3w[nz - 1];
                const double X = di, Y = dj, Z = dk;
                const double dv = S[(size_t)(l + dk) * n01 + (size_t)(j + dj) * n0 + (i + di)] - ps;
                gq[0] = gq[0] + (w * X) * dv;
                gq[1] = gq[1] + (w * Y) * dv;
                gq[2] = gq[2] + (w * Z) * dv;
                gq[3] = gq[3] + (w * (0.5 * X * X)) * dv;
                gq[4] = gq[4] + (w * (0.5 * Y * Y)) * dv;
                gq[5] = gq[5] + (w * (0.5 * Z * Z)) * dv;
                gq[6] = gq[6] + (w * (X * Y)) * dv;
                gq[7] = gq[7] + (w * (Y * Z)) * dv;
                gq[8] = gq[8] + (w * (Z * X)) * dv;
            }
    const double P0 = gq[0] / B.s3D1, P1 = gq[1] / B.s3D1, P2 = gq[2] / B.s3D1;
    const double tq = B.s3B * (gq[3] + gq[4] + gq[5]) / (B.s3A + 2.0 * B.s3B);
    const double amb = B.s3A - B.s3B;
    const double P3 = (gq[3] - tq) / amb, P4 = (gq[4] - tq) / amb, P5 = (gq[5] - tq) / amb;
    const double P6 = gq[6] / B.s3DX, P7 = gq[7] / B.s3DX, P8 = gq[8] / B.s3DX;
    const double psi = ps + (s0 * P0 + s1 * P1 + s2 * P2 + 0.5 * s0 * s0 * P3 + 0.5 * s1 * s1 * P4 +
                             0.5 * s2 * s2 * P5 + s0 * s1 * P6 + s1 * s2 * P7 + s2 * s0 * P8);
    const double gx = (P0 + s0 * P3 + s1 * P6 + s2 * P8) / h;
    const double gy = (P1 + s1 * P4 + s0 * P6 + s2 * P7) / h;
    const double gz = (P2 + s2 * P5 + s1 * P7 + s0 * P8) / h;
    // g = R g_xi
    g[0] = R[0] * gx + R[1] * gy + R[2] * gz;
    g[1] = R[3] * gx + R[4] * gy + R[5] * gz;
    g[2] = R[6] * gx + R[7] * gy + R[8] * gz;
    return psi;
}

// psi and grad psi of discrete-SDF body b at the point x of a DIM mesh
template <int DIM>
__device__ __forceinline__ double sdf_eval(const BodiesDev& B, int b, const double* x, double* g) {
    if constexpr (DIM == 2)
        return sdf_psi(B, b, x[0], x[1], g);
    else
        return sdf_psi3(B, b, x, g);
}

// Velocity of a body point x (Eq. velocity_moving_boundary): V_trans + omega x r,
// r = x - centre.  A body without rotation returns V_trans untouched.
template <int DIM>
__device__ __forceinline__ void body_velocity(const BodiesDev& B, int b, const double* __restrict__ pos,
                                              size_t Nc, int c, double v[DIM]) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) v[a] = B.vel[b][a];
    if (!B.rot[b]) return;
    double r[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) r[a] = pos[a * Nc + c] - B.c[b][a];
    const double* w = B.om[b];
    const double x[3] = {w[1] * r[2] - w[2] * r[1], w[2] * r[0] - w[0] * r[2], w[0] * r[1] - w[1] * r[0]};
#pragma unroll
    for (int a = 0; a < DIM; ++a) v[a] += x[a];
}

// dV/dt . n at a body point (Eq. dvdt_moving_boundary):
// (dV_trans/dt + domega x r + omega x (omega x r)) . n.
template <int DIM>
__device__ __forceinline__ double body_accel_dot_n(const BodiesDev& B, int b, const double* __restrict__ pos,
                                                   const double* __restrict__ normal, size_t Nc, int c) {
    double acc = 0.0;
    if (!B.rot[b]) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) acc += B.dvdt[b][a] * normal[a * Nc + c];
        return acc;
    }
    double r[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) r[a] = pos[a * Nc + c] - B.c[b][a];
    const double* w = B.om[b];
    const double* g = B.dom[b];
    const double wr[3] = {w[1] * r[2] - w[2] * r[1], w[2] * r[0] - w[0] * r[2], w[0] * r[1] - w[1] * r[0]};
    const double gr[3] = {g[1] * r[2] - g[2] * r[1], g[2] * r[0] - g[0] * r[2], g[0] * r[1] - g[1] * r[0]};
    const double wwr[3] = {w[1] * wr[2] - w[2] * wr[1], w[2] * wr[0] - w[0] * wr[2], w[0] * wr[1] - w[1] * wr[0]};
#pragma unroll
    for (int a = 0; a < DIM; ++a) acc += (B.dvdt[b][a] + gr[a] + wwr[a]) * normal[a * Nc + c];
    return acc;
}

struct BcDev {
    int type[MCD_MAX_IDS];
    int pin_first;
};

// Storage of one stencil set (weight and matrix planes at the padded plane
// stride MeshDev::mps; per-cell arrays [Nc]).
struct SetDev {
    double* phi;        // [nb][S+1][mps]
    uint32_t* vmask;    // [Nc] bit s: slot s is a value row
    uint32_t* nmask;    // [Nc] bit s: slot s is a Neumann row; bit S: own Neumann row
    uint32_t* kmask;    // [Nc] unknown rows: bit s: slot s is a value row whose DP is not an unknown
                        // (its value moves to the PPE's right-hand side); 0 at other rows
    double* amat;       // [S][mps] PPE matrix of the unknown rows, plane stride MeshDev::mps; the slots of
                        // known value neighbours (kmask) keep their weights, centre = -sum of the others
    float* amat32;      // [S][mps] unknown rows and columns, difference form (centre = row sum)
    uint8_t* unknown;   // [Nc]
    double rs;
};

template <int DIM> struct Dims;
template <> struct Dims<2> { static constexpr int NB = 5, S = 9, CEN = 4; };
template <> struct Dims<3> { static constexpr int NB = 9, S = 27, CEN = 13; };

// ---------------------------------------------------------------------------
// Geometry helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ void cell_ijk(const MeshDev& m, int c, int ijk[3]) {
    ijk[0] = c % m.n[0];
    int r = c / m.n[0];
    ijk[1] = r % m.n[1];
    ijk[2] = r / m.n[1];
}

// Neighbour of cell ijk at slot s (offset (s%3-1, s/3%3-1, s/9-1)).  Returns
// false outside a non-periodic mesh.  shift[a] = wrap * L_a so that the
// neighbour's image position is x_j + shift[a].
template <int DIM>
__device__ __forceinline__ bool neighbour(const MeshDev& m, const int ijk[3], int s, int& j, double shift[3]) {
    int o[3] = {s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1};
    int idx = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int ii = ijk[a] + o[a];
        int w = 0;
        if (ii < 0) {
            if (!m.periodic[a]) return false;
            ii += m.n[a];
            w = -1;
        } else if (ii >= m.n[a]) {
            if (!m.periodic[a]) return false;
            ii -= m.n[a];
            w = 1;
        }
        shift[a] = (double)w * m.length[a];
        idx += ii * stride;
        stride *= m.n[a];
    }
    j = idx;
    return true;
}

// The same without branches: when the neighbour lies outside a
// non-periodic mesh, j = self and shift = 0 (and false is returned), so that
// j is always a valid index.
template <int DIM>
__device__ __forceinline__ bool neighbour_or_self(const MeshDev& m, const int ijk[3], int s, int self, int& j,
                                                  double shift[3]) {
    const int o[3] = {s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1};
    int idx = 0, stride = 1;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int ii = ijk[a] + o[a];
        const bool lo = ii < 0, hi = ii >= m.n[a];
        ii = lo ? ii + m.n[a] : (hi ? ii - m.n[a] : ii);
        ok = ok && (!(lo || hi) || m.periodic[a] != 0);
        shift[a] = (double)(lo ? -1 : (hi ? 1 : 0)) * m.length[a];
        idx += ii * stride;
        stride *= m.n[a];
    }
    j = ok ? idx : self;
    if (!ok)
        for (int a = 0; a < DIM; ++a) shift[a] = 0.0;
    return ok;
}

template <int DIM>
__device__ __forceinline__ constexpr int slot_nonzeros(int s) {
    int o[3] = {s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1};
    int nz = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) nz += (o[a] != 0);
    return nz;
}

// cos x from its Taylor series through x^20 (error below 1e-10 for
// |x| <= pi, below 1e-16 for |x| <= pi/2), by Horner in x^2 with + and *
// only, so that it gives the same bits wherever it is evaluated: the weight
// beta of the boundary-fitted arrangement (bit-exact DP positions) and the
// cos^2 MLS weight (bit-exact stencil weights).  Coefficients (-1)^k / (2k)!,
// the factorials exact in FP64 up to 20!.
__device__ __forceinline__ double series_cos(double x) {
#pragma clang fp contract(off)
    double c[11];
    double f = 1.0;
#pragma unroll
    for (int k = 0; k <= 10; ++k) {
        if (k > 0) f = f * (double)(2 * k - 1) * (double)(2 * k);
        c[k] = (k % 2 ? -1.0 : 1.0) / f;
    }
    const double x2 = x * x;
    double p = c[10];
#pragma unroll
    for (int k = 9; k >= 0; --k) p = p * x2 + c[k];
    return p;
}

// exp(-t) for 0 <= t <= 4 as (e^{-t/8})^8, with e^{-u} from its Taylor
// series through u^17 by Horner (+ and * only; coefficients 1/k!, exact
// factorials), then three squarings: the Gaussian MLS weight with the same
// bits wherever it is evaluated (relative error a few 1e-15).
__device__ __forceinline__ double series_exp_neg(double t) {
#pragma clang fp contract(off)
    double c[18];
    double f = 1.0;
#pragma unroll
    for (int k = 0; k < 18; ++k) {
        if (k > 0) f = f * (double)k;
        c[k] = 1.0 / f;
    }
    const double u = -(t * 0.125);
    double p = c[17];
#pragma unroll
    for (int k = 16; k >= 0; --k) p = p * u + c[k];
    p = p * p;
    p = p * p;
    return p * p;
}

// 0: no row, 1: value row (inner or Dirichlet id), 2: Neumann row.
__device__ __forceinline__ int row_kind(int rj, const BcDev& bc) {
    if (rj == MCD_ROLE_INNER) return 1;
    if (rj <= 0) return 0;
    return bc.type[rj & (MCD_MAX_IDS - 1)] == MCD_BC_NEUMANN ? 2 : 1;
}

__device__ __forceinline__ bool is_unknown(int rj, int j, const BcDev& bc) {
    if (bc.pin_first && j == 0) return false;
    if (rj == MCD_ROLE_INNER) return true;
    if (rj <= 0) return false;
    return bc.type[rj & (MCD_MAX_IDS - 1)] == MCD_BC_NEUMANN;
}

// ---------------------------------------------------------------------------
// Quadratic basis (Eq. p_ic) and its normal derivative
// 3D order: X, Y, Z, X^2/2, Y^2/2, Z^2/2, XY, YZ, ZX
// ---------------------------------------------------------------------------

template <int DIM> __device__ __forceinline__ void basis(const double* X, double* p);
template <> __device__ __forceinline__ void basis<2>(const double* X, double* p) {
    p[0] = X[0];
    p[1] = X[1];
    p[2] = 0.5 * X[0] * X[0];
    p[3] = X[0] * X[1];
    p[4] = 0.5 * X[1] * X[1];
}
template <> __device__ __forceinline__ void basis<3>(const double* X, double* p) {
    p[0] = X[0];
    p[1] = X[1];
    p[2] = X[2];
    p[3] = 0.5 * X[0] * X[0];
    p[4] = 0.5 * X[1] * X[1];
    p[5] = 0.5 * X[2] * X[2];
    p[6] = X[0] * X[1];
    p[7] = X[1] * X[2];
    p[8] = X[2] * X[0];
}

template <int DIM> __device__ __forceinline__ void basis_normal(const double* X, const double* nv, double* p);
template <> __device__ __forceinline__ void basis_normal<2>(const double* X, const double* nv, double* p) {
    p[0] = nv[0];
    p[1] = nv[1];
    p[2] = nv[0] * X[0];
    p[3] = nv[0] * X[1] + nv[1] * X[0];
    p[4] = nv[1] * X[1];
}
template <> __device__ __forceinline__ void basis_normal<3>(const double* X, const double* nv, double* p) {
    p[0] = nv[0];
    p[1] = nv[1];
    p[2] = nv[2];
    p[3] = nv[0] * X[0];
    p[4] = nv[1] * X[1];
    p[5] = nv[2] * X[2];
    p[6] = nv[0] * X[1] + nv[1] * X[0];
    p[7] = nv[1] * X[2] + nv[2] * X[1];
    p[8] = nv[2] * X[0] + nv[0] * X[2];
}

// Pure second-derivative components (sum / r_s^2 = laplacian).
template <int DIM> __device__ __forceinline__ double diag2(const double* P);
template <> __device__ __forceinline__ double diag2<2>(const double* P) { return P[2] + P[4]; }
template <> __device__ __forceinline__ double diag2<3>(const double* P) { return P[3] + P[4] + P[5]; }

// ---------------------------------------------------------------------------
// Reductions (wave64 shuffles, then LDS across the 4 waves of a block)
// ---------------------------------------------------------------------------

// Adds to *ctr the number of active lanes of the wave whose flag is set,
// with one atomic per wave instead of one per lane (many lanes adding to one
// counter serialise at the cache).
__device__ __forceinline__ void wave_count_add(int* ctr, bool flag) {
    const unsigned long long act = __ballot(1);
    const unsigned long long fm = __ballot(flag);
    if ((int)__lane_id() == __ffsll((unsigned long long)act) - 1 && fm != 0ull) atomicAdd(ctr, (int)__popcll(fm));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sums N values over the block; result valid in thread 0.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double (*lds)[kBlock / 64]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) lds[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) s += lds[q][w];
            v[q] = s;
        }
    }
}

// Maps the hardware block index to a logical one so that the blocks each XCD
// receives (hardware dispatch is round-robin over the 8 XCDs) cover one
// contiguous range of cells; neighbouring rows then share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
    const int per = nblocks >> 3;
    if ((nblocks & 7) != 0) return b;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// Host-side launchers (defined in the .hip sources)
// ---------------------------------------------------------------------------

struct Ctx;

hipError_t launch_roles(const MeshDev& m, const BodiesDev& B, double band_l0, int8_t* role, int8_t* role_prev,
                        double* pos, double* pos_prev, uint8_t* trans, uint8_t* band, int* counts,
                        int* latch, hipStream_t st);
// host constants of the boundary-fitted arrangement (half_alpha = 0: off)
struct FitDev {
    double half_alpha, re, pi_over_re;
};
hipError_t launch_relax(const MeshDev& m, const BodiesDev& B, double kl0, const double* spring, double eps_l0,
                        const FitDev& fit, const int8_t* role, const uint8_t* band, const double* pin, double* pout,
                        const int box_lo[3], const int box_n[3], unsigned long long* dmax, int sweep,
                        int* state, hipStream_t st);
hipError_t launch_copy_band(const MeshDev& m, const uint8_t* band, const double* src, double* dst,
                            const int box_lo[3], const int box_n[3], hipStream_t st);
hipError_t launch_normals(const MeshDev& m, const BodiesDev& B, const int8_t* role, const double* pos,
                          double* normal, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st);
hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t st);

hipError_t launch_mls_build(const MeshDev& m, const double* pos, const int8_t* role, const double* normal,
                            const BcDev& bc, double re, double rs, int wkind, const SetDev& set, int* counters,
                            int* latch, hipStream_t st);

hipError_t launch_apply(const MeshDev& m, const SetDev& set, int op, const double* in, int ncomp,
                        const double* fneu, const double* shift, double* out, double scale, hipStream_t st);
hipError_t launch_remap(const MeshDev& m, const SetDev& set_prev, const double* u, const double* pos_prev,
                        const double* pos, const int8_t* role_prev, const int8_t* role, const BodiesDev& Bprev,
                        const BodiesDev& Bnew, double* out, int* counters, hipStream_t st);
hipError_t launch_advect_diffuse(const MeshDev& m, const SetDev& set, const double* ut, double dt, double nu,
                                 const double* pos, const int8_t* role, const BodiesDev& B, double* ustar,
                                 hipStream_t st);
hipError_t launch_neumann_pressure(const MeshDev& m, const double* pos, const int8_t* role, const double* normal,
                                   const BodiesDev& B, double* f, hipStream_t st);
hipError_t launch_project(const MeshDev& m, const SetDev& set, const double* P, const double* f,
                          const double* ustar, double dt, const double* pos, const int8_t* role, const BodiesDev& B,
                          double* u, hipStream_t st);
hipError_t launch_force(const MeshDev& m, const SetDev& su, const SetDev& sp, const double* u, const double* p,
                        const double* fneu, const double* pos, const int8_t* role, const double* normal,
                        const BodiesDev& B, double mu, double* out, int* cnt, hipStream_t st);

// PPE on a (2H+1)^2 MLS support (2D comparison path, wide.hip)
struct WideWork;
struct WideResult {
    int iterations = 0;
    int converged = 0;
    int singular = 0;
    double true_rel_residual = 0.0;
    double build_ms = 0.0;
    double solve_ms = 0.0;
};
hipError_t wide_ppe(const MeshDev& m, WideWork** slot, int H, double re, double rs, int wkind, const double* pos,
                    const int8_t* role, const double* normal, const BcDev& bc, const double* rhs, const double* f,
                    double* p, double tol, int max_iter, WideResult* res, hipStream_t st);
hipError_t wide_lap_planes(const WideWork* w, double* out, hipStream_t st);
void wide_free(WideWork* w);

struct KrylovWork;
struct SolveParams {
    double tol;
    int max_iter;
    int precision;
    int caller_guess;
    double inner_tol;
    int max_outer;
    int check_every;
    int max_inner;
    double fp64_below;
    int precond;
};
struct SolveOut {
    int iterations, restarts, refinements, converged;
    int bad;                     // the right-hand side was not finite (nothing solved)
    double rel, bnorm;
};
hipError_t krylov_alloc(const MeshDev& m, KrylovWork** out);
void krylov_free(KrylovWork* w);
hipError_t krylov_profile(KrylovWork* w, int enable);
bool krylov_mg_usable(const KrylovWork* w);
hipError_t krylov_mg_apply(const MeshDev& m, KrylovWork& w, const SetDev& set, const double* in, double* out,
                           int* levels, hipStream_t st);
hipError_t krylov_set_shape(const MeshDev& m, KrylovWork& w, int grid, int depth);
void krylov_get_shape(const KrylovWork& w, int* grid, int* depth, int* blocks);
hipError_t krylov_autotune(const MeshDev& m, const SetDev& set, KrylovWork& w, int iters, int max_cand,
                           int* n_out, int* grid_out, int* depth_out, double* us_out, int* chosen);
void krylov_profile_read(KrylovWork* w, double* ms_p, long long* n_p, double* ms_s, long long* n_s, double* ms32,
                         long long* n32, int reset);
hipError_t solve_ppe_impl(const MeshDev& m, const SetDev& set, KrylovWork& w, const double* rhs, const double* fneu,
                          double* p, const SolveParams& sp, SolveOut* out, int* bad, hipStream_t st);
// Multigrid preconditioner and the Bi-CGSTAB that uses it (mg.hip).
struct MgWork;
struct MgVecs {
    double *x, *r, *rhat, *p, *v, *s, *t, *ph, *sh;   // [Nc] FP64
    const double* b;                                  // effective right-hand side
};
struct MgResult {
    int iterations = 0, restarts = 0, converged = 0, coarse_singular = 0;
    int bad = 0;                 // the right-hand side was not finite (nothing solved)
    double rel = 0.0, bnorm = 0.0;
};
hipError_t mg_alloc(const MeshDev& m, MgWork** out);
void mg_free(MgWork* w);
bool mg_usable(const MgWork* w);
hipError_t mg_setup(const MeshDev& m, MgWork& w, const SetDev& set, hipStream_t st);
// bad: device flag of a non-finite right-hand side (set by the b_eff kernel),
// read back with the first residual's totals
hipError_t mg_bicgstab(const MeshDev& m, MgWork& w, const SetDev& set, const MgVecs& V, double tol, int max_iter,
                       bool f32_products, const int* bad, hipStream_t st, MgResult* out);
hipError_t mg_apply(const MeshDev& m, MgWork& w, const SetDev& set, const double* in, double* out, int* levels,
                    hipStream_t st);

hipError_t noalloc_setup(int device);
size_t noalloc_scratch_bytes();
hipError_t ppe_residual_noalloc_impl(int device, const MeshDev& m, const SetDev& set, const double* rhs,
                                     const double* fneu, const double* p, double* r, double norms[2], int* bad_out,
                                     hipStream_t st);
hipError_t ppe_residual_impl(const MeshDev& m, const SetDev& set, KrylovWork& w, const double* rhs, const double* fneu,
                             const double* p, double* r, double norms[2], int* bad, hipStream_t st);

struct UNet;
hipError_t unet_create(int dim, int D, int H, int W, int L, const int* ch, int body_id, int wall_id, UNet** out);
void unet_free(UNet* u);
hipError_t unet_weights_to_bf16(UNet& u, hipStream_t st);
hipError_t unet_infer(UNet& u, const double* b, const double* pprev, const int8_t* role, const BcDev& bc,
                      double* out, hipStream_t st);
hipError_t unet_train_step(UNet& u, const double* b, const double* pprev, const double* Pt, const int8_t* role,
                           const BcDev& bc, float lr, hipStream_t st, double* loss_out);
size_t unet_nparams(const UNet& u);
float* unet_theta(UNet& u);
float* unet_grad(UNet& u);
float* unet_head_out(UNet& u);
void unet_reset_optimizer(UNet& u, hipStream_t st);
void unet_set_output_scale(UNet& u, double s);

}  // namespace mcd
