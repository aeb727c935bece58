// C ABI of libmcd: argument validation, context state, launches.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

using namespace mcd;

namespace {

enum {
    CNT_TRANS = 0,       // [0..8] transition histogram, [9] band cells, [10] role errors
    CNT_MLS = 16,        // [16] singular inner, [17] singular other, [18] first singular inner DP
    CNT_LATCH_ROLE = 32,
    CNT_LATCH_SING = 33,
    CNT_REMAP = 40,      // [40] shifted, [41] fallback
    CNT_BAD = 48,        // non-finite PPE right-hand side
    CNT_N = 64
};

struct SetStore {
    SetDev dev{};
    int built = 0;
};

// The stored FP64 matrix keeps, in the slots of an unknown row, the weights
// of its known value neighbours (bits of kmask); the exported copy [S][Nc]
// is the matrix itself, with those columns zero.
__global__ void k_export_matrix(int Nc, const uint32_t* __restrict__ kmask, double* __restrict__ a) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Nc; c += gridDim.x * blockDim.x) {
        uint32_t km = kmask[c];
        while (km) {
            const int s = __builtin_ctz(km);
            km &= km - 1u;
            a[(size_t)s * Nc + c] = 0.0;
        }
    }
}

}  // namespace

struct mcd_ctx {
    mcd_mesh_desc desc{};
    mcd_params prm{};
    MeshDev m{};
    hipStream_t stream = nullptr;
    int dim = 2, NB = 5, S = 9;
    size_t Nc = 0;
    SetStore sets[MCD_MAX_SETS];
    double* pos_tmp = nullptr;
    uint8_t* band = nullptr;
    unsigned long long* dmax = nullptr;
    int max_sweeps_alloc = 0;
    int* relax_state = nullptr;
    int* cnt = nullptr;
    int* cnt_host = nullptr;    // pinned
    double* fbuf = nullptr;     // fluid-force results: [bodies][2] doubles, then [bodies][3] ints
    KrylovWork* kw = nullptr;
    // host constants of the arrangement (computed once, used identically by every call)
    double kl0 = 0, spring[4] = {0, 0, 0, 0}, eps_l0 = 0, band_l0 = 0, re = 0, rs = 0;
    FitDev fit{0.0, 0.0, 0.0};
    BodiesDev sdft{};           // discrete-SDF interpolation constants (sdfc, sdfD1 ...)
    bool sdf_ok = false;
    // captured call sequences (mcd_graph_begin/end): the calls of a capture are
    // recorded on a private stream and launched as one graph on `stream`
    hipStream_t cap_st = nullptr;
    hipStream_t user_st = nullptr;
    int capturing = -1;
    bool cap_failed = false;
    hipGraphExec_t gexec[MCD_MAX_GRAPHS] = {};
    int g_inst[MCD_MAX_GRAPHS] = {}, g_upd[MCD_MAX_GRAPHS] = {};
    WideWork* ww = nullptr;     // wide-support PPE comparison path (allocated on first use)
    int device = -1;            // device current at mcd_create
    std::string err;
};

// Closed form of the chi_c = 1 quadratic MLS over the 3x3 nodes of a regular
// grid (offsets X, Y in units of h, weight W(|X|; r_e / l0) of the context,
// basis p = (X, Y, X^2/2, XY, Y^2/2)).  By the symmetry of the support the
// normal matrix is block diagonal: X and Y each with sum w X^2 =
// 2 w1 + 4 w2 = D1, XY with sum w X^2 Y^2 = 4 w2 = D3, and the pair
// (X^2/2, Y^2/2) with [[A, B], [B, A]], A = D1 / 4, B = w2 (w1, w2: the
// weights of the edge and corner nodes).  The per-node factors w_k p_q(X_k)
// are exact.  False when a weight vanishes (r_e not beyond sqrt 2).  The 3D
// constants (3x3x3 nodes) are set alongside.
static bool sdf_table(int wkind, double re, BodiesDev* t) {
#pragma clang fp contract(off)
    auto wfun = [&](double r) {
        if (!(r <= re)) return 0.0;
        if (wkind == MCD_WEIGHT_COS2) {
            const double a = cos(M_PI * r / (2.0 * re));
            return a * a;
        }
        return exp(-4.0 * r * r / (re * re));
    };
    const double w1 = wfun(1.0), w2 = wfun(sqrt(2.0));
    if (!(w1 > 0.0) || !(w2 > 0.0)) return false;
    int k = 0;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
            if (di == 0 && dj == 0) continue;
            const double w = (di != 0 && dj != 0) ? w2 : w1;
            const double X = di, Y = dj;
            t->sdfc[0][k] = w * X;
            t->sdfc[1][k] = w * Y;
            t->sdfc[2][k] = w * (0.5 * X * X);
            t->sdfc[3][k] = w * (X * Y);
            t->sdfc[4][k] = w * (0.5 * Y * Y);
            ++k;
        }
    t->sdfD1 = 2.0 * w1 + 4.0 * w2;
    t->sdfD3 = 4.0 * w2;
    t->sdfA = t->sdfD1 / 4.0;
    t->sdfB = w2;
    t->sdfDet = t->sdfA * t->sdfA - t->sdfB * t->sdfB;
    // 3D: face, edge and corner node weights; D1 = sum w X^2, DX = sum w X^2 Y^2
    const double w3 = wfun(sqrt(3.0));
    t->s3w[0] = w1;
    t->s3w[1] = w2;
    t->s3w[2] = w3;
    t->s3D1 = 2.0 * w1 + 8.0 * w2 + 8.0 * w3;
    t->s3DX = 4.0 * w2 + 8.0 * w3;
    t->s3A = t->s3D1 / 4.0;
    t->s3B = t->s3DX / 4.0;
    return true;
}

static mcd_status fail(mcd_ctx* c, mcd_status s, const char* fmt, const char* detail = "") {
    if (c) {
        char buf[512];
        snprintf(buf, sizeof(buf), fmt, detail);
        c->err = buf;
        if (c->capturing >= 0) c->cap_failed = true;   // the recorded sequence is incomplete
    }
    return s;
}

static mcd_status hipfail(mcd_ctx* c, hipError_t e, const char* where) {
    if (c) {
        c->err = std::string(where) + ": " + hipGetErrorString(e);
        if (c->capturing >= 0) c->cap_failed = true;
    }
    return MCD_ERR_HIP;
}

// calls that wait for the device (or read results back) cannot be recorded
#define NO_CAPTURE(ctx, name)                                                              \
    do {                                                                                   \
        if ((ctx)->capturing >= 0) return fail(ctx, MCD_ERR_ARG, name ": not allowed while a graph is captured%s"); \
    } while (0)

#define HIPCHK(ctx, expr, where)                    \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return hipfail(ctx, _e, where); \
    } while (0)

static bool make_bodies(mcd_ctx* c, const mcd_body* bodies, int n, BodiesDev* out) {
#pragma clang fp contract(off)
    *out = BodiesDev{};
    if (n < 0 || n > MCD_MAX_BODIES || (n > 0 && !bodies)) return false;
    // ascending id order: ties of the nearest-body rule go to the lower id
    int order[MCD_MAX_BODIES];
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order, order + n, [&](int a, int b) { return bodies[a].id < bodies[b].id; });
    out->n = n;
    for (int k = 0; k < n; ++k) {
        const mcd_body& b = bodies[order[k]];
        if (b.id < 1 || b.id >= MCD_MAX_IDS || (c->desc.walls && b.id == c->desc.wall_id)) return false;
        if (k > 0 && b.id == out->id[k - 1]) return false;     // ids are distinct
        if (!(b.radius > 0) || !isfinite(b.radius)) return false;
        out->sdf[k] = nullptr;
        if (b.sdf) {
            // discrete SDF: a valid grid whose inner nodes cover the ball of the far
            // radius, a unit posture axis (3D), computable interpolation constants
            const int d = c->dim;
            if (!c->sdf_ok || !(b.sdf_h > 0) || !isfinite(b.sdf_h) || !isfinite(b.theta)) return false;
            const double rho = b.radius + (c->prm.band_over_l0 + 2.0) * c->m.l0;
            for (int a = 0; a < d; ++a) {
                if (b.sdf_n[a] < 3 || !isfinite(b.sdf_origin[a])) return false;
                if (!(b.sdf_origin[a] + b.sdf_h <= -rho) || !(b.sdf_origin[a] + (b.sdf_n[a] - 2) * b.sdf_h >= rho))
                    return false;
                out->sn[k][a] = b.sdf_n[a];
                out->so[k][a] = b.sdf_origin[a];
            }
            out->sdf[k] = b.sdf;
            out->sh[k] = b.sdf_h;
            const double ct = cos(b.theta), st = sin(b.theta);
            out->cth[k] = ct;
            out->sth[k] = st;
            if (d == 3) {
                const double a0 = b.axis[0], a1 = b.axis[1], a2 = b.axis[2];
                if (!isfinite(a0) || !isfinite(a1) || !isfinite(a2)) return false;
                if (!(fabs(a0 * a0 + a1 * a1 + a2 * a2 - 1.0) <= 1e-12)) return false;
                // Rodrigues: R = cos I + sin [a]x + (1 - cos) a a^T, row-major
                const double oc = 1.0 - ct;
                double* R = out->post[k];
                R[0] = ct + oc * a0 * a0;
                R[1] = oc * a0 * a1 - st * a2;
                R[2] = oc * a0 * a2 + st * a1;
                R[3] = oc * a1 * a0 + st * a2;
                R[4] = ct + oc * a1 * a1;
                R[5] = oc * a1 * a2 - st * a0;
                R[6] = oc * a2 * a0 - st * a1;
                R[7] = oc * a2 * a1 + st * a0;
                R[8] = ct + oc * a2 * a2;
            }
            out->far2[k] = rho * rho;
        }
        out->id[k] = b.id;
        for (int a = 0; a < 3; ++a) {
            if (!isfinite(b.centre[a]) || !isfinite(b.velocity[a]) || !isfinite(b.dvdt[a])) return false;
            if (!isfinite(b.omega[a]) || !isfinite(b.domega_dt[a])) return false;
            if (c->dim == 2 && a < 2 && (b.omega[a] != 0.0 || b.domega_dt[a] != 0.0)) return false;
            out->c[k][a] = b.centre[a];
            out->vel[k][a] = b.velocity[a];
            out->dvdt[k][a] = b.dvdt[a];
            out->om[k][a] = b.omega[a];
            out->dom[k][a] = b.domega_dt[a];
            if (b.omega[a] != 0.0 || b.domega_dt[a] != 0.0) out->rot[k] = 1;
        }
        out->any_rot |= out->rot[k];
        out->R[k] = b.radius;
        out->R2[k] = b.radius * b.radius;
    }
    // the context's discrete-SDF interpolation constants
    memcpy(out->sdfc, c->sdft.sdfc, sizeof(out->sdfc));
    out->sdfD1 = c->sdft.sdfD1;
    out->sdfD3 = c->sdft.sdfD3;
    out->sdfA = c->sdft.sdfA;
    out->sdfB = c->sdft.sdfB;
    out->sdfDet = c->sdft.sdfDet;
    for (int q = 0; q < 3; ++q) out->s3w[q] = c->sdft.s3w[q];
    out->s3D1 = c->sdft.s3D1;
    out->s3DX = c->sdft.s3DX;
    out->s3A = c->sdft.s3A;
    out->s3B = c->sdft.s3B;
    return true;
}

static bool make_bc(const mcd_bc_table* bc, BcDev* out) {
    *out = BcDev{};
    if (!bc) return false;
    for (int i = 0; i < MCD_MAX_IDS; ++i) {
        if (bc->type[i] != MCD_BC_DIRICHLET && bc->type[i] != MCD_BC_NEUMANN) return false;
        out->type[i] = bc->type[i];
    }
    out->pin_first = bc->pin_first ? 1 : 0;
    return true;
}

static bool valid_set(mcd_ctx* c, int set, bool need_built) {
    return c && set >= 0 && set < MCD_MAX_SETS && (!need_built || c->sets[set].built);
}

extern "C" {

mcd_status mcd_create(const mcd_mesh_desc* mesh, const mcd_params* prm, void* hip_stream, mcd_ctx** out) {
    if (!mesh || !prm || !out) return MCD_ERR_ARG;
    *out = nullptr;
    const int dim = mesh->dim;
    if (dim != 2 && dim != 3) return MCD_ERR_ARG;
    long long Nc = 1;
    for (int a = 0; a < dim; ++a) {
        if (mesh->n[a] < 3 || mesh->n[a] > (1 << 16)) return MCD_ERR_ARG;
        Nc *= mesh->n[a];
    }
    if (Nc > (1LL << 30)) return MCD_ERR_ARG;
    if (!(mesh->l0 > 0) || !isfinite(mesh->l0)) return MCD_ERR_ARG;
    if (mesh->walls && (mesh->wall_id < 1 || mesh->wall_id >= MCD_MAX_IDS)) return MCD_ERR_ARG;
    if (!(prm->re_over_l0 > 0) || !(prm->rs_over_l0 > 0) || !(prm->kappa > 0) || !(prm->band_over_l0 >= 0) ||
        !(prm->eps_relax >= 0) || (prm->weight_kind != MCD_WEIGHT_COS2 && prm->weight_kind != MCD_WEIGHT_GAUSS) ||
        !(prm->fit_alpha >= 0 && prm->fit_alpha <= 1) ||
        (prm->fit_alpha > 0 && (!(prm->fit_re_over_l0 > 0) || !isfinite(prm->fit_re_over_l0))))
        return MCD_ERR_ARG;
    mcd_ctx* c = new mcd_ctx();
    c->desc = *mesh;
    c->prm = *prm;
    c->stream = (hipStream_t)hip_stream;
    c->dim = dim;
    c->NB = dim == 2 ? 5 : 9;
    c->S = dim == 2 ? 9 : 27;
    c->Nc = (size_t)Nc;
    MeshDev& m = c->m;
    m.dim = dim;
    m.Nc = (int)Nc;
    m.l0 = mesh->l0;
    for (int a = 0; a < 3; ++a) {
        m.n[a] = a < dim ? mesh->n[a] : 1;
        m.origin[a] = a < dim ? mesh->origin[a] : 0.0;
        m.periodic[a] = a < dim ? (mesh->periodic[a] ? 1 : 0) : 0;
        m.length[a] = (double)m.n[a] * mesh->l0;
    }
    m.walls = mesh->walls ? 1 : 0;
    m.wall_id = mesh->wall_id;
    m.mps = padded_plane_stride((size_t)Nc);
    const double l0 = mesh->l0;
    c->kl0 = prm->kappa * l0;
    c->spring[0] = 0.0;
    c->spring[1] = l0;
    c->spring[2] = sqrt(2.0) * l0;
    c->spring[3] = sqrt(3.0) * l0;
    c->eps_l0 = prm->eps_relax * l0;
    c->band_l0 = prm->band_over_l0 * l0;
    if (prm->fit_alpha > 0) {
        const double re_fit = prm->fit_re_over_l0 * l0;
        c->fit = FitDev{prm->fit_alpha * 0.5, re_fit, M_PI / re_fit};
    }
    c->re = prm->re_over_l0 * l0;
    c->sdf_ok = sdf_table(prm->weight_kind, prm->re_over_l0, &c->sdft);
    c->rs = prm->rs_over_l0 * l0;

    auto alloc = [&](void** p, size_t bytes) {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) e = hipMemset(*p, 0, bytes);
        return e;
    };
    hipError_t e = hipSuccess;
    const size_t N = c->Nc;
    for (int s = 0; s < MCD_MAX_SETS && e == hipSuccess; ++s) {
        SetDev& d = c->sets[s].dev;
        d.rs = c->rs;
        e = alloc((void**)&d.phi, (size_t)c->NB * (c->S + 1) * m.mps * sizeof(double));
        if (e == hipSuccess) e = alloc((void**)&d.vmask, N * sizeof(uint32_t));
        if (e == hipSuccess) e = alloc((void**)&d.nmask, N * sizeof(uint32_t));
        if (e == hipSuccess) e = alloc((void**)&d.kmask, N * sizeof(uint32_t));
        if (e == hipSuccess) e = alloc((void**)&d.amat, (size_t)c->S * m.mps * sizeof(double));
        if (e == hipSuccess) e = alloc((void**)&d.amat32, (size_t)c->S * m.mps * sizeof(float));
        if (e == hipSuccess) e = alloc((void**)&d.unknown, N);
    }
    c->max_sweeps_alloc = 4096;
    if (e == hipSuccess) e = alloc((void**)&c->pos_tmp, (size_t)dim * N * sizeof(double));
    if (e == hipSuccess) e = alloc((void**)&c->band, N);
    if (e == hipSuccess) e = alloc((void**)&c->dmax, (size_t)c->max_sweeps_alloc * sizeof(unsigned long long));
    if (e == hipSuccess) e = alloc((void**)&c->relax_state, 4 * sizeof(int));
    if (e == hipSuccess) e = alloc((void**)&c->cnt, CNT_N * sizeof(int));
    if (e == hipSuccess) e = alloc((void**)&c->fbuf, 4 * MCD_MAX_BODIES * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->cnt_host, CNT_N * sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = krylov_alloc(c->m, &c->kw);
    if (e == hipSuccess) e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = noalloc_setup(c->device);     // scratch address of this device, once per device
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        mcd_destroy(c);
        return e == hipErrorOutOfMemory ? MCD_ERR_OOM : MCD_ERR_HIP;
    }
    *out = c;
    return MCD_OK;
}

// ---------------------------------------------------------------------------
// Lifetime while recordings are open.  Destroying a context or a model frees
// device memory and waits for its stream; either, done while any context of
// the process has a recording open (mcd_graph_begin .. mcd_graph_end), can
// make the runtime invalidate that recording.  Destruction is therefore
// deferred until the last open recording of the process has ended.
// ---------------------------------------------------------------------------

static std::mutex g_life_mu;
static int g_open_recordings = 0;
static std::vector<mcd_ctx*> g_pending_ctx;
static std::vector<mcd_model*> g_pending_model;

static void destroy_ctx_now(mcd_ctx* c);
static void destroy_model_now(mcd_model* md);

static void recording_opened() {
    std::lock_guard<std::mutex> lk(g_life_mu);
    ++g_open_recordings;
}

// A recording ended; when it was the last open one, destroys what waited.
static void recording_closed() {
    std::vector<mcd_ctx*> ctxs;
    std::vector<mcd_model*> models;
    {
        std::lock_guard<std::mutex> lk(g_life_mu);
        if (g_open_recordings > 0) --g_open_recordings;
        if (g_open_recordings > 0) return;
        ctxs.swap(g_pending_ctx);
        models.swap(g_pending_model);
    }
    for (mcd_model* md : models) destroy_model_now(md);
    for (mcd_ctx* c : ctxs) destroy_ctx_now(c);
}

void mcd_destroy(mcd_ctx* c) {
    if (!c) return;
    if (c->capturing >= 0) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(c->cap_st, &g);
        if (g) (void)hipGraphDestroy(g);
        c->stream = c->user_st;
        c->capturing = -1;
        (void)hipGetLastError();
        recording_closed();
    }
    {
        std::lock_guard<std::mutex> lk(g_life_mu);
        if (g_open_recordings > 0) {
            g_pending_ctx.push_back(c);
            return;
        }
    }
    destroy_ctx_now(c);
}

int mcd_pending_destroys(void) {
    std::lock_guard<std::mutex> lk(g_life_mu);
    return (int)(g_pending_ctx.size() + g_pending_model.size());
}

static void destroy_ctx_now(mcd_ctx* c) {
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < MCD_MAX_GRAPHS; ++k)
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    wide_free(c->ww);
    if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
    for (int s = 0; s < MCD_MAX_SETS; ++s) {
        SetDev& d = c->sets[s].dev;
        void* ptrs[7] = {d.phi, d.vmask, d.nmask, d.kmask, d.amat, d.amat32, d.unknown};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
    }
    void* ptrs[6] = {c->pos_tmp, c->band, c->dmax, c->relax_state, c->cnt, c->fbuf};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (c->cnt_host) (void)hipHostFree(c->cnt_host);
    krylov_free(c->kw);
    delete c;
}

mcd_status mcd_set_stream(mcd_ctx* c, void* hip_stream) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_set_stream");
    c->stream = (hipStream_t)hip_stream;
    return MCD_OK;
}

const char* mcd_last_error(const mcd_ctx* c) { return c ? c->err.c_str() : "null context"; }

mcd_status mcd_sync(mcd_ctx* c) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_sync");
    HIPCHK(c, hipStreamSynchronize(c->stream), "mcd_sync");
    HIPCHK(c, hipMemcpy(c->cnt_host, c->cnt, CNT_N * sizeof(int), hipMemcpyDeviceToHost), "mcd_sync copy");
    const int role_err = c->cnt_host[CNT_LATCH_ROLE], sing = c->cnt_host[CNT_LATCH_SING];
    HIPCHK(c, launch_fill_i32(c->cnt + CNT_LATCH_ROLE, 2, 0, c->stream), "mcd_sync clear");
    HIPCHK(c, hipStreamSynchronize(c->stream), "mcd_sync clear");
    if (sing) {
        char buf[64];
        snprintf(buf, sizeof(buf), "%d", sing);
        return fail(c, MCD_ERR_SINGULAR, "singular MLS moment matrix at %s inner DPs", buf);
    }
    if (role_err) {
        char buf[64];
        snprintf(buf, sizeof(buf), "%d", role_err);
        return fail(c, MCD_ERR_ROLE, "%s void<->inner role transitions", buf);
    }
    return MCD_OK;
}

mcd_status mcd_update_dps(mcd_ctx* c, const mcd_body* bodies, int n_bodies, int max_sweeps, double* pos,
                          int8_t* role, double* pos_prev, int8_t* role_prev, uint8_t* trans, double* normal,
                          mcd_update_info* info) {
    if (!c) return MCD_ERR_ARG;
    if (!pos || !role || !pos_prev || !role_prev || !trans || !normal)
        return fail(c, MCD_ERR_ARG, "mcd_update_dps: null array%s");
    if (max_sweeps < 0 || max_sweeps > c->max_sweeps_alloc)
        return fail(c, MCD_ERR_ARG, "mcd_update_dps: max_sweeps out of range%s");
    if (info) NO_CAPTURE(c, "mcd_update_dps with info");
    BodiesDev B;
    if (!make_bodies(c, bodies, n_bodies, &B)) return fail(c, MCD_ERR_ARG, "mcd_update_dps: invalid bodies%s");
    const MeshDev& m = c->m;
    hipStream_t st = c->stream;
    const size_t N = c->Nc;
    HIPCHK(c, launch_fill_i32(c->cnt + CNT_TRANS, 11, 0, st), "fill");
    HIPCHK(c, launch_roles(m, B, c->band_l0, role, role_prev, pos, pos_prev, trans, c->band, c->cnt + CNT_TRANS,
                           c->cnt + CNT_LATCH_ROLE, st),
           "roles");
    // bounding box of the band: cells whose centroid lies within R + band of a body
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, bn[3] = {1, 1, 1};
    bool any = false;
    for (int b = 0; b < B.n; ++b) {
        int l[3] = {0, 0, 0}, h[3] = {0, 0, 0};
        for (int a = 0; a < c->dim; ++a) {
            const double ext = B.R[b] + c->band_l0 + m.l0;
            l[a] = (int)floor((B.c[b][a] - ext - m.origin[a]) / m.l0) - 1;
            h[a] = (int)floor((B.c[b][a] + ext - m.origin[a]) / m.l0) + 1;
            l[a] = std::max(l[a], 0);
            h[a] = std::min(h[a], m.n[a] - 1);
        }
        for (int a = 0; a < c->dim; ++a) {
            lo[a] = any ? std::min(lo[a], l[a]) : l[a];
            hi[a] = any ? std::max(hi[a], h[a]) : h[a];
        }
        any = true;
    }
    if (any)
        for (int a = 0; a < c->dim; ++a) bn[a] = std::max(0, hi[a] - lo[a] + 1);
    else
        bn[0] = 0;
    const bool box = bn[0] > 0 && bn[1] > 0 && bn[2] > 0;
    HIPCHK(c, launch_fill_i32(c->relax_state, 4, 0, st), "fill");
    if (max_sweeps > 0) {
        HIPCHK(c, launch_fill_u64(c->dmax, max_sweeps, 0ull, st), "fill");
        HIPCHK(c, hipMemcpyAsync(c->pos_tmp, pos, (size_t)c->dim * N * sizeof(double), hipMemcpyDeviceToDevice, st),
               "copy");
    }
    for (int s = 0; s < max_sweeps; ++s) {
        const double* pin = (s & 1) ? c->pos_tmp : pos;
        double* pout = (s & 1) ? pos : c->pos_tmp;
        // an empty band (no body) still runs one sweep over nothing, as in the definition
        HIPCHK(c, launch_relax(m, B, c->kl0, c->spring, c->eps_l0, c->fit, role, c->band, pin, pout, lo, box ? bn : lo, c->dmax,
                               s, c->relax_state, st),
               "relax");
    }
    if (max_sweeps & 1) HIPCHK(c, launch_copy_band(m, c->band, c->pos_tmp, pos, lo, bn, st), "copy back");
    HIPCHK(c, launch_normals(m, B, role, pos, normal, st), "normals");
    if (info) {
        HIPCHK(c, hipStreamSynchronize(st), "mcd_update_dps");
        int h[16];
        int rs[4];
        HIPCHK(c, hipMemcpy(h, c->cnt + CNT_TRANS, 11 * sizeof(int), hipMemcpyDeviceToHost), "copy");
        HIPCHK(c, hipMemcpy(rs, c->relax_state, 4 * sizeof(int), hipMemcpyDeviceToHost), "copy");
        for (int k = 0; k < 9; ++k) info->counts[k] = h[k];
        info->band_cells = h[9];
        info->role_errors = h[10];
        info->sweeps = rs[1];
        if (h[10]) {
            HIPCHK(c, launch_fill_i32(c->cnt + CNT_LATCH_ROLE, 1, 0, st), "fill");
            return fail(c, MCD_ERR_ROLE, "mcd_update_dps: void<->inner role transition%s");
        }
    }
    return MCD_OK;
}

mcd_status mcd_build_stencils(mcd_ctx* c, int set, const double* pos, const int8_t* role, const double* normal,
                              const mcd_bc_table* bc) {
    if (!c) return MCD_ERR_ARG;
    if (!valid_set(c, set, false)) return fail(c, MCD_ERR_ARG, "mcd_build_stencils: bad set index%s");
    if (!pos || !role || !normal) return fail(c, MCD_ERR_ARG, "mcd_build_stencils: null array%s");
    BcDev b;
    if (!make_bc(bc, &b)) return fail(c, MCD_ERR_ARG, "mcd_build_stencils: invalid bc table%s");
    HIPCHK(c, launch_fill_i32(c->cnt + CNT_MLS, 2, 0, c->stream), "fill");
    HIPCHK(c, launch_fill_i32(c->cnt + CNT_MLS + 2, 1, 0x7fffffff, c->stream), "fill");
    HIPCHK(c, launch_mls_build(c->m, pos, role, normal, b, c->re, c->rs, c->prm.weight_kind, c->sets[set].dev,
                               c->cnt + CNT_MLS, c->cnt + CNT_LATCH_SING, c->stream),
           "mls_build");
    c->sets[set].built = 1;
    return MCD_OK;
}

mcd_status mcd_get_stencils(mcd_ctx* c, int set, double* phi, uint32_t* masks, double* amat) {
    if (!c) return MCD_ERR_ARG;
    if (!valid_set(c, set, true)) return fail(c, MCD_ERR_ARG, "mcd_get_stencils: set not built%s");
    const size_t N = c->Nc;
    const SetDev& d = c->sets[set].dev;
    hipStream_t st = c->stream;
    if (phi)
        HIPCHK(c, hipMemcpy2DAsync(phi, N * sizeof(double), d.phi, c->m.mps * sizeof(double), N * sizeof(double),
                                   (size_t)c->NB * (c->S + 1), hipMemcpyDeviceToDevice, st),
               "copy");
    if (masks) {
        HIPCHK(c, hipMemcpyAsync(masks, d.vmask, N * sizeof(uint32_t), hipMemcpyDeviceToDevice, st), "copy");
        HIPCHK(c, hipMemcpyAsync(masks + N, d.nmask, N * sizeof(uint32_t), hipMemcpyDeviceToDevice, st), "copy");
    }
    if (amat) {
        HIPCHK(c, hipMemcpy2DAsync(amat, N * sizeof(double), d.amat, c->m.mps * sizeof(double), N * sizeof(double),
                                   (size_t)c->S, hipMemcpyDeviceToDevice, st),
               "copy");
        const int g = (int)std::min<size_t>((N + kBlock - 1) / kBlock, 4096);
        hipLaunchKernelGGL(k_export_matrix, dim3(g), dim3(kBlock), 0, st, (int)N, d.kmask, amat);
        HIPCHK(c, hipGetLastError(), "export");
    }
    return MCD_OK;
}

mcd_status mcd_apply(mcd_ctx* c, int set, int op, const double* in, int ncomp, const double* neumann_f,
                     const double* shift, double* out) {
    if (!c) return MCD_ERR_ARG;
    if (!valid_set(c, set, true)) return fail(c, MCD_ERR_ARG, "mcd_apply: set not built%s");
    if (!in || !out) return fail(c, MCD_ERR_ARG, "mcd_apply: null array%s");
    switch (op) {
        case MCD_OP_PHI:
        case MCD_OP_GRAD:
            if (ncomp != 1) return fail(c, MCD_ERR_ARG, "mcd_apply: PHI/GRAD need ncomp = 1%s");
            break;
        case MCD_OP_LAP:
            if (ncomp < 1 || ncomp > 16) return fail(c, MCD_ERR_ARG, "mcd_apply: bad ncomp%s");
            break;
        case MCD_OP_DIV:
            if (ncomp != c->dim) return fail(c, MCD_ERR_ARG, "mcd_apply: DIV needs ncomp = dim%s");
            break;
        case MCD_OP_SHIFT:
            if (ncomp < 1 || ncomp > 16 || !shift) return fail(c, MCD_ERR_ARG, "mcd_apply: SHIFT needs shift%s");
            break;
        default:
            return fail(c, MCD_ERR_ARG, "mcd_apply: unknown op%s");
    }
    HIPCHK(c, launch_apply(c->m, c->sets[set].dev, op, in, ncomp, neumann_f, shift, out, 1.0, c->stream), "apply");
    return MCD_OK;
}

mcd_status mcd_remap(mcd_ctx* c, int set_prev, const double* u, const double* pos_prev, const double* pos,
                     const int8_t* role_prev, const int8_t* role, const mcd_body* bodies_prev,
                     const mcd_body* bodies_new, int n_bodies, double* out) {
    if (!c) return MCD_ERR_ARG;
    if (!valid_set(c, set_prev, true)) return fail(c, MCD_ERR_ARG, "mcd_remap: set not built%s");
    if (!u || !pos_prev || !pos || !role_prev || !role || !out || u == out)
        return fail(c, MCD_ERR_ARG, "mcd_remap: null or aliased array%s");
    BodiesDev Bp, Bn;
    if (!make_bodies(c, bodies_prev, n_bodies, &Bp) || !make_bodies(c, bodies_new, n_bodies, &Bn))
        return fail(c, MCD_ERR_ARG, "mcd_remap: invalid bodies%s");
    HIPCHK(c, launch_fill_i32(c->cnt + CNT_REMAP, 2, 0, c->stream), "fill");
    HIPCHK(c, launch_remap(c->m, c->sets[set_prev].dev, u, pos_prev, pos, role_prev, role, Bp, Bn, out,
                           c->cnt + CNT_REMAP, c->stream),
           "remap");
    return MCD_OK;
}

mcd_status mcd_advect_diffuse(mcd_ctx* c, int set, const double* ut, double dt, double nu, const double* pos,
                              const int8_t* role, const mcd_body* bodies, int n_bodies, double* ustar, double* rhs) {
    if (!c) return MCD_ERR_ARG;
    if (!valid_set(c, set, true)) return fail(c, MCD_ERR_ARG, "mcd_advect_diffuse: set not built%s");
    if (!ut || !role || !ustar || ut == ustar) return fail(c, MCD_ERR_ARG, "mcd_advect_diffuse: bad arrays%s");
    if (!(dt > 0) || !(nu >= 0) || !isfinite(dt) || !isfinite(nu))
        return fail(c, MCD_ERR_ARG, "mcd_advect_diffuse: bad dt/nu%s");
    BodiesDev B;
    if (!make_bodies(c, bodies, n_bodies, &B)) return fail(c, MCD_ERR_ARG, "mcd_advect_diffuse: invalid bodies%s");
    if (B.any_rot && !pos) return fail(c, MCD_ERR_ARG, "mcd_advect_diffuse: a rotating body needs pos%s");
    HIPCHK(c, launch_advect_diffuse(c->m, c->sets[set].dev, ut, dt, nu, pos, role, B, ustar, c->stream), "advect");
    if (rhs)
        HIPCHK(c, launch_apply(c->m, c->sets[set].dev, MCD_OP_DIV, ustar, c->dim, nullptr, nullptr, rhs, 1.0 / dt,
                               c->stream),
               "rhs");
    return MCD_OK;
}

mcd_status mcd_neumann_pressure(mcd_ctx* c, const double* pos, const int8_t* role, const double* normal,
                                const mcd_body* bodies, int n_bodies, double* f) {
    if (!c) return MCD_ERR_ARG;
    if (!role || !normal || !f) return fail(c, MCD_ERR_ARG, "mcd_neumann_pressure: null array%s");
    BodiesDev B;
    if (!make_bodies(c, bodies, n_bodies, &B)) return fail(c, MCD_ERR_ARG, "mcd_neumann_pressure: invalid bodies%s");
    if (B.any_rot && !pos) return fail(c, MCD_ERR_ARG, "mcd_neumann_pressure: a rotating body needs pos%s");
    HIPCHK(c, launch_neumann_pressure(c->m, pos, role, normal, B, f, c->stream), "neumann");
    return MCD_OK;
}

mcd_status mcd_project(mcd_ctx* c, int set, const double* P, const double* f, const double* ustar, double dt,
                       const double* pos, const int8_t* role, const mcd_body* bodies, int n_bodies, double* u) {
    if (!c) return MCD_ERR_ARG;
    if (!valid_set(c, set, true)) return fail(c, MCD_ERR_ARG, "mcd_project: set not built%s");
    if (!P || !ustar || !role || !u || u == ustar) return fail(c, MCD_ERR_ARG, "mcd_project: bad arrays%s");
    if (!(dt > 0) || !isfinite(dt)) return fail(c, MCD_ERR_ARG, "mcd_project: bad dt%s");
    BodiesDev B;
    if (!make_bodies(c, bodies, n_bodies, &B)) return fail(c, MCD_ERR_ARG, "mcd_project: invalid bodies%s");
    if (B.any_rot && !pos) return fail(c, MCD_ERR_ARG, "mcd_project: a rotating body needs pos%s");
    HIPCHK(c, launch_project(c->m, c->sets[set].dev, P, f, ustar, dt, pos, role, B, u, c->stream), "project");
    return MCD_OK;
}

mcd_status mcd_fluid_force(mcd_ctx* c, int set_u, int set_p, const double* u, const double* p,
                           const double* neumann_f, const double* pos, const int8_t* role, const double* normal,
                           const mcd_body* bodies, int n_bodies, double mu, double* force, int* counts) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_fluid_force");
    if (c->dim != 2) return fail(c, MCD_ERR_ARG, "mcd_fluid_force: 2D meshes only%s");
    if (!valid_set(c, set_u, true) || !valid_set(c, set_p, true))
        return fail(c, MCD_ERR_ARG, "mcd_fluid_force: set not built%s");
    if (!u || !p || !pos || !role || !normal || !force || n_bodies < 1 || !(mu >= 0) || !isfinite(mu))
        return fail(c, MCD_ERR_ARG, "mcd_fluid_force: invalid arguments%s");
    BodiesDev B;
    if (!make_bodies(c, bodies, n_bodies, &B)) return fail(c, MCD_ERR_ARG, "mcd_fluid_force: invalid bodies%s");
    double* dout = c->fbuf;
    int* dcnt = (int*)(c->fbuf + 2 * MCD_MAX_BODIES);
    HIPCHK(c, launch_force(c->m, c->sets[set_u].dev, c->sets[set_p].dev, u, p, neumann_f, pos, role, normal, B, mu,
                           dout, dcnt, c->stream),
           "fluid_force");
    double hf[2 * MCD_MAX_BODIES];
    int hc[3 * MCD_MAX_BODIES];
    HIPCHK(c, hipMemcpyAsync(hf, dout, 2 * B.n * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy");
    HIPCHK(c, hipMemcpyAsync(hc, dcnt, 3 * B.n * sizeof(int), hipMemcpyDeviceToHost, c->stream), "copy");
    HIPCHK(c, hipStreamSynchronize(c->stream), "fluid_force");
    for (int k = 0; k < n_bodies; ++k) {
        int s = -1;                   // the body's slot in id order
        for (int q = 0; q < B.n; ++q)
            if (B.id[q] == bodies[k].id) s = q;
        if (hc[3 * s + 2]) return fail(c, MCD_ERR_ARG, "mcd_fluid_force: more than 4096 boundary DPs on a body%s");
        force[2 * k] = hf[2 * s];
        force[2 * k + 1] = hf[2 * s + 1];
        if (counts) {
            counts[2 * k] = hc[3 * s];
            counts[2 * k + 1] = hc[3 * s + 1];
        }
    }
    return MCD_OK;
}

mcd_status mcd_solve_ppe(mcd_ctx* c, int set, const double* rhs, const double* neumann_f, double* p,
                         const mcd_solve_opts* opts, mcd_solve_info* info) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_solve_ppe");
    if (!valid_set(c, set, true)) return fail(c, MCD_ERR_ARG, "mcd_solve_ppe: set not built%s");
    if (!rhs || !p || !opts || !info) return fail(c, MCD_ERR_ARG, "mcd_solve_ppe: null argument%s");
    if (!(opts->tol > 0) || opts->max_iter < 1 ||
        (opts->precision != MCD_PREC_FP64 && opts->precision != MCD_PREC_FP32_REFINE &&
         opts->precision != MCD_PREC_FP32_MATRIX) ||
        (opts->guess != MCD_GUESS_ZERO && opts->guess != MCD_GUESS_CALLER) ||
        (opts->precond != MCD_PRECOND_NONE && opts->precond != MCD_PRECOND_JACOBI &&
         opts->precond != MCD_PRECOND_MG))
        return fail(c, MCD_ERR_ARG, "mcd_solve_ppe: invalid options%s");
    if (opts->precond == MCD_PRECOND_MG && opts->precision == MCD_PREC_FP32_REFINE)
        return fail(c, MCD_ERR_ARG,
                    "mcd_solve_ppe: the multigrid preconditioner takes precision FP64 or FP32_MATRIX (its cycle runs in FP32)%s");
    if (opts->precond == MCD_PRECOND_MG && !krylov_mg_usable(c->kw))
        return fail(c, MCD_ERR_ARG, "mcd_solve_ppe: this mesh cannot be coarsened to 64 cells (multigrid)%s");
    if (opts->precision != MCD_PREC_FP64 &&
        (!(opts->inner_tol > 0) || !(opts->inner_tol < 1) || opts->max_outer < 1 || opts->max_inner < 0 ||
         !(opts->fp64_below >= 0) || !(opts->fp64_below < 1)))
        return fail(c, MCD_ERR_ARG, "mcd_solve_ppe: invalid refinement options%s");
    SolveParams sp{opts->tol,       opts->max_iter,  opts->precision, opts->guess == MCD_GUESS_CALLER,
                   opts->inner_tol, opts->max_outer, opts->check_every, opts->max_inner,
                   opts->fp64_below, opts->precond};
    HIPCHK(c, launch_fill_i32(c->cnt + CNT_BAD, 1, 0, c->stream), "fill");
    SolveOut o;
    // the solve returns after its own stream (ordered after this one) is idle,
    // with the right-hand side's check in o.bad
    HIPCHK(c, solve_ppe_impl(c->m, c->sets[set].dev, *c->kw, rhs, neumann_f, p, sp, &o, c->cnt + CNT_BAD, c->stream),
           "solve");
    const int bad = o.bad;
    info->iterations = o.iterations;
    info->restarts = o.restarts;
    info->refinements = o.refinements;
    info->converged = o.converged;
    info->true_rel_residual = o.rel;
    info->rhs_norm = o.bnorm;
    if (bad) return fail(c, MCD_ERR_ARG, "mcd_solve_ppe: non-finite right-hand side%s");
    if (!o.converged) return fail(c, MCD_ERR_NOT_CONVERGED, "mcd_solve_ppe: tolerance not reached%s");
    return MCD_OK;
}

mcd_status mcd_mg_apply(mcd_ctx* c, int set, const double* in, double* out, int* levels) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_mg_apply");
    if (!valid_set(c, set, true)) return fail(c, MCD_ERR_ARG, "mcd_mg_apply: set not built%s");
    if (!in || !out || !levels) return fail(c, MCD_ERR_ARG, "mcd_mg_apply: null argument%s");
    if (!krylov_mg_usable(c->kw))
        return fail(c, MCD_ERR_ARG, "mcd_mg_apply: this mesh cannot be coarsened to 64 cells%s");
    HIPCHK(c, krylov_mg_apply(c->m, *c->kw, c->sets[set].dev, in, out, levels, c->stream), "mcd_mg_apply");
    return MCD_OK;
}

mcd_status mcd_ppe_residual(mcd_ctx* c, int set, const double* rhs, const double* neumann_f, const double* p,
                            double* r, double* norms) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_ppe_residual");
    if (!valid_set(c, set, true)) return fail(c, MCD_ERR_ARG, "mcd_ppe_residual: set not built%s");
    if (!rhs || !p || !r) return fail(c, MCD_ERR_ARG, "mcd_ppe_residual: null argument%s");
    HIPCHK(c, launch_fill_i32(c->cnt + CNT_BAD, 1, 0, c->stream), "fill");
    if (!norms) {      // r only: enqueued, no wait and no check of the right-hand side
        HIPCHK(c, ppe_residual_impl(c->m, c->sets[set].dev, *c->kw, rhs, neumann_f, p, r, nullptr, c->cnt + CNT_BAD,
                                    c->stream),
               "residual");
        return MCD_OK;
    }
    double nr[2] = {0.0, 0.0};
    HIPCHK(c, ppe_residual_impl(c->m, c->sets[set].dev, *c->kw, rhs, neumann_f, p, r, nr, c->cnt + CNT_BAD, c->stream),
           "residual");
    int bad = 0;
    HIPCHK(c, hipMemcpy(&bad, c->cnt + CNT_BAD, sizeof(int), hipMemcpyDeviceToHost), "copy");
    if (bad) return fail(c, MCD_ERR_ARG, "mcd_ppe_residual: non-finite right-hand side%s");
    norms[0] = nr[0];
    norms[1] = nr[1];
    return MCD_OK;
}

mcd_status mcd_ppe_residual_noalloc(mcd_ctx* c, int set, const double* rhs, const double* neumann_f,
                                    const double* p, double* r, double* norms) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_ppe_residual_noalloc");
    if (!valid_set(c, set, true)) return fail(c, MCD_ERR_ARG, "mcd_ppe_residual_noalloc: set not built%s");
    if (!rhs || !p || !r) return fail(c, MCD_ERR_ARG, "mcd_ppe_residual_noalloc: null argument%s");
    double nr[2] = {0.0, 0.0};
    int bad = 0;
    HIPCHK(c, ppe_residual_noalloc_impl(c->device, c->m, c->sets[set].dev, rhs, neumann_f, p, r, nr, &bad,
                                        c->stream),
           "residual (no allocation)");
    if (bad) return fail(c, MCD_ERR_ARG, "mcd_ppe_residual_noalloc: non-finite right-hand side%s");
    if (norms) {
        norms[0] = nr[0];
        norms[1] = nr[1];
    }
    return MCD_OK;
}

size_t mcd_noalloc_scratch_bytes(void) { return noalloc_scratch_bytes(); }

// ---------------------------------------------------------------------------
// Learned initial guess
// ---------------------------------------------------------------------------

struct mcd_model {
    mcd_ctx* ctx;
    UNet* net;
};

mcd_status mcd_model_create(mcd_ctx* c, int levels, const int* channels, int body_id, mcd_model** out) {
    if (!c || !channels || !out) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_model_create");
    *out = nullptr;
    if (levels < 2 || levels > 5) return fail(c, MCD_ERR_ARG, "mcd_model_create: levels must be 2..5%s");
    const int H = c->m.n[1], W = c->m.n[0], D = c->dim == 3 ? c->m.n[2] : 1;
    const int q = 1 << (levels - 1);
    if ((H % q) || (W % q) || (c->dim == 3 && (D % q)))
        return fail(c, MCD_ERR_ARG, "mcd_model_create: mesh not divisible by 2^(levels-1)%s");
    for (int l = 0; l < levels; ++l)
        if (channels[l] < 16 || channels[l] > 256 || channels[l] % 16)
            return fail(c, MCD_ERR_ARG, "mcd_model_create: channels must be multiples of 16 in [16, 256]%s");
    if (body_id < 1 || body_id >= MCD_MAX_IDS) return fail(c, MCD_ERR_ARG, "mcd_model_create: bad body id%s");
    UNet* u = nullptr;
    hipError_t e = unet_create(c->dim, D, H, W, levels, channels, body_id, c->desc.walls ? c->desc.wall_id : -2, &u);
    if (e != hipSuccess) {
        unet_free(u);
        return e == hipErrorOutOfMemory ? MCD_ERR_OOM : hipfail(c, e, "mcd_model_create");
    }
    *out = new mcd_model{c, u};
    return MCD_OK;
}

void mcd_model_destroy(mcd_model* md) {
    if (!md) return;
    {
        std::lock_guard<std::mutex> lk(g_life_mu);
        if (g_open_recordings > 0) {
            g_pending_model.push_back(md);
            return;
        }
    }
    destroy_model_now(md);
}

static void destroy_model_now(mcd_model* md) {
    (void)hipStreamSynchronize(md->ctx->stream);
    unet_free(md->net);
    delete md;
}

size_t mcd_model_num_params(const mcd_model* md) { return md ? unet_nparams(*md->net) : 0; }

mcd_status mcd_model_set_params(mcd_model* md, const float* theta, size_t n) {
    if (!md || !theta || n != unet_nparams(*md->net)) return MCD_ERR_ARG;
    NO_CAPTURE(md->ctx, "mcd_model_set_params");
    mcd_ctx* c = md->ctx;
    HIPCHK(c, hipMemcpyAsync(unet_theta(*md->net), theta, n * 4, hipMemcpyHostToDevice, c->stream), "set_params");
    HIPCHK(c, unet_weights_to_bf16(*md->net, c->stream), "set_params");
    unet_reset_optimizer(*md->net, c->stream);
    HIPCHK(c, hipStreamSynchronize(c->stream), "set_params");
    return MCD_OK;
}

mcd_status mcd_model_get_params(mcd_model* md, float* theta, size_t n) {
    if (!md || !theta || n != unet_nparams(*md->net)) return MCD_ERR_ARG;
    NO_CAPTURE(md->ctx, "mcd_model_get_params");
    mcd_ctx* c = md->ctx;
    HIPCHK(c, hipStreamSynchronize(c->stream), "get_params");
    HIPCHK(c, hipMemcpy(theta, unet_theta(*md->net), n * 4, hipMemcpyDeviceToHost), "get_params");
    return MCD_OK;
}

mcd_status mcd_model_get_grads(mcd_model* md, float* grad, size_t n) {
    if (!md || !grad || n != unet_nparams(*md->net)) return MCD_ERR_ARG;
    NO_CAPTURE(md->ctx, "mcd_model_get_grads");
    mcd_ctx* c = md->ctx;
    HIPCHK(c, hipStreamSynchronize(c->stream), "get_grads");
    HIPCHK(c, hipMemcpy(grad, unet_grad(*md->net), n * 4, hipMemcpyDeviceToHost), "get_grads");
    return MCD_OK;
}

mcd_status mcd_model_output(mcd_model* md, float* h) {
    if (!md || !h) return MCD_ERR_ARG;
    NO_CAPTURE(md->ctx, "mcd_model_output");
    mcd_ctx* c = md->ctx;
    HIPCHK(c, hipMemcpyAsync(h, unet_head_out(*md->net), c->Nc * 4, hipMemcpyDeviceToDevice, c->stream), "output");
    return MCD_OK;
}

mcd_status mcd_model_set_output_scale(mcd_model* md, double s) {
    if (!md) return MCD_ERR_ARG;
    NO_CAPTURE(md->ctx, "mcd_model_set_output_scale");
    if (!(s > 0) || !isfinite(s)) return fail(md->ctx, MCD_ERR_ARG, "mcd_model_set_output_scale: s must be > 0%s");
    unet_set_output_scale(*md->net, s);
    return MCD_OK;
}

mcd_status mcd_model_infer(mcd_model* md, const double* rhs, const double* p_prev, const int8_t* role,
                           const mcd_bc_table* bc, double* p_out) {
    if (!md || !rhs || !p_prev || !role || !p_out) return MCD_ERR_ARG;
    NO_CAPTURE(md->ctx, "mcd_model_infer");
    mcd_ctx* c = md->ctx;
    BcDev b;
    if (!make_bc(bc, &b)) return fail(c, MCD_ERR_ARG, "mcd_model_infer: invalid bc table%s");
    HIPCHK(c, unet_infer(*md->net, rhs, p_prev, role, b, p_out, c->stream), "mcd_model_infer");
    return MCD_OK;
}

mcd_status mcd_model_train_step(mcd_model* md, const double* rhs, const double* p_prev, const double* p_target,
                                const int8_t* role, const mcd_bc_table* bc, double lr, double* loss) {
    if (!md || !rhs || !p_prev || !p_target || !role) return MCD_ERR_ARG;
    NO_CAPTURE(md->ctx, "mcd_model_train_step");
    mcd_ctx* c = md->ctx;
    BcDev b;
    if (!make_bc(bc, &b)) return fail(c, MCD_ERR_ARG, "mcd_model_train_step: invalid bc table%s");
    if (!(lr >= 0) || !isfinite(lr)) return fail(c, MCD_ERR_ARG, "mcd_model_train_step: bad learning rate%s");
    HIPCHK(c, unet_train_step(*md->net, rhs, p_prev, p_target, role, b, (float)lr, c->stream, loss),
           "mcd_model_train_step");
    return MCD_OK;
}

mcd_status mcd_autotune(mcd_ctx* c, int set, int iters, mcd_tuning* out) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_autotune");
    if (!valid_set(c, set, true)) return fail(c, MCD_ERR_ARG, "mcd_autotune: set not built%s");
    if (!out || iters < 1 || iters > 100000) return fail(c, MCD_ERR_ARG, "mcd_autotune: invalid arguments%s");
    *out = mcd_tuning{};
    out->chosen = -1;
    HIPCHK(c, hipStreamSynchronize(c->stream), "autotune");
    HIPCHK(c, krylov_autotune(c->m, c->sets[set].dev, *c->kw, iters, MCD_TUNE_MAX, &out->n, out->grid, out->depth,
                              out->us_per_iter, &out->chosen),
           "autotune");
    return MCD_OK;
}

mcd_status mcd_set_shape(mcd_ctx* c, int grid, int depth) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_set_shape");
    const hipError_t e = krylov_set_shape(c->m, *c->kw, grid, depth);
    if (e == hipErrorInvalidValue) return fail(c, MCD_ERR_ARG, "mcd_set_shape: shape outside the limits%s");
    HIPCHK(c, e, "set_shape");
    return MCD_OK;
}

mcd_status mcd_get_shape(mcd_ctx* c, int* grid, int* depth, int* blocks) {
    if (!c) return MCD_ERR_ARG;
    if (!grid || !depth || !blocks) return fail(c, MCD_ERR_ARG, "mcd_get_shape: null argument%s");
    krylov_get_shape(*c->kw, grid, depth, blocks);
    return MCD_OK;
}

mcd_status mcd_profile(mcd_ctx* c, int enable) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_profile");
    HIPCHK(c, krylov_profile(c->kw, enable ? 1 : 0), "mcd_profile");
    return MCD_OK;
}

mcd_status mcd_profile_read(mcd_ctx* c, double* ms_p, long long* n_p, double* ms_s, long long* n_s, int reset) {
    if (!c || !ms_p || !n_p || !ms_s || !n_s) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_profile_read");
    krylov_profile_read(c->kw, ms_p, n_p, ms_s, n_s, nullptr, nullptr, reset);
    return MCD_OK;
}

mcd_status mcd_profile_read_split(mcd_ctx* c, double* ms, long long* n, int reset) {
    if (!c || !ms || !n) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_profile_read_split");
    double p, s;
    long long np_, ns_;
    double m32[2];
    long long c32[2];
    krylov_profile_read(c->kw, &p, &np_, &s, &ns_, m32, c32, reset);
    ms[0] = p - m32[0];
    ms[1] = s - m32[1];
    ms[2] = m32[0];
    ms[3] = m32[1];
    n[0] = np_ - c32[0];
    n[1] = ns_ - c32[1];
    n[2] = c32[0];
    n[3] = c32[1];
    return MCD_OK;
}

mcd_status mcd_ppe_wide(mcd_ctx* c, int half, double re_over_l0, const double* pos, const int8_t* role,
                        const double* normal, const mcd_bc_table* bc, const double* rhs, const double* neumann_f,
                        double* p, double tol, int max_iter, mcd_wide_info* info) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_ppe_wide");
    if (c->dim != 2) return fail(c, MCD_ERR_ARG, "mcd_ppe_wide: 2D meshes only%s");
    if (half < 1 || half > 4 || c->m.n[0] < 2 * half + 1 || c->m.n[1] < 2 * half + 1)
        return fail(c, MCD_ERR_ARG, "mcd_ppe_wide: half width outside 1 .. 4 or wider than the mesh%s");
    if (!(re_over_l0 > 0) || !isfinite(re_over_l0) || !(tol > 0) || max_iter < 0)
        return fail(c, MCD_ERR_ARG, "mcd_ppe_wide: bad r_e, tolerance or iteration limit%s");
    if (!pos || !role || !normal || !rhs || !p || !info) return fail(c, MCD_ERR_ARG, "mcd_ppe_wide: null array%s");
    BcDev B;
    if (!make_bc(bc, &B)) return fail(c, MCD_ERR_ARG, "mcd_ppe_wide: invalid boundary table%s");
    WideResult r;
    HIPCHK(c, wide_ppe(c->m, &c->ww, half, re_over_l0 * c->m.l0, c->rs, c->prm.weight_kind, pos, role, normal, B, rhs,
                       neumann_f, p, tol, max_iter, &r, c->stream),
           "mcd_ppe_wide");
    info->iterations = r.iterations;
    info->converged = r.converged;
    info->singular = r.singular;
    info->true_rel_residual = r.true_rel_residual;
    info->build_ms = r.build_ms;
    info->solve_ms = r.solve_ms;
    if (r.singular) return fail(c, MCD_ERR_SINGULAR, "mcd_ppe_wide: singular MLS fits%s");
    if (!r.converged) return fail(c, MCD_ERR_NOT_CONVERGED, "mcd_ppe_wide: not converged%s");
    return MCD_OK;
}

mcd_status mcd_ppe_wide_matrix(mcd_ctx* c, double* A) {
    if (!c) return MCD_ERR_ARG;
    NO_CAPTURE(c, "mcd_ppe_wide_matrix");
    if (!A || !c->ww) return fail(c, MCD_ERR_ARG, "mcd_ppe_wide_matrix: no wide PPE assembled yet%s");
    HIPCHK(c, wide_lap_planes(c->ww, A, c->stream), "mcd_ppe_wide_matrix");
    HIPCHK(c, hipStreamSynchronize(c->stream), "mcd_ppe_wide_matrix");
    return MCD_OK;
}

mcd_status mcd_graph_begin(mcd_ctx* c, int slot) {
    if (!c) return MCD_ERR_ARG;
    if (slot < 0 || slot >= MCD_MAX_GRAPHS) return fail(c, MCD_ERR_ARG, "mcd_graph_begin: slot out of range%s");
    NO_CAPTURE(c, "mcd_graph_begin");
    if (!c->cap_st) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking), "capture stream");
    // relaxed: other work of this thread (an allocator, another stream) does not
    // invalidate the recording; the recorded calls themselves never wait
    HIPCHK(c, hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeRelaxed), "mcd_graph_begin");
    recording_opened();
    c->user_st = c->stream;
    c->stream = c->cap_st;
    c->capturing = slot;
    c->cap_failed = false;
    return MCD_OK;
}

mcd_status mcd_graph_end(mcd_ctx* c, int slot, int launch) {
    if (!c) return MCD_ERR_ARG;
    if (c->capturing < 0 || slot != c->capturing)
        return fail(c, MCD_ERR_ARG, "mcd_graph_end: no capture of this slot is open%s");
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_st, &g);
    c->stream = c->user_st;
    c->capturing = -1;
    recording_closed();
    if (ec != hipSuccess || c->cap_failed || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();      // the failed recording leaves no error behind for later calls
        const bool failed = c->cap_failed;
        c->cap_failed = false;
        if (failed) {
            c->err = "mcd_graph_end: a call failed while the graph was captured (" + c->err + "); nothing was run";
            return MCD_ERR_ARG;
        }
        return hipfail(c, ec != hipSuccess ? ec : hipErrorInvalidValue, "mcd_graph_end");
    }
    hipError_t e = hipErrorInvalidValue;
    if (c->gexec[slot]) {
        // same sequence of calls as the slot's executable graph: update it in place
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res;
        e = hipGraphExecUpdate(c->gexec[slot], g, &bad, &res);
        if (e == hipSuccess && res == hipGraphExecUpdateSuccess) {
            c->g_upd[slot]++;
        } else {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(c->gexec[slot]);
            c->gexec[slot] = nullptr;
            e = hipErrorInvalidValue;
        }
    }
    if (!c->gexec[slot]) {
        e = hipGraphInstantiate(&c->gexec[slot], g, nullptr, nullptr, 0);
        if (e != hipSuccess) c->gexec[slot] = nullptr;
        else c->g_inst[slot]++;
    }
    (void)hipGraphDestroy(g);
    HIPCHK(c, e, "mcd_graph_end instantiate");
    if (launch) HIPCHK(c, hipGraphLaunch(c->gexec[slot], c->stream), "mcd_graph_end launch");
    return MCD_OK;
}

mcd_status mcd_graph_launch(mcd_ctx* c, int slot) {
    if (!c) return MCD_ERR_ARG;
    if (slot < 0 || slot >= MCD_MAX_GRAPHS || !c->gexec[slot])
        return fail(c, MCD_ERR_ARG, "mcd_graph_launch: slot holds no graph%s");
    NO_CAPTURE(c, "mcd_graph_launch");
    HIPCHK(c, hipGraphLaunch(c->gexec[slot], c->stream), "mcd_graph_launch");
    return MCD_OK;
}

mcd_status mcd_graph_stats(mcd_ctx* c, int slot, int* instantiated, int* updated) {
    if (!c) return MCD_ERR_ARG;
    if (slot < 0 || slot >= MCD_MAX_GRAPHS || !instantiated || !updated)
        return fail(c, MCD_ERR_ARG, "mcd_graph_stats: bad argument%s");
    *instantiated = c->g_inst[slot];
    *updated = c->g_upd[slot];
    return MCD_OK;
}

}  // extern "C"
