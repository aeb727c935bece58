// Learned PPE initial guess: a U-Net on the background mesh (one DP per
// cell makes DP arrays channels-last images: (y, x, C) in 2D, (z, y, x, C)
// in 3D, x fastest).  Kernels are templated on the dimension: a "3x3"
// convolution has 9 taps in 2D and 27 in 3D, pooling and upsampling act on
// 2x2 or 2x2x2 blocks.
//
// BF16 weights and activations, FP32 accumulation on the matrix cores
// (v_mfma_f32_32x32x16_bf16).  A 3x3 convolution is an implicit GEMM:
//   Y[p][n] = sum_t sum_k In[p + o_t][k] W[t][n][k],
// rows = pixels, columns = output channels, K = taps x input channels.
// The input In of a decoder convolution is concat(skip (this level),
// nearest 2x upsample of the coarser level) and is read directly from the
// two tensors, so neither the upsampled image nor the concatenation is ever
// written.  The data gradient is the same kernel with the tap-flipped,
// transposed weights; the weight gradient is a GEMM over pixels with
// deterministic per-chunk partial sums.
//
// Lane layout of the 32x32x16 bf16 MFMA (gfx950): lane l holds
// A[row = l%32][k = 8(l/32) + j], B[k = 8(l/32) + j][col = l%32], j = 0..7,
// and D element i at row 8(i/4) + 4(l/32) + i%4, col l%32.
#include "common.h"

namespace mcd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kIn = 16;       // packed input channels
constexpr int kMaxLevels = 5;

// Input of a convolution: concat(x0 (c0 channels, D x H x W), up2(x1) (c1
// channels, (D/2 in 3D, else 1) x (H/2) x (W/2))).  D = 1 and zs = 0 in 2D;
// zs = 1 in 3D (the coarse level is halved in z too).
struct ConvIn {
    const __bf16* x0;
    int c0;
    const __bf16* x1;
    int c1;
    int D, H, W;
    int zs;
};

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
    return z;
}

__device__ __forceinline__ bool outside(const ConvIn& in, int z, int y, int x) {
    return z < 0 || z >= in.D || y < 0 || y >= in.H || x < 0 || x >= in.W;
}

// pixel index of (z, y, x) in the fine image and of its parent in the coarse one
__device__ __forceinline__ size_t fine_px(const ConvIn& in, int z, int y, int x) {
    return ((size_t)z * in.H + y) * in.W + x;
}
__device__ __forceinline__ size_t coarse_px(const ConvIn& in, int z, int y, int x) {
    return ((size_t)(z >> in.zs) * (in.H >> 1) + (y >> 1)) * (in.W >> 1) + (x >> 1);
}

// 8 consecutive input channels [k0, k0 + 8) at (z, y, x); zero outside the image.
__device__ __forceinline__ bf16x8 load8(const ConvIn& in, int z, int y, int x, int k0) {
    if (outside(in, z, y, x)) return zero8();
    if (k0 < in.c0) return *(const bf16x8*)(in.x0 + fine_px(in, z, y, x) * in.c0 + k0);
    return *(const bf16x8*)(in.x1 + coarse_px(in, z, y, x) * in.c1 + (k0 - in.c0));
}

__device__ __forceinline__ __bf16 load1(const ConvIn& in, int z, int y, int x, int k) {
    if (outside(in, z, y, x)) return (__bf16)0.0f;
    if (k < in.c0) return in.x0[fine_px(in, z, y, x) * in.c0 + k];
    return in.x1[coarse_px(in, z, y, x) * in.c1 + (k - in.c0)];
}

// taps of a convolution and the offset of tap t along z, y, x (-1..1)
template <int DIM>
struct Taps {
    static constexpr int T = DIM == 3 ? 27 : 9;
    static constexpr int HZ = DIM == 3 ? 3 : 1;     // planes of the halo
    __device__ static int dz(int t) { return DIM == 3 ? t / 9 - 1 : 0; }
    __device__ static int dy(int t) { return (t / 3) % 3 - 1; }
    __device__ static int dx(int t) { return t % 3 - 1; }
};

// Implicit-GEMM 3x3 convolution on LDS tiles.  Wk: [T][NT*32][K] bf16
// (K = c0 + c1, zero rows for n >= cout).  A block of 4 waves owns a tile of
// 4 image rows x 32 columns of one plane (wave w: row w, one pixel per MFMA
// row).  The input is staged through LDS 16 channels at a time as a
// (4+2) x (32+2) halo tile (times the 3 planes z-1..z+1 in 3D), so each
// input pixel is read from memory once per chunk and the taps read their A
// fragments (8 channels per lane) from LDS; B fragments come from the
// (cache-resident) weights.  The epilogue (bias, ReLU, BF16) goes through a
// per-wave 32 x 32 LDS tile so that every lane stores 16 contiguous bytes;
// cout must be a multiple of 16.
constexpr int kCR = 4, kCC = 32, kHR = kCR + 2, kHC = kCC + 2, kHalo = kHR * kHC;

// Epilogue of a 32-pixel x 32-channel accumulator tile of wave `wave`: bias,
// ReLU and BF16 through the wave's 32 x 32 LDS tile sw (rows kSW apart, so
// that the two halves of the wave write different banks), so that every lane
// stores 16 contiguous bytes of output plane z.
constexpr int kSW = 40;
__device__ __forceinline__ void conv_epilogue(const f32x16& acc, __bf16* sw, const ConvIn& in, int l, int wave,
                                              int tx0, int ty0, int z, int nt, const float* __restrict__ bias,
                                              int cout, int relu, __bf16* __restrict__ Y) {
    const int row = l >> 1, col0 = 16 * (l & 1);
    const int y = ty0 + wave, x = tx0 + row;
    const int n = nt * 32 + (l & 31);
    const float bn = (bias && n < cout) ? bias[n] : 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        float v = acc[i] + bn;
        if (relu) v = fmaxf(v, 0.0f);
        sw[(8 * (i >> 2) + 4 * (l >> 5) + (i & 3)) * kSW + (l & 31)] = (__bf16)v;
    }
    __syncthreads();
    const int nc = nt * 32 + col0;
    if (y < in.H && x < in.W && nc < cout) {
        const bf16x8* src = (const bf16x8*)(sw + row * kSW + col0);
        bf16x8* dst = (bf16x8*)(Y + fine_px(in, z, y, x) * cout + nc);
        dst[0] = src[0];
        dst[1] = src[1];
    }
}

// Grid: x = column tiles, y = row tiles x planes, z = 32-column tiles of
// output channels (so that small coarse-level images still spread over the
// whole chip).  Used for 2D; 3D convolutions go through k_conv3_march.
template <int DIM>
__global__ __launch_bounds__(256) void k_conv_mfma(ConvIn in, const __bf16* __restrict__ Wk, int np,
                                                   const float* __restrict__ bias, int cout, int relu,
                                                   __bf16* __restrict__ Y) {
    using TP = Taps<DIM>;
    __shared__ __attribute__((aligned(16))) __bf16 tile[TP::HZ * kHalo * 16];
    __shared__ __attribute__((aligned(16))) __bf16 stage[4][32 * kSW];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int nty = (in.H + kCR - 1) / kCR;
    const int tx0 = blockIdx.x * kCC, ty0 = (blockIdx.y % nty) * kCR, z = blockIdx.y / nty, nt = blockIdx.z;
    const int K = in.c0 + in.c1;
    const int half = 8 * (l >> 5);
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += 16) {
        // stage channels [k0, k0 + 16) of the halo tile: 2 vectors of 8 per pixel
        for (int v = threadIdx.x; v < 2 * TP::HZ * kHalo; v += 256) {
            const int px = v >> 1, hv = v & 1;
            const int pz = px / kHalo, pr = px % kHalo;
            const int y = ty0 - 1 + pr / kHC, x = tx0 - 1 + pr % kHC;
            *(bf16x8*)(tile + px * 16 + 8 * hv) = load8(in, z - TP::HZ / 2 + pz, y, x, k0 + 8 * hv);
        }
        __syncthreads();
        const __bf16* wn = Wk + (size_t)(nt * 32 + (l & 31)) * K + k0 + half;
#pragma unroll
        for (int t = 0; t < TP::T; ++t) {
            // halo offsets 0..2 along z (3D), y, x
            const int hz = TP::dz(t) + TP::HZ / 2, hy = TP::dy(t) + 1, hx = TP::dx(t) + 1;
            const bf16x8 a = *(const bf16x8*)(tile + ((hz * kHR + wave + hy) * kHC + (l & 31) + hx) * 16 + half);
            const bf16x8 b = *(const bf16x8*)(wn + (size_t)t * np * K);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    conv_epilogue(acc, stage[wave], in, l, wave, tx0, ty0, z, nt, bias, cout, relu, Y);
}

// 3D convolution marching along z.  A block owns a 4 x 32 tile of one
// column of up to zb consecutive output planes and one 32-wide tile of
// output channels (grid: x = column tiles, y = row tiles x plane groups,
// z = channel tiles).  Work proceeds in stages (input plane p, 16-channel
// chunk): the stage's 6 x 34 halo tile and the 27 taps' B fragments of the
// chunk are staged in LDS (the B fragments once per block when K is one
// chunk), and the next stage's loads are issued into registers before the
// matrix-core work of the current one.  Plane p contributes to the outputs
// p + 1, p and p - 1 (taps with dz = -1, 0, +1), kept in three rolling
// accumulators; the A fragment of a (dy, dx) offset is read once for the
// three of them.  After plane p the output p - 1 is complete and goes
// through conv_epilogue.  Each input plane is read once per block instead of
// three times.
constexpr int kTap3 = 27, kWVec = kTap3 * 32 * 2;      // B vectors (8 bf16) of a chunk
constexpr int kAReg = (2 * kHalo + 255) / 256, kBReg = (kWVec + 255) / 256;
// LDS stride of a pixel's 16 input channels (A): 48 bytes, so that the
// 16-byte fragment reads of consecutive lanes fall in different banks
constexpr int kPX = 24;

__global__ __launch_bounds__(256, 3) void k_conv3_march(ConvIn in, const __bf16* __restrict__ Wk, int np,
                                                     const float* __restrict__ bias, int cout, int relu, int zb,
                                                     __bf16* __restrict__ Y) {
    __shared__ __attribute__((aligned(16))) __bf16 tile[kHalo * kPX];
    __shared__ __attribute__((aligned(16))) __bf16 wt[kTap3 * 32 * 16];
    __shared__ __attribute__((aligned(16))) __bf16 stage[4][32 * kSW];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int nty = (in.H + kCR - 1) / kCR;
    const int tx0 = blockIdx.x * kCC, ty0 = (blockIdx.y % nty) * kCR, z0 = (blockIdx.y / nty) * zb;
    const int nt = blockIdx.z;
    const int z1 = z0 + zb < in.D ? z0 + zb : in.D;      // outputs [z0, z1)
    const int K = in.c0 + in.c1;
    const int nch = K / 16;
    const int half = 8 * (l >> 5);
    const int pf = z0 - 1 > 0 ? z0 - 1 : 0, pl = z1 < in.D - 1 ? z1 : in.D - 1;
    const int nst = (pl - pf + 1) * nch;                 // stages (plane, chunk), planes [pf, pl]
    bf16x8 ra[kAReg], rb[kBReg];
    auto fetch = [&](int si) {
        const int p = pf + si / nch, k0 = (si % nch) * 16;
#pragma unroll
        for (int j = 0; j < kAReg; ++j) {
            const int v = threadIdx.x + 256 * j;
            if (v < 2 * kHalo) {
                const int px = v >> 1, hv = v & 1;
                ra[j] = load8(in, p, ty0 - 1 + px / kHC, tx0 - 1 + px % kHC, k0 + 8 * hv);
            }
        }
        if (nch > 1 || si == 0) {
#pragma unroll
            for (int j = 0; j < kBReg; ++j) {
                const int v = threadIdx.x + 256 * j;
                if (v < kWVec) {
                    const int t = v >> 6, n = (v >> 1) & 31, hv = v & 1;
                    rb[j] = *(const bf16x8*)(Wk + ((size_t)t * np + nt * 32 + n) * K + k0 + 8 * hv);
                }
            }
        }
    };
    auto publish = [&](int si) {
#pragma unroll
        for (int j = 0; j < kAReg; ++j) {
            const int v = threadIdx.x + 256 * j;
            if (v < 2 * kHalo) *(bf16x8*)(tile + (v >> 1) * kPX + 8 * (v & 1)) = ra[j];
        }
        if (nch > 1 || si == 0) {
#pragma unroll
            for (int j = 0; j < kBReg; ++j) {
                const int v = threadIdx.x + 256 * j;
                if (v < kWVec) *(bf16x8*)(wt + ((v >> 6) * 32 + ((v >> 1) & 31)) * 16 + 8 * (v & 1)) = rb[j];
            }
        }
    };
    f32x16 a0, a1, a2;                                   // outputs p - 1, p, p + 1
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        a0[i] = 0.0f;
        a1[i] = 0.0f;
        a2[i] = 0.0f;
    }
    int si = 0;
    if (nst > 0) fetch(0);
    for (int p = z0 - 1; p <= z1; ++p) {
        if (p >= 0 && p < in.D) {
            const bool o0 = p - 1 >= z0 && p - 1 < z1, o1 = p >= z0 && p < z1, o2 = p + 1 >= z0 && p + 1 < z1;
            for (int c = 0; c < nch; ++c, ++si) {
                publish(si);
                __syncthreads();
                if (si + 1 < nst) fetch(si + 1);
                const __bf16* wl = wt + (l & 31) * 16 + half;
#pragma unroll
                for (int hy = 0; hy < 3; ++hy)
#pragma unroll
                    for (int hx = 0; hx < 3; ++hx) {
                        const int t2 = hy * 3 + hx;           // tap within a plane
                        const bf16x8 a = *(const bf16x8*)(tile + ((wave + hy) * kHC + (l & 31) + hx) * kPX + half);
                        // output p - 1 reads plane p with dz = +1 (taps 18..26), output p with dz = 0
                        // (taps 9..17), output p + 1 with dz = -1 (taps 0..8)
                        if (o0) a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                    a, *(const bf16x8*)(wl + (18 + t2) * 32 * 16), a0, 0, 0, 0);
                        if (o1) a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                    a, *(const bf16x8*)(wl + (9 + t2) * 32 * 16), a1, 0, 0, 0);
                        if (o2) a2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                    a, *(const bf16x8*)(wl + t2 * 32 * 16), a2, 0, 0, 0);
                    }
                __syncthreads();
            }
        }
        if (p - 1 >= z0 && p - 1 < z1)
            conv_epilogue(a0, stage[wave], in, l, wave, tx0, ty0, p - 1, nt, bias, cout, relu, Y);
        a0 = a1;
        a1 = a2;
#pragma unroll
        for (int i = 0; i < 16; ++i) a2[i] = 0.0f;
    }
}

// Weight gradient: part[chunk][t][k][n] = sum over the chunk's pixels p of
// In[p + o_t][k] dY[p][n]  (k < K padded to 32, n < cout padded to 32).
// One wave per (t, k-tile, n-tile) output tile; blockIdx.x = pixel chunk.
template <int DIM>
__global__ __launch_bounds__(256) void k_conv_wgrad(ConvIn in, const __bf16* __restrict__ dY, int cout, int ktiles,
                                                    int ntiles, int chunk, float* __restrict__ part) {
    using TP = Taps<DIM>;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int tile = blockIdx.y * 4 + wave;
    const int per_tap = ktiles * ntiles;
    if (tile >= TP::T * per_tap) return;
    const int t = tile / per_tap, kt = (tile % per_tap) / ntiles, nt = tile % ntiles;
    const int dz = TP::dz(t), dy = TP::dy(t), dx = TP::dx(t);
    const int K = in.c0 + in.c1;
    const int P = in.D * in.H * in.W;
    const int q_begin = blockIdx.x * chunk;
    const int q_end = min(P, q_begin + chunk);
    const int k = kt * 32 + (l & 31), n = nt * 32 + (l & 31);
    const int half = 8 * (l >> 5);
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    for (int q0 = q_begin; q0 < q_end; q0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int q = q0 + half + j;
            const bool ok = q < q_end;
            const int x = ok ? q % in.W : 0, y = ok ? (q / in.W) % in.H : 0, z = ok ? q / (in.W * in.H) : 0;
            a[j] = (ok && k < K) ? load1(in, z + dz, y + dy, x + dx, k) : (__bf16)0.0f;
            b[j] = (ok && n < cout) ? dY[(size_t)q * cout + n] : (__bf16)0.0f;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    // D rows are k (from A), columns n (from B)
    const int Kp = ktiles * 32, Np = ntiles * 32;
    float* dst = part + ((size_t)blockIdx.x * TP::T + t) * Kp * Np;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int kr = kt * 32 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
        dst[(size_t)kr * Np + n] = acc[i];
    }
}

// grad[t][k][n] (theta layout W[t][ci][co]) = sum over chunks of part (T taps).
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nchunks, int T, int K, int cout, int Kp, int Np,
                               float* __restrict__ g) {
    const int total = T * K * cout;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int t = e / (K * cout), k = (e / cout) % K, n = e % cout;
        double s = 0.0;
        for (int c = 0; c < nchunks; ++c) s += part[((size_t)c * T + t) * Kp * Np + (size_t)k * Np + n];
        g[e] = (float)s;
    }
}

// Column sums of a [P][C] bf16 matrix (C a multiple of 8, at most 256):
// partials per block, then a reduction.  Thread (rho, g) of a block sums
// channels [8g, 8g + 8) over rows r0 + rho, r0 + rho + R, ... with 16-byte
// loads (consecutive threads read consecutive bytes of a row), then the R
// row phases are summed in a fixed order through LDS.
__global__ __launch_bounds__(256) void k_colsum_part(const __bf16* __restrict__ X, int P, int C, int rows_per_block,
                                                     float* __restrict__ part) {
    __shared__ float red[2048];
    const int G = C / 8, R = 256 / G;
    const int g = threadIdx.x % G, rho = threadIdx.x / G;
    const int r0 = blockIdx.x * rows_per_block, r1 = min(P, r0 + rows_per_block);
    float acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.0f;
    if (rho < R) {
        for (int r = r0 + rho; r < r1; r += R) {
            const bf16x8 v = *(const bf16x8*)(X + (size_t)r * C + 8 * g);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] += (float)v[j];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) red[rho * C + 8 * g + j] = acc[j];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        float sum = 0.0f;
        for (int q = 0; q < R; ++q) sum += red[q * C + c];
        part[(size_t)blockIdx.x * C + c] = sum;
    }
}

__global__ void k_colsum_reduce(const float* __restrict__ part, int nblk, int C, float* __restrict__ g) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(size_t)b * C + c];
        g[c] = (float)s;
    }
}

__global__ void k_relu_mask(__bf16* __restrict__ g, const __bf16* __restrict__ y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (!((float)y[i] > 0.0f)) g[i] = (__bf16)0.0f;
}

// Sum over the 2x2 (2D) or 2x2x2 (3D) block of coarse pixel (z, y, x) of a
// fine D x H x W image, channel offset `c` of row width C.
template <int DIM>
__device__ __forceinline__ float block_sum2(const __bf16* __restrict__ f, int H, int W, int C, int z, int y, int x,
                                            int c) {
    float s = 0.0f;
#pragma unroll
    for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz) {
        const int zf = DIM == 3 ? 2 * z + dz : z;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx)
                s += (float)f[(((size_t)zf * H + 2 * y + dy) * W + 2 * x + dx) * C + c];
    }
    return s;
}

// Mean pool over 2x2 (2x2x2) blocks: out (D' x H/2 x W/2 x C) from in
// (D x H x W x C), D' = D/2 in 3D, 1 in 2D.
template <int DIM>
__global__ void k_pool(const __bf16* __restrict__ in, int D, int H, int W, int C, __bf16* __restrict__ out) {
    const int H2 = H >> 1, W2 = W >> 1, D2 = DIM == 3 ? D >> 1 : 1;
    const int total = D2 * H2 * W2 * C;
    const float f = DIM == 3 ? 0.125f : 0.25f;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int c = e % C, p = e / C, x = p % W2, y = (p / W2) % H2, z = p / (W2 * H2);
        out[e] = (__bf16)(f * block_sum2<DIM>(in, H, W, C, z, y, x, c));
    }
}

// g_fine (D x H x W x C) += g_coarse / 4 (/ 8 in 3D) broadcast over each block.
template <int DIM>
__global__ void k_pool_bwd_add(const __bf16* __restrict__ gc, int D, int H, int W, int C, __bf16* __restrict__ gf) {
    const int total = D * H * W * C;
    const int zs = DIM == 3 ? 1 : 0;
    const float f = DIM == 3 ? 0.125f : 0.25f;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int c = e % C, p = e / C, x = p % W, y = (p / W) % H, z = p / (W * H);
        const size_t pc = ((size_t)(z >> zs) * (H >> 1) + (y >> 1)) * (W >> 1) + (x >> 1);
        gf[e] = (__bf16)((float)gf[e] + f * (float)gc[pc * C + c]);
    }
}

// Gradient of concat(skip, up2(coarse)): skip part written to gs, upsample
// part summed over each 2x2 (2x2x2) block into gcoarse.
template <int DIM>
__global__ void k_cat_split(const __bf16* __restrict__ gcat, int D, int H, int W, int c0, int c1,
                            __bf16* __restrict__ gs, __bf16* __restrict__ gcoarse) {
    const int C = c0 + c1;
    const int n_skip = D * H * W * c0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_skip; e += gridDim.x * blockDim.x) {
        const int c = e % c0, p = e / c0;
        gs[e] = gcat[(size_t)p * C + c];
    }
    const int H2 = H >> 1, W2 = W >> 1, D2 = DIM == 3 ? D >> 1 : 1;
    const int n_c = D2 * H2 * W2 * c1;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_c; e += gridDim.x * blockDim.x) {
        const int c = e % c1, p = e / c1, x = p % W2, y = (p / W2) % H2, z = p / (W2 * H2);
        gcoarse[e] = (__bf16)block_sum2<DIM>(gcat, H, W, C, z, y, x, c0 + c);
    }
}

// ---------------------------------------------------------------------------
// Head (C -> 1, FP32 on the vector units), input packing, loss, Adam
// ---------------------------------------------------------------------------

// h[p] = bh + sum_t sum_c X[p + o_t][c] Wh[t][c]  (C a multiple of 8: 16-byte loads)
template <int DIM>
__global__ void k_head_fwd(const __bf16* __restrict__ X, int D, int H, int W, int C, const float* __restrict__ Wh,
                           const float* __restrict__ bh, float* __restrict__ h) {
    using TP = Taps<DIM>;
    const int P = D * H * W;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        const int x = p % W, y = (p / W) % H, z = p / (W * H);
        float s = bh[0];
        for (int t = 0; t < TP::T; ++t) {
            const int zz = z + TP::dz(t), yy = y + TP::dy(t), xx = x + TP::dx(t);
            if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
            const bf16x8* xp = (const bf16x8*)(X + (((size_t)zz * H + yy) * W + xx) * C);
            const float* wp = Wh + t * C;
            for (int q = 0; q < C / 8; ++q) {
                const bf16x8 v = xp[q];
#pragma unroll
                for (int j = 0; j < 8; ++j) s += (float)v[j] * wp[8 * q + j];
            }
        }
        h[p] = s;
    }
}

// gX[p][c] = sum_t dh[p - o_t] Wh[t][c]
template <int DIM>
__global__ void k_head_bwd_data(const float* __restrict__ dh, int D, int H, int W, int C,
                                const float* __restrict__ Wh, __bf16* __restrict__ gX) {
    using TP = Taps<DIM>;
    const int total = D * H * W * C;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int c = e % C, p = e / C, x = p % W, y = (p / W) % H, z = p / (W * H);
        float s = 0.0f;
        for (int t = 0; t < TP::T; ++t) {
            const int zz = z - TP::dz(t), yy = y - TP::dy(t), xx = x - TP::dx(t);
            if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
            s += dh[((size_t)zz * H + yy) * W + xx] * Wh[t * C + c];
        }
        gX[e] = (__bf16)s;
    }
}

// partials of dWh[t][c] = sum_p X[p + o_t][c] dh[p] and dbh = sum_p dh[p]
// (C a multiple of 8, at most 256).  blockIdx.y selects a group of nine taps
// (one group in 2D, three in 3D).  Thread (rho, g) accumulates channels
// [8g, 8g + 8) of the group's taps over pixels r0 + rho, r0 + rho + R, ...
// with 16-byte loads; the R row phases are then summed tap by tap in a fixed
// order through LDS.  part[block][t C + c], part[block][T C] = bias (group 0).
template <int DIM>
__global__ __launch_bounds__(256) void k_head_wgrad_part(const __bf16* __restrict__ X, int D, int H, int W, int C,
                                                         const float* __restrict__ dh, int rows_per_block,
                                                         float* __restrict__ part) {
    using TP = Taps<DIM>;
    __shared__ float red[2048];
    __shared__ float redb[256];
    const int P = D * H * W, r0 = blockIdx.x * rows_per_block, r1 = min(P, r0 + rows_per_block);
    const int n = TP::T * C + 1;
    const int tg = 9 * blockIdx.y;
    const int G = C / 8, R = 256 / G;
    const int g = threadIdx.x % G, rho = threadIdx.x / G;
    float acc[9][8];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[t][j] = 0.0f;
    float db = 0.0f;
    if (rho < R) {
        for (int p = r0 + rho; p < r1; p += R) {
            const float w = dh[p];
            if (g == 0) db += w;
            const int x = p % W, y = (p / W) % H, z = p / (W * H);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int zz = z + TP::dz(tg + t), yy = y + TP::dy(tg + t), xx = x + TP::dx(tg + t);
                if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                const bf16x8 v = *(const bf16x8*)(X + (((size_t)zz * H + yy) * W + xx) * C + 8 * g);
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[t][j] += (float)v[j] * w;
            }
        }
    }
    redb[threadIdx.x] = (rho < R && g == 0) ? db : 0.0f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        if (rho < R) {
#pragma unroll
            for (int j = 0; j < 8; ++j) red[rho * C + 8 * g + j] = acc[t][j];
        }
        __syncthreads();
        for (int c = threadIdx.x; c < C; c += blockDim.x) {
            float sum = 0.0f;
            for (int q = 0; q < R; ++q) sum += red[q * C + c];
            part[(size_t)blockIdx.x * n + (tg + t) * C + c] = sum;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && blockIdx.y == 0) {
        float sum = 0.0f;
        for (int q = 0; q < R; ++q) sum += redb[q * G];
        part[(size_t)blockIdx.x * n + TP::T * C] = sum;
    }
}

// unknown cells of the PPE (inner and Neumann ids)
__device__ __forceinline__ bool unk_of(int r, const BcDev& bc) {
    if (r == MCD_ROLE_INNER) return true;
    if (r <= 0) return false;
    return bc.type[r & (MCD_MAX_IDS - 1)] == MCD_BC_NEUMANN;
}

// partials over unknown cells of r^2, p^2 and the cell count
__global__ __launch_bounds__(256) void k_sumsq_part(const double* __restrict__ r, const double* __restrict__ p,
                                                    const int8_t* __restrict__ role, BcDev bc, int P,
                                                    double* __restrict__ part) {
    __shared__ double lds[3][4];
    double sr = 0.0, sp = 0.0, n = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < P; c += gridDim.x * blockDim.x)
        if (unk_of(role[c], bc)) {
            sr += r[c] * r[c];
            sp += p[c] * p[c];
            n += 1.0;
        }
    double v[3] = {sr, sp, n};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = v[0];
        part[3 * blockIdx.x + 1] = v[1];
        part[3 * blockIdx.x + 2] = v[2];
    }
}

// rms[0] = rms(r), rms[1] = rms(p) over unknown cells (1 where 0), one block
__global__ void k_rms(const double* __restrict__ part, int nblk, double* rms) {
    __shared__ double lds[3][4];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        v[0] += part[3 * b];
        v[1] += part[3 * b + 1];
        v[2] += part[3 * b + 2];
    }
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        const double rr = v[2] > 0 ? sqrt(v[0] / v[2]) : 1.0;
        const double rp = v[2] > 0 ? sqrt(v[1] / v[2]) : 1.0;
        rms[0] = rr > 0 ? rr : 1.0;
        rms[1] = rp > 0 ? rp : 1.0;
    }
}

__global__ void k_pack(const double* __restrict__ r, const double* __restrict__ pprev,
                       const int8_t* __restrict__ role, BcDev bc, int body_id, int wall_id, int P,
                       const double* __restrict__ rms, __bf16* __restrict__ x0) {
    const double inv_r = 1.0 / rms[0], inv_p = 1.0 / rms[1];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < P; c += gridDim.x * blockDim.x) {
        const int ro = role[c];
        const bool u = unk_of(ro, bc);
        float v[kIn];
#pragma unroll
        for (int q = 0; q < kIn; ++q) v[q] = 0.0f;
        v[0] = u ? (float)(r[c] * inv_r) : 0.0f;
        v[1] = u ? (float)(pprev[c] * inv_p) : 0.0f;
        v[2] = ro == MCD_ROLE_INNER ? 1.0f : 0.0f;
        v[3] = ro == body_id ? 1.0f : 0.0f;
        v[4] = ro == wall_id ? 1.0f : 0.0f;
#pragma unroll
        for (int q = 0; q < kIn; ++q) x0[(size_t)c * kIn + q] = (__bf16)v[q];
    }
}

// partials of num = sum_u (h - t)^2 and den = sum_u t^2, t = (P - Pprev) / (s rms(r))
__global__ __launch_bounds__(256) void k_loss_part(const float* __restrict__ h, const double* __restrict__ Pt,
                                                   const double* __restrict__ pprev, const int8_t* __restrict__ role,
                                                   BcDev bc, int P, const double* __restrict__ rms, double scale,
                                                   double* __restrict__ part) {
    __shared__ double lds[2][4];
    const double inv = 1.0 / (scale * rms[0]);
    double num = 0.0, den = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < P; c += gridDim.x * blockDim.x)
        if (unk_of(role[c], bc)) {
            const double t = (Pt[c] - pprev[c]) * inv;
            const double d = (double)h[c] - t;
            num += d * d;
            den += t * t;
        }
    double v[2] = {num, den};
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
    }
}

// loss = num / den (one block); den = 1 where it is 0
__global__ void k_loss_finish(const double* __restrict__ part, int nblk, double* loss) {
    __shared__ double lds[2][4];
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        v[0] += part[2 * b];
        v[1] += part[2 * b + 1];
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        loss[1] = v[1] > 0 ? v[1] : 1.0;
        loss[0] = v[0] / loss[1];
    }
}

// dh = 2 (h - t) / den at unknown cells, 0 elsewhere
__global__ void k_loss_grad(const float* __restrict__ h, const double* __restrict__ Pt,
                            const double* __restrict__ pprev, const int8_t* __restrict__ role, BcDev bc, int P,
                            const double* __restrict__ rms, double scale, const double* __restrict__ loss,
                            float* __restrict__ dh) {
    const double inv = 1.0 / (scale * rms[0]), den = loss[1];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < P; c += gridDim.x * blockDim.x) {
        float g = 0.0f;
        if (unk_of(role[c], bc)) g = (float)(2.0 * ((double)h[c] - (Pt[c] - pprev[c]) * inv) / den);
        dh[c] = g;
    }
}

// guess = pprev + s rms(r) h at unknown cells (FP64); other cells untouched
__global__ void k_unpack(const float* __restrict__ h, const double* __restrict__ pprev,
                         const int8_t* __restrict__ role, BcDev bc, int P, const double* __restrict__ rms,
                         double scale, double* __restrict__ out) {
    const double f = scale * rms[0];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < P; c += gridDim.x * blockDim.x)
        if (unk_of(role[c], bc)) out[c] = pprev[c] + f * (double)h[c];
}

// Adam (Kingma & Ba) on FP32 master weights with bias correction.
__global__ void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, size_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] = th[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// theta W[t][ci][co] -> forward Wf[t][n = co (padded)][k = ci] and data-gradient
// Wb[t][n = ci (padded)][k = co] = W[T - 1 - t][ci][co] (the tap of the opposite offset)
__global__ void k_weights_bf16(const float* __restrict__ W, int T, int cin, int cout, int npf, int npb,
                               __bf16* __restrict__ Wf, __bf16* __restrict__ Wb) {
    const int nf = T * npf * cin, nb = T * npb * cout;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += gridDim.x * blockDim.x) {
        const int t = e / (npf * cin), n = (e / cin) % npf, k = e % cin;
        Wf[e] = (__bf16)(n < cout ? W[(t * cin + k) * cout + n] : 0.0f);
    }
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nb; e += gridDim.x * blockDim.x) {
        const int t = e / (npb * cout), n = (e / cout) % npb, k = e % cout;
        Wb[e] = (__bf16)(n < cin ? W[((T - 1 - t) * cin + n) * cout + k] : 0.0f);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct ConvLayer {
    int cin, cout;       // cin includes both concat inputs
    size_t w_off, b_off; // offsets in the flat parameter vector
    int npf, npb;        // padded column counts of the forward / data-gradient GEMMs
    __bf16 *Wf, *Wb;
};

struct UNet {
    int L;
    int ch[kMaxLevels];
    int dim, T;          // 2 or 3; taps per convolution (9 or 27)
    int D, H, W;         // level-0 image (D = 1 in 2D)
    int body_id, wall_id;
    size_t nparams;
    float *theta, *grad, *m, *v;
    int nlayers;
    ConvLayer layers[4 * kMaxLevels + 1];
    // activations (bf16) and gradients
    __bf16* x0;
    __bf16 *in[kMaxLevels], *ea[kMaxLevels], *eb[kMaxLevels], *da[kMaxLevels], *db[kMaxLevels];
    __bf16 *g_eb[kMaxLevels], *g_ea[kMaxLevels], *g_da[kMaxLevels], *g_db[kMaxLevels], *g_in[kMaxLevels];
    __bf16* g_cat;       // largest concat gradient
    float *h, *dh;
    float* part;         // weight-gradient partials
    size_t part_cap;     // floats
    double* red;         // reduction scratch
    double* rms;         // [2]: rms(r), rms(p_prev)
    double out_scale;    // s of the guess p_prev + s rms(r) h
    double* loss;        // [2]
    double* loss_host;   // pinned [2]
    long long step;
};

static inline int grid_of(size_t n, int block = 256) {
    size_t g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

static hipError_t launch_conv(const ConvIn& in, const __bf16* Wk, int np, const float* bias, int cout, int relu,
                              __bf16* Y, hipStream_t st) {
    if (np % 32) return hipErrorInvalidValue;
    const int gx = (in.W + kCC - 1) / kCC, gy = (in.H + kCR - 1) / kCR;
    if (in.zs) {
        // planes per block: the most (up to 8) that still leave at least 1024 blocks
        int zb = 8;
        while (zb > 1 && (long long)gx * gy * ((in.D + zb - 1) / zb) * (np / 32) < 1024) zb >>= 1;
        const dim3 g(gx, gy * ((in.D + zb - 1) / zb), np / 32), b(256);
        hipLaunchKernelGGL(k_conv3_march, g, b, 0, st, in, Wk, np, bias, cout, relu, zb, Y);
    } else {
        const dim3 g(gx, gy * in.D, np / 32), b(256);
        hipLaunchKernelGGL(k_conv_mfma<2>, g, b, 0, st, in, Wk, np, bias, cout, relu, Y);
    }
    return hipGetLastError();
}

// weight and bias gradient of one conv layer into u.grad
static hipError_t layer_grads(UNet& u, const ConvLayer& Lr, const ConvIn& in, const __bf16* dY, hipStream_t st) {
    const int P = in.D * in.H * in.W;
    const int K = in.c0 + in.c1;
    const int kt = (K + 31) / 32, nt = (Lr.cout + 31) / 32;
    const size_t tile_floats = (size_t)u.T * kt * 32 * nt * 32;
    int nchunks = (int)(u.part_cap / tile_floats);
    if (nchunks > 256) nchunks = 256;
    if (nchunks < 1) return hipErrorInvalidValue;
    int chunk = (P + nchunks - 1) / nchunks;
    chunk = (chunk + 15) / 16 * 16;
    nchunks = (P + chunk - 1) / chunk;
    const int tiles = u.T * kt * nt;
    if (u.dim == 3)
        hipLaunchKernelGGL(k_conv_wgrad<3>, dim3(nchunks, (tiles + 3) / 4), dim3(256), 0, st, in, dY, Lr.cout, kt, nt,
                           chunk, u.part);
    else
        hipLaunchKernelGGL(k_conv_wgrad<2>, dim3(nchunks, (tiles + 3) / 4), dim3(256), 0, st, in, dY, Lr.cout, kt, nt,
                           chunk, u.part);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid_of((size_t)u.T * K * Lr.cout)), dim3(256), 0, st, u.part, nchunks,
                       u.T, K, Lr.cout, kt * 32, nt * 32, u.grad + Lr.w_off);
    const int rows = (P + 255) / 256;
    const int nb = (P + rows - 1) / rows;
    hipLaunchKernelGGL(k_colsum_part, dim3(nb), dim3(256), 0, st, dY, P, Lr.cout, rows, u.part);
    hipLaunchKernelGGL(k_colsum_reduce, dim3(1), dim3(256), 0, st, u.part, nb, Lr.cout, u.grad + Lr.b_off);
    return hipGetLastError();
}

// image extent of level l (D = 1 in 2D)
struct Lvl {
    int D, H, W;
    size_t P() const { return (size_t)D * H * W; }
};
static Lvl level(const UNet& u, int l) {
    return Lvl{u.dim == 3 ? u.D >> l : 1, u.H >> l, u.W >> l};
}

static ConvIn conv_in(const UNet& u, const __bf16* x0, int c0, const __bf16* x1, int c1, const Lvl& v) {
    return ConvIn{x0, c0, x1, c1, v.D, v.H, v.W, u.dim == 3 ? 1 : 0};
}

hipError_t unet_weights_to_bf16(UNet& u, hipStream_t st) {
    for (int i = 0; i < u.nlayers - 1; ++i) {
        const ConvLayer& Lr = u.layers[i];
        hipLaunchKernelGGL(k_weights_bf16, dim3(grid_of((size_t)u.T * 256 * 256)), dim3(256), 0, st,
                           u.theta + Lr.w_off, u.T, Lr.cin, Lr.cout, Lr.npf, Lr.npb, Lr.Wf, Lr.Wb);
    }
    return hipGetLastError();
}

// launch helpers of the dimension-templated element kernels
#define UNET_LAUNCH(u, kern, grid, ...)                                                        \
    do {                                                                                       \
        if ((u).dim == 3)                                                                      \
            hipLaunchKernelGGL(kern<3>, grid, dim3(256), 0, st, __VA_ARGS__);                  \
        else                                                                                   \
            hipLaunchKernelGGL(kern<2>, grid, dim3(256), 0, st, __VA_ARGS__);                  \
    } while (0)

// Forward pass; leaves the head output h (FP32) and all activations.
hipError_t unet_forward(UNet& u, const double* b, const double* pprev, const int8_t* role, const BcDev& bc,
                        hipStream_t st) {
    const int P = (int)level(u, 0).P();
    const int nb = 256;
    hipLaunchKernelGGL(k_sumsq_part, dim3(nb), dim3(256), 0, st, b, pprev, role, bc, P, u.red);
    hipLaunchKernelGGL(k_rms, dim3(1), dim3(256), 0, st, u.red, nb, u.rms);
    hipLaunchKernelGGL(k_pack, dim3(grid_of(P)), dim3(256), 0, st, b, pprev, role, bc, u.body_id, u.wall_id, P,
                       u.rms, u.x0);
    int li = 0;
    for (int l = 0; l < u.L; ++l) {
        const Lvl v = level(u, l);
        const __bf16* src = u.x0;
        int csrc = kIn;
        if (l > 0) {
            const Lvl f = level(u, l - 1);
            UNET_LAUNCH(u, k_pool, dim3(grid_of(v.P() * u.ch[l - 1])), u.eb[l - 1], f.D, f.H, f.W, u.ch[l - 1],
                        u.in[l]);
            src = u.in[l];
            csrc = u.ch[l - 1];
        }
        const ConvLayer& A = u.layers[li++];
        hipError_t e = launch_conv(conv_in(u, src, csrc, nullptr, 0, v), A.Wf, A.npf, u.theta + A.b_off, A.cout, 1,
                                   u.ea[l], st);
        if (e != hipSuccess) return e;
        const ConvLayer& B = u.layers[li++];
        e = launch_conv(conv_in(u, u.ea[l], u.ch[l], nullptr, 0, v), B.Wf, B.npf, u.theta + B.b_off, B.cout, 1,
                        u.eb[l], st);
        if (e != hipSuccess) return e;
    }
    for (int l = u.L - 2; l >= 0; --l) {
        const Lvl v = level(u, l);
        const __bf16* coarse = (l + 1 == u.L - 1) ? u.eb[l + 1] : u.db[l + 1];
        const ConvLayer& A = u.layers[li++];
        hipError_t e = launch_conv(conv_in(u, u.eb[l], u.ch[l], coarse, u.ch[l + 1], v), A.Wf, A.npf,
                                   u.theta + A.b_off, A.cout, 1, u.da[l], st);
        if (e != hipSuccess) return e;
        const ConvLayer& B = u.layers[li++];
        e = launch_conv(conv_in(u, u.da[l], u.ch[l], nullptr, 0, v), B.Wf, B.npf, u.theta + B.b_off, B.cout, 1,
                        u.db[l], st);
        if (e != hipSuccess) return e;
    }
    const ConvLayer& Hd = u.layers[li];
    const __bf16* last = u.L > 1 ? u.db[0] : u.eb[0];
    UNET_LAUNCH(u, k_head_fwd, dim3(grid_of(P)), last, u.D, u.H, u.W, u.ch[0], u.theta + Hd.w_off,
                u.theta + Hd.b_off, u.h);
    return hipGetLastError();
}

static hipError_t bwd_data(const UNet& u, const ConvLayer& Lr, const __bf16* dY, const Lvl& v, __bf16* dX,
                           hipStream_t st) {
    // data gradient = forward convolution of dY with the flipped, transposed weights
    return launch_conv(conv_in(u, dY, Lr.cout, nullptr, 0, v), Lr.Wb, Lr.npb, nullptr, Lr.cin, 0, dX, st);
}

// Forward, loss against the target pressure, backward, Adam step.
hipError_t unet_train_step(UNet& u, const double* b, const double* pprev, const double* Pt, const int8_t* role,
                           const BcDev& bc, float lr, hipStream_t st, double* loss_out) {
    hipError_t e = unet_forward(u, b, pprev, role, bc, st);
    if (e != hipSuccess) return e;
    const int P = (int)level(u, 0).P();
    const int nb = 256;
    hipLaunchKernelGGL(k_loss_part, dim3(nb), dim3(256), 0, st, u.h, Pt, pprev, role, bc, P, u.rms, u.out_scale,
                       u.red);
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, st, u.red, nb, u.loss);
    hipLaunchKernelGGL(k_loss_grad, dim3(grid_of(P)), dim3(256), 0, st, u.h, Pt, pprev, role, bc, P, u.rms,
                       u.out_scale, u.loss, u.dh);
    // head
    const int nl = u.nlayers;
    const ConvLayer& Hd = u.layers[nl - 1];
    const int C0 = u.ch[0];
    const __bf16* last = u.L > 1 ? u.db[0] : u.eb[0];
    __bf16* g_last = u.L > 1 ? u.g_db[0] : u.g_eb[0];
    UNET_LAUNCH(u, k_head_bwd_data, dim3(grid_of((size_t)P * C0)), u.dh, u.D, u.H, u.W, C0, u.theta + Hd.w_off,
                g_last);
    {
        const int rows = (P + 255) / 256, nblk = (P + rows - 1) / rows;
        UNET_LAUNCH(u, k_head_wgrad_part, dim3(nblk, u.T / 9), last, u.D, u.H, u.W, C0, u.dh, rows, u.part);
        hipLaunchKernelGGL(k_colsum_reduce, dim3(1), dim3(256), 0, st, u.part, nblk, u.T * C0 + 1,
                           u.grad + Hd.w_off);
    }
    // decoder, unwound from level 0 upwards (layer index of dec(l)a: 2L + 2(L-2-l))
    for (int l = 0; l <= u.L - 2; ++l) {
        const Lvl v = level(u, l);
        const size_t n = v.P() * u.ch[l];
        const ConvLayer& A = u.layers[2 * u.L + 2 * (u.L - 2 - l)];
        const ConvLayer& B = u.layers[2 * u.L + 2 * (u.L - 2 - l) + 1];
        hipLaunchKernelGGL(k_relu_mask, dim3(grid_of(n)), dim3(256), 0, st, u.g_db[l], u.db[l], n);
        if ((e = layer_grads(u, B, conv_in(u, u.da[l], u.ch[l], nullptr, 0, v), u.g_db[l], st)) != hipSuccess)
            return e;
        if ((e = bwd_data(u, B, u.g_db[l], v, u.g_da[l], st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_relu_mask, dim3(grid_of(n)), dim3(256), 0, st, u.g_da[l], u.da[l], n);
        const __bf16* coarse = (l + 1 == u.L - 1) ? u.eb[l + 1] : u.db[l + 1];
        if ((e = layer_grads(u, A, conv_in(u, u.eb[l], u.ch[l], coarse, u.ch[l + 1], v), u.g_da[l], st)) !=
            hipSuccess)
            return e;
        if ((e = bwd_data(u, A, u.g_da[l], v, u.g_cat, st)) != hipSuccess) return e;
        __bf16* gcoarse = (l + 1 == u.L - 1) ? u.g_eb[l + 1] : u.g_db[l + 1];
        UNET_LAUNCH(u, k_cat_split, dim3(grid_of(v.P() * u.ch[l])), u.g_cat, v.D, v.H, v.W, u.ch[l], u.ch[l + 1],
                    u.g_eb[l], gcoarse);
    }
    // encoder, from the bottom
    for (int l = u.L - 1; l >= 0; --l) {
        const Lvl v = level(u, l);
        const size_t n = v.P() * u.ch[l];
        const ConvLayer& A = u.layers[2 * l];
        const ConvLayer& B = u.layers[2 * l + 1];
        hipLaunchKernelGGL(k_relu_mask, dim3(grid_of(n)), dim3(256), 0, st, u.g_eb[l], u.eb[l], n);
        if ((e = layer_grads(u, B, conv_in(u, u.ea[l], u.ch[l], nullptr, 0, v), u.g_eb[l], st)) != hipSuccess)
            return e;
        if ((e = bwd_data(u, B, u.g_eb[l], v, u.g_ea[l], st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_relu_mask, dim3(grid_of(n)), dim3(256), 0, st, u.g_ea[l], u.ea[l], n);
        const __bf16* src = l > 0 ? u.in[l] : u.x0;
        const int csrc = l > 0 ? u.ch[l - 1] : kIn;
        if ((e = layer_grads(u, A, conv_in(u, src, csrc, nullptr, 0, v), u.g_ea[l], st)) != hipSuccess) return e;
        if (l > 0) {
            if ((e = bwd_data(u, A, u.g_ea[l], v, u.g_in[l], st)) != hipSuccess) return e;
            const Lvl f = level(u, l - 1);
            UNET_LAUNCH(u, k_pool_bwd_add, dim3(grid_of(f.P() * u.ch[l - 1])), u.g_in[l], f.D, f.H, f.W,
                        u.ch[l - 1], u.g_eb[l - 1]);
        }
    }
    u.step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)u.step), c2 = 1.0f - powf(b2, (float)u.step);
    if (lr > 0.0f) {
        hipLaunchKernelGGL(k_adam, dim3(grid_of(u.nparams)), dim3(256), 0, st, u.theta, u.m, u.v, u.grad, u.nparams,
                           lr, b1, b2, 1e-8f, c1, c2);
        if ((e = unet_weights_to_bf16(u, st)) != hipSuccess) return e;
    }
    if (loss_out) {
        if ((e = hipMemcpyAsync(u.loss_host, u.loss, 2 * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        *loss_out = u.loss_host[0];
    }
    return hipGetLastError();
}

hipError_t unet_infer(UNet& u, const double* b, const double* pprev, const int8_t* role, const BcDev& bc,
                      double* out, hipStream_t st) {
    hipError_t e = unet_forward(u, b, pprev, role, bc, st);
    if (e != hipSuccess) return e;
    const int P = (int)level(u, 0).P();
    hipLaunchKernelGGL(k_unpack, dim3(grid_of(P)), dim3(256), 0, st, u.h, pprev, role, bc, P, u.rms, u.out_scale,
                       out);
    return hipGetLastError();
}

static hipError_t dalloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes < 16 ? 16 : bytes);
    if (e == hipSuccess) e = hipMemset(*p, 0, bytes < 16 ? 16 : bytes);
    return e;
}

void unet_free(UNet* u) {
    if (!u) return;
    void* ptrs[] = {u->theta, u->grad, u->m, u->v, u->x0, u->g_cat, u->h, u->dh, u->part, u->red, u->rms, u->loss};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (u->loss_host) (void)hipHostFree(u->loss_host);
    for (int l = 0; l < kMaxLevels; ++l) {
        void* q[] = {u->in[l], u->ea[l], u->eb[l], u->da[l], u->db[l], u->g_eb[l], u->g_ea[l], u->g_da[l],
                     u->g_db[l], u->g_in[l]};
        for (void* p : q)
            if (p) (void)hipFree(p);
    }
    for (int i = 0; i < u->nlayers; ++i) {
        if (u->layers[i].Wf) (void)hipFree(u->layers[i].Wf);
        if (u->layers[i].Wb) (void)hipFree(u->layers[i].Wb);
    }
    delete u;
}

// Layer table in the flat parameter order: enc0a, enc0b, ..., dec(L-2)a,
// dec(L-2)b, ..., dec0a, dec0b, head; each W[T][cin][cout] then b[cout].
hipError_t unet_create(int dim, int D, int H, int W, int L, const int* ch, int body_id, int wall_id, UNet** out) {
    UNet* u = new UNet{};
    *out = u;
    u->L = L;
    u->dim = dim;
    u->T = dim == 3 ? 27 : 9;
    u->D = dim == 3 ? D : 1;
    u->H = H;
    u->W = W;
    u->body_id = body_id;
    u->wall_id = wall_id;
    u->out_scale = 1.0;
    for (int l = 0; l < L; ++l) u->ch[l] = ch[l];
    size_t off = 0;
    int n = 0;
    auto add = [&](int cin, int cout) {
        ConvLayer& Lr = u->layers[n++];
        Lr.cin = cin;
        Lr.cout = cout;
        Lr.w_off = off;
        off += (size_t)u->T * cin * cout;
        Lr.b_off = off;
        off += cout;
        Lr.npf = (cout + 31) / 32 * 32;
        Lr.npb = (cin + 31) / 32 * 32;
    };
    int prev = kIn;
    for (int l = 0; l < L; ++l) {
        add(prev, ch[l]);
        add(ch[l], ch[l]);
        prev = ch[l];
    }
    for (int l = L - 2; l >= 0; --l) {
        add(ch[l] + ch[l + 1], ch[l]);
        add(ch[l], ch[l]);
    }
    add(ch[0], 1);
    u->nlayers = n;
    u->nparams = off;
    hipError_t e;
    const size_t np = off;
    if ((e = dalloc((void**)&u->theta, np * 4)) != hipSuccess) return e;
    if ((e = dalloc((void**)&u->grad, np * 4)) != hipSuccess) return e;
    if ((e = dalloc((void**)&u->m, np * 4)) != hipSuccess) return e;
    if ((e = dalloc((void**)&u->v, np * 4)) != hipSuccess) return e;
    for (int i = 0; i < n - 1; ++i) {
        ConvLayer& Lr = u->layers[i];
        if ((e = dalloc((void**)&Lr.Wf, (size_t)u->T * Lr.npf * Lr.cin * 2)) != hipSuccess) return e;
        if ((e = dalloc((void**)&Lr.Wb, (size_t)u->T * Lr.npb * Lr.cout * 2)) != hipSuccess) return e;
    }
    const size_t P = level(*u, 0).P();
    if ((e = dalloc((void**)&u->x0, P * kIn * 2)) != hipSuccess) return e;
    size_t catmax = 0, partmax = 0;
    for (int l = 0; l < L; ++l) {
        const size_t Pl = level(*u, l).P();
        const size_t c = ch[l];
        if (l > 0 && (e = dalloc((void**)&u->in[l], Pl * ch[l - 1] * 2)) != hipSuccess) return e;
        if (l > 0 && (e = dalloc((void**)&u->g_in[l], Pl * ch[l - 1] * 2)) != hipSuccess) return e;
        if ((e = dalloc((void**)&u->ea[l], Pl * c * 2)) != hipSuccess) return e;
        if ((e = dalloc((void**)&u->eb[l], Pl * c * 2)) != hipSuccess) return e;
        if ((e = dalloc((void**)&u->g_ea[l], Pl * c * 2)) != hipSuccess) return e;
        if ((e = dalloc((void**)&u->g_eb[l], Pl * c * 2)) != hipSuccess) return e;
        if (l <= L - 2) {
            if ((e = dalloc((void**)&u->da[l], Pl * c * 2)) != hipSuccess) return e;
            if ((e = dalloc((void**)&u->db[l], Pl * c * 2)) != hipSuccess) return e;
            if ((e = dalloc((void**)&u->g_da[l], Pl * c * 2)) != hipSuccess) return e;
            if ((e = dalloc((void**)&u->g_db[l], Pl * c * 2)) != hipSuccess) return e;
            catmax = catmax > Pl * (c + ch[l + 1]) ? catmax : Pl * (c + ch[l + 1]);
        }
    }
    for (int i = 0; i < n; ++i) {
        const size_t kt = (u->layers[i].cin + 31) / 32, nt = (u->layers[i].cout + 31) / 32;
        const size_t t = (size_t)u->T * kt * 32 * nt * 32;
        partmax = partmax > t ? partmax : t;
    }
    const size_t head_part = (size_t)256 * (u->T * 256 + 1);
    u->part_cap = partmax * 64 > head_part ? partmax * 64 : head_part;
    if ((e = dalloc((void**)&u->g_cat, (catmax ? catmax : 16) * 2)) != hipSuccess) return e;
    if ((e = dalloc((void**)&u->h, P * 4)) != hipSuccess) return e;
    if ((e = dalloc((void**)&u->dh, P * 4)) != hipSuccess) return e;
    if ((e = dalloc((void**)&u->part, u->part_cap * 4)) != hipSuccess) return e;
    if ((e = dalloc((void**)&u->red, 1024 * sizeof(double))) != hipSuccess) return e;
    if ((e = dalloc((void**)&u->rms, 2 * sizeof(double))) != hipSuccess) return e;
    if ((e = dalloc((void**)&u->loss, 2 * sizeof(double))) != hipSuccess) return e;
    if ((e = hipHostMalloc((void**)&u->loss_host, 2 * sizeof(double), hipHostMallocDefault)) != hipSuccess) return e;
    return hipDeviceSynchronize();
}

size_t unet_nparams(const UNet& u) { return u.nparams; }
float* unet_theta(UNet& u) { return u.theta; }
float* unet_grad(UNet& u) { return u.grad; }
float* unet_head_out(UNet& u) { return u.h; }
void unet_set_output_scale(UNet& u, double s) { u.out_scale = s; }
void unet_reset_optimizer(UNet& u, hipStream_t st) {
    (void)hipMemsetAsync(u.m, 0, u.nparams * 4, st);
    (void)hipMemsetAsync(u.v, 0, u.nparams * 4, st);
    u.step = 0;
}

}  // namespace mcd
