// zsur_kernels.hip -- gfx950 kernels of the design surrogate: a BF16 MFMA
// GEMM with FP32 accumulation (the convolutions' forward, data-gradient and
// weight-gradient contractions), im2col/col2im for 3x3 dilated convolutions
// with periodic phi and zero r padding, and the element-wise pieces of
// training (activation gradient, MSE, Adam).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include <string>

#include "../../include/zsur.h"

namespace {

thread_local std::string g_err;

zsur_status fail(zsur_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

zsur_status launched(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ZSUR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return ZSUR_OK;
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// FP32 -> bf16, round to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float act_apply(float v, int act, float slope)
{
    return (act == ZSUR_ACT_LEAKY && v < 0.f) ? slope * v : v;
}

// Block tile 64 (m) x 64 (n), K in steps of 32; four wavefronts, each
// owning a 32 x 32 quarter as 2 x 2 MFMA tiles of 16 x 16.  Both operand
// tiles are staged in LDS with k contiguous ([row][k], rows padded to 40
// bf16 = 80 B so that each lane's eight k values are one 16 B read).  The
// 16x16x32 MFMA takes, in lane l, row l % 16 of A and column l % 16 of B with
// eight k values each; A and B are loaded with the same k order, so the
// contraction does not depend on which k the hardware pairs them with.  The
// result lane l, register r is C[4 (l / 16) + r][l % 16] of the 16 x 16 tile.
constexpr int TM = 64, TN = 64, TK = 32, LDK = TK + 8;

// operand tile loads: mode 1 and 2 read eight consecutive elements along the
// operand's unit-stride index with one 16 B load (mode 1: along k, mode 2:
// along the tile's row index m or n), mode 0 one element at a time
__device__ __forceinline__ void tile_load(uint16_t (*S)[LDK], const uint16_t *__restrict__ P, long s_row, long s_k,
                                          int mode, int r0, int R, int k0, int kend, int tid)
{
    if (mode == 1) {                  // k contiguous: row tid/4, eight k from (tid%4)*8
        const int rr = tid >> 2, kk = (tid & 3) * 8;
        const int gr = r0 + rr, gk = k0 + kk;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gr < R) {
            if (gk + 7 < kend) {
                v = *reinterpret_cast<const uint4 *>(P + (long)gr * s_row + gk);
            } else {
                uint16_t t[8];
                for (int e = 0; e < 8; ++e) t[e] = (gk + e < kend) ? P[(long)gr * s_row + gk + e] : (uint16_t)0;
                __builtin_memcpy(&v, t, sizeof v);
            }
        }
        *reinterpret_cast<uint4 *>(&S[rr][kk]) = v;
    } else if (mode == 2) {           // row index contiguous: k tid/8, eight rows from (tid%8)*8
        const int kk = tid >> 3, rr = (tid & 7) * 8;
        const int gr = r0 + rr, gk = k0 + kk;
        uint16_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (gk < kend) {
            if (gr + 7 < R) {
                const uint4 v = *reinterpret_cast<const uint4 *>(P + gr + (long)gk * s_k);
                __builtin_memcpy(t, &v, sizeof t);
            } else {
                for (int e = 0; e < 8; ++e) t[e] = (gr + e < R) ? P[(long)(gr + e) + (long)gk * s_k] : (uint16_t)0;
            }
        }
        for (int e = 0; e < 8; ++e) S[rr + e][kk] = t[e];
    } else {
        for (int e = tid; e < 64 * TK; e += 256) {
            int rr, kk;
            if (s_k == 1) { rr = e / TK; kk = e % TK; }
            else { rr = e % 64; kk = e / 64; }
            const int gr = r0 + rr, gk = k0 + kk;
            S[rr][kk] = (gr < R && gk < kend) ? P[(long)gr * s_row + (long)gk * s_k] : (uint16_t)0;
        }
    }
}

// The vector modes in two halves, so that the next k-tile's global loads are
// in flight while the current tile's MFMAs run: fetch (global -> eight bf16
// in a register) and put (register -> LDS), the same elements and zero
// fill as tile_load.
__device__ __forceinline__ uint4 tile_fetch(const uint16_t *__restrict__ P, long s_row, long s_k, int mode, int r0,
                                            int R, int k0, int kend, int tid)
{
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (mode == 1) {
        const int gr = r0 + (tid >> 2), gk = k0 + (tid & 3) * 8;
        if (gr < R) {
            if (gk + 7 < kend) {
                v = *reinterpret_cast<const uint4 *>(P + (long)gr * s_row + gk);
            } else {
                uint16_t t[8];
                for (int e = 0; e < 8; ++e) t[e] = (gk + e < kend) ? P[(long)gr * s_row + gk + e] : (uint16_t)0;
                __builtin_memcpy(&v, t, sizeof v);
            }
        }
    } else {
        const int gk = k0 + (tid >> 3), gr = r0 + (tid & 7) * 8;
        if (gk < kend) {
            if (gr + 7 < R) {
                v = *reinterpret_cast<const uint4 *>(P + gr + (long)gk * s_k);
            } else {
                uint16_t t[8];
                for (int e = 0; e < 8; ++e) t[e] = (gr + e < R) ? P[(long)(gr + e) + (long)gk * s_k] : (uint16_t)0;
                __builtin_memcpy(&v, t, sizeof v);
            }
        }
    }
    return v;
}

__device__ __forceinline__ void tile_put(uint16_t (*S)[LDK], uint4 v, int mode, int tid)
{
    if (mode == 1) {
        *reinterpret_cast<uint4 *>(&S[tid >> 2][(tid & 3) * 8]) = v;
    } else {
        uint16_t t[8];
        __builtin_memcpy(t, &v, sizeof t);
        const int kk = tid >> 3, rr = (tid & 7) * 8;
        for (int e = 0; e < 8; ++e) S[rr + e][kk] = t[e];
    }
}

__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const uint16_t *__restrict__ A, long sam,
                                                   long sak, const uint16_t *__restrict__ B, long sbk, long sbn,
                                                   float *C, long ldc, uint16_t *Cb, const float *bias, int act,
                                                   float slope, int split, float *work, int amode, int bmode)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[TM][LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // the M tiles of one N column are consecutive blocks, so the B tile they
    // share is read from HBM once and from the L2 by the others
    const int gm = (M + TM - 1) / TM;
    const int m0 = (int)(blockIdx.x % (unsigned)gm) * TM, n0 = (int)(blockIdx.x / (unsigned)gm) * TN, z = blockIdx.z;
    const int kper = ((K + split - 1) / split + TK - 1) / TK * TK;
    const int kbeg = z * kper, kend = min(K, kbeg + kper);
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    floatx4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // both operands in a vector mode: the next k-tile is fetched into
    // registers before the current one's MFMAs (same values, same order)
    const bool pipe = amode != 0 && bmode != 0;
    uint4 ra = make_uint4(0u, 0u, 0u, 0u), rb = ra;
    if (pipe && kbeg < kend) {
        ra = tile_fetch(A, sam, sak, amode, m0, M, kbeg, kend, tid);
        rb = tile_fetch(B, sbn, sbk, bmode, n0, N, kbeg, kend, tid);
    }
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        if (pipe) {
            tile_put(As, ra, amode, tid);
            tile_put(Bs, rb, bmode, tid);
        } else {
            tile_load(As, A, sam, sak, amode, m0, M, k0, kend, tid);
            tile_load(Bs, B, sbn, sbk, bmode, n0, N, k0, kend, tid);
        }
        __syncthreads();
        if (pipe && k0 + TK < kend) {
            ra = tile_fetch(A, sam, sak, amode, m0, M, k0 + TK, kend, tid);
            rb = tile_fetch(B, sbn, sbk, bmode, n0, N, k0 + TK, kend, tid);
        }
        const int g8 = 8 * (lane >> 4), r16 = lane & 15;
        for (int i = 0; i < 2; ++i) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&As[wm + i * 16 + r16][g8]);
            for (int j = 0; j < 2; ++j) {
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Bs[wn + j * 16 + r16][g8]);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m >= M || n >= N) continue;
                float v = acc[i][j][r];
                if (split == 1) {
                    if (bias) v += bias[m];
                    v = act_apply(v, act, slope);
                    C[(long)m * ldc + n] = v;
                    if (Cb) Cb[(long)m * ldc + n] = f2bf(v);
                } else {
                    work[((long)z * M + m) * N + n] = v;
                }
            }
}

// sum of the split-K partial products in slice order, then bias and activation
__global__ void splitk_reduce(int M, int N, int split, const float *work, float *C, long ldc, uint16_t *Cb,
                              const float *bias, int act, float slope)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)M * N) return;
    const int m = (int)(q / N), n = (int)(q % N);
    float v = 0.f;
    for (int z = 0; z < split; ++z) v += work[(long)z * M * N + q];
    if (bias) v += bias[m];
    v = act_apply(v, act, slope);
    C[(long)m * ldc + n] = v;
    if (Cb) Cb[(long)m * ldc + n] = f2bf(v);
}

// grid: x over groups of four pixels, y over the C*9 rows of cols
__global__ void im2col_kernel(const float *x, int C, int B, int H, int W, int dil, uint16_t *cols)
{
    const int N = B * H * W;
    const int row = blockIdx.y;
    const int c = row / 9, t = row % 9, ky = t / 3, kx = t % 3;
    const int n0 = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
    if (n0 >= N) return;
    const float *xc = x + (size_t)c * N;
    uint16_t *out = cols + (size_t)row * N;
    int xw = n0 % W, y = (n0 / W) % H, b = n0 / (W * H);
    for (int e = 0; e < 4 && n0 + e < N; ++e) {
        const int ys = y + dil * (ky - 1);
        int xs = (xw + dil * (kx - 1)) % W;
        if (xs < 0) xs += W;
        const float v = (ys >= 0 && ys < H) ? xc[((size_t)b * H + ys) * W + xs] : 0.f;
        out[n0 + e] = f2bf(v);
        if (++xw == W) {
            xw = 0;
            if (++y == H) { y = 0; ++b; }
        }
    }
}

__global__ void col2im_kernel(const float *dcols, int C, int B, int H, int W, int dil, float *dx)
{
    const long N = (long)B * H * W;
    const long total = (long)C * N;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (long)gridDim.x * blockDim.x) {
        const long n = q % N;
        const int c = (int)(q / N);
        const int xw = (int)(n % W), y = (int)((n / W) % H), b = (int)(n / ((long)W * H));
        float s = 0.f;
        for (int ky = 0; ky < 3; ++ky) {
            const int yo = y - dil * (ky - 1);        // output row whose tap ky reads row y
            if (yo < 0 || yo >= H) continue;
            for (int kx = 0; kx < 3; ++kx) {
                int xo = (xw - dil * (kx - 1)) % W;
                if (xo < 0) xo += W;
                s += dcols[(long)(c * 9 + ky * 3 + kx) * N + ((long)b * H + yo) * W + xo];
            }
        }
        dx[q] = s;
    }
}

__global__ void act_grad_kernel(const float *y, const float *dy, float *dz, uint16_t *dzb, size_t n, float slope)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const float g = dy[q] * (y[q] > 0.f ? 1.f : slope);
        dz[q] = g;
        if (dzb) dzb[q] = f2bf(g);
    }
}

// fixed-order block reduction of 256 values
__device__ float block_sum(float v)
{
    __shared__ float s[256];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    const float r = s[0];
    __syncthreads();
    return r;
}

// two passes: block (m, p) sums slice p of row m, then one block per row
// adds the slices in order
constexpr int ROW_SLICES = 64;

__global__ void rowsum_pass1(const float *x, int N, float *partial)
{
    const long m = blockIdx.y;
    const int p = blockIdx.x;
    const int len = (N + ROW_SLICES - 1) / ROW_SLICES;
    const int lo = p * len, hi = min(N, lo + len);
    float v = 0.f;
    for (int n = lo + (int)threadIdx.x; n < hi; n += 256) v += x[m * N + n];
    v = block_sum(v);
    if (threadIdx.x == 0) partial[m * ROW_SLICES + p] = v;
}

__global__ void rowsum_pass2(const float *partial, float *out)
{
    const long m = blockIdx.x;
    float v = (int)threadIdx.x < ROW_SLICES ? partial[m * ROW_SLICES + threadIdx.x] : 0.f;
    v = block_sum(v);
    if (threadIdx.x == 0) out[m] = v;
}

__global__ void mse_pass1(const float *p, const float *t, size_t n, float *d, float *partial)
{
    float s = 0.f;
    const float inv = 1.f / (float)n;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
        const float e = p[q] - t[q];
        d[q] = 2.f * e * inv;
        s += e * e;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void mse_pass2(const float *partial, int nb, size_t n, float *loss)
{
    float s = 0.f;
    for (int q = threadIdx.x; q < nb; q += 256) s += partial[q];
    s = block_sum(s);
    if (threadIdx.x == 0) loss[0] = s / (float)n;
}

__global__ void to_bf16_kernel(const float *x, uint16_t *y, size_t n)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
        y[q] = f2bf(x[q]);
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2, uint16_t *pb)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const float gq = g[q];
        const float mq = b1 * m[q] + (1.f - b1) * gq;
        const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
        m[q] = mq;
        v[q] = vq;
        const float pq = p[q] - lr * (mq / bc1) / (sqrtf(vq / bc2) + eps);
        p[q] = pq;
        if (pb) pb[q] = f2bf(pq);
    }
}

unsigned grid_for(size_t n, unsigned cap = 65535u * 4u)
{
    size_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    return (unsigned)(g > cap ? cap : g);
}

}  // namespace

extern "C" {

zsur_status zsur_gemm(int M, int N, int K, const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk,
                      long sbn, float *C, long ldc, uint16_t *Cb, const float *bias, int act, float slope,
                      int split, float *work, void *stream)
{
    if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !C || split < 1 || (split > 1 && !work))
        return fail(ZSUR_ERR_ARG, "zsur_gemm: bad sizes or pointers (M %d N %d K %d split %d)", M, N, K, split);
    hipStream_t s = (hipStream_t)stream;
    // vector tile loads where the unit-stride index, the other stride and the
    // base allow 16 B-aligned chunks of eight
    auto mode = [](const uint16_t *P, long s_row, long s_k) {
        if (((uintptr_t)P & 15u) != 0) return 0;
        if (s_k == 1 && s_row % 8 == 0) return 1;
        if (s_row == 1 && s_k % 8 == 0) return 2;
        return 0;
    };
    const int amode = mode(A, sam, sak), bmode = mode(B, sbn, sbk);
    const long tiles = (long)((N + TN - 1) / TN) * ((M + TM - 1) / TM);
    if (tiles > 0x7fffffffL || split > 65535) return fail(ZSUR_ERR_ARG, "zsur_gemm: too many tiles");
    dim3 grid((unsigned)tiles, 1, split);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, Cb, bias, act,
                       slope, split, work, amode, bmode);
    if (split > 1)
        hipLaunchKernelGGL(splitk_reduce, dim3(grid_for((size_t)M * N, 1u << 30)), dim3(256), 0, s, M, N, split,
                           work, C, ldc, Cb, bias, act, slope);
    return launched("zsur_gemm");
}

zsur_status zsur_im2col(const float *x, int C, int B, int H, int W, int dil, uint16_t *cols, void *stream)
{
    if (C <= 0 || B <= 0 || H <= 0 || W <= 0 || dil < 1 || !x || !cols) return fail(ZSUR_ERR_ARG, "zsur_im2col");
    if ((long)B * H * W > 0x7fffffffL || C * 9 > 65535) return fail(ZSUR_ERR_ARG, "zsur_im2col: too large");
    const int N = B * H * W;
    dim3 grid((unsigned)((N + 1023) / 1024), (unsigned)(C * 9));
    hipLaunchKernelGGL(im2col_kernel, grid, dim3(256), 0, (hipStream_t)stream, x, C, B, H, W, dil, cols);
    return launched("zsur_im2col");
}

zsur_status zsur_col2im(const float *dcols, int C, int B, int H, int W, int dil, float *dx, void *stream)
{
    if (C <= 0 || B <= 0 || H <= 0 || W <= 0 || dil < 1 || !dcols || !dx) return fail(ZSUR_ERR_ARG, "zsur_col2im");
    hipLaunchKernelGGL(col2im_kernel, dim3(grid_for((size_t)C * B * H * W)), dim3(256), 0, (hipStream_t)stream,
                       dcols, C, B, H, W, dil, dx);
    return launched("zsur_col2im");
}

zsur_status zsur_act_grad(const float *y, const float *dy, float *dz, uint16_t *dzb, size_t n, float slope,
                          void *stream)
{
    if (!y || !dy || !dz || n == 0) return fail(ZSUR_ERR_ARG, "zsur_act_grad");
    hipLaunchKernelGGL(act_grad_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, y, dy, dz, dzb, n,
                       slope);
    return launched("zsur_act_grad");
}

zsur_status zsur_rowsum(const float *x, int M, int N, float *out, float *partial, void *stream)
{
    if (!x || !out || !partial || M <= 0 || N <= 0 || M > 65535) return fail(ZSUR_ERR_ARG, "zsur_rowsum");
    hipLaunchKernelGGL(rowsum_pass1, dim3(ROW_SLICES, M), dim3(256), 0, (hipStream_t)stream, x, N, partial);
    hipLaunchKernelGGL(rowsum_pass2, dim3(M), dim3(256), 0, (hipStream_t)stream, partial, out);
    return launched("zsur_rowsum");
}

zsur_status zsur_mse(const float *p, const float *t, size_t n, float *d, float *loss, float *partial, void *stream)
{
    if (!p || !t || !d || !loss || !partial || n == 0) return fail(ZSUR_ERR_ARG, "zsur_mse");
    const unsigned nb = grid_for(n, 1024u);
    hipLaunchKernelGGL(mse_pass1, dim3(nb), dim3(256), 0, (hipStream_t)stream, p, t, n, d, partial);
    hipLaunchKernelGGL(mse_pass2, dim3(1), dim3(256), 0, (hipStream_t)stream, partial, (int)nb, n, loss);
    return launched("zsur_mse");
}

zsur_status zsur_to_bf16(const float *x, uint16_t *y, size_t n, void *stream)
{
    if (!x || !y || n == 0) return fail(ZSUR_ERR_ARG, "zsur_to_bf16");
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, n);
    return launched("zsur_to_bf16");
}

zsur_status zsur_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                      float eps, int t, uint16_t *pb, void *stream)
{
    if (!p || !g || !m || !v || n == 0 || t < 1) return fail(ZSUR_ERR_ARG, "zsur_adam");
    const float bc1 = 1.f - powf(b1, (float)t), bc2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, p, g, m, v, n, lr, b1, b2,
                       eps, bc1, bc2, pb);
    return launched("zsur_adam");
}

const char *zsur_last_error(void) { return g_err.c_str(); }

}  // extern "C"
