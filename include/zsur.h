/*
 * zsur.h -- C ABI of the surrogate kernels (gfx950): a small convolutional
 * network that maps a zone's design-layer pattern to its complex exit-plane
 * DFT fields, so that inner design iterations can run on it while the FDTD
 * (libzda) stays the arbiter that re-verifies every k-th iterate.  The
 * surrogate is not part of arXiv 2501.07979; it is the learned accelerator
 * of its inverse-design loop (the paper's gradient is the adjoint of the
 * section "Differentiable FDTD in cylindrical coordinates", which the
 * surrogate's own gradient stands in for between checks).
 *
 * Conventions shared by every call:
 *  - bf16 operands are IEEE bfloat16 bit patterns (uint16_t), rounded to
 *    nearest even from FP32; every product is accumulated in FP32 by the
 *    MFMA units (v_mfma_f32_16x16x32_bf16).
 *  - Activations are channel-major: [C][B][H][W] with W (phi) fastest,
 *    i.e. a C x N matrix with N = B*H*W.  Convolutions are 3x3 with
 *    dilation d, periodic padding along W (the wedge's phi period; fields
 *    are stored with the Bloch phase removed) and zero padding along H (r).
 *  - All pointers are device pointers the caller owns; nothing is allocated
 *    by the library.  `stream` is a hipStream_t (NULL = the null stream);
 *    every call is asynchronous on it.
 *  - Return: ZSUR_OK, ZSUR_ERR_ARG (a size <= 0 where one is required, a
 *    NULL pointer, a split count < 1), ZSUR_ERR_HIP (a launch failed; the
 *    text is in zsur_last_error()).
 */
#ifndef ZSUR_H
#define ZSUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { ZSUR_OK = 0, ZSUR_ERR_ARG = 1, ZSUR_ERR_HIP = 2 } zsur_status;

#define ZSUR_ACT_NONE 0
#define ZSUR_ACT_LEAKY 1   /* y = z for z > 0, slope * z otherwise */

/* C(m, n) = act( sum_k A(m, k) B(k, n) + bias[m] ), m < M, n < N, k < K.
 * A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn] (bf16, element
 * strides, so either operand may be read transposed); C[m*ldc + n] FP32;
 * Cb (optional, may be NULL) receives a bf16 copy of C with the same
 * layout.  bias may be NULL.  split > 1 cuts K into `split` slices whose
 * partial products go to work[split][M][N] (FP32, caller-owned, at least
 * split*M*N floats) and are summed in a fixed order by a second kernel, so
 * results do not depend on scheduling. */
zsur_status zsur_gemm(int M, int N, int K, const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk,
                      long sbn, float *C, long ldc, uint16_t *Cb, const float *bias, int act, float slope,
                      int split, float *work, void *stream);

/* cols[(c*9 + ky*3 + kx)][b*H*W + y*W + x] = bf16( x_in[c][b][y + d(ky-1)][(x + d(kx-1)) mod W] ),
 * zero where y + d(ky-1) is outside [0, H).  x_in FP32 [C][B][H][W].
 * B*H*W < 2^31 and C*9 <= 65535. */
zsur_status zsur_im2col(const float *x, int C, int B, int H, int W, int dil, uint16_t *cols, void *stream);

/* The adjoint of zsur_im2col: dx[c][b][y][x] = sum of dcols entries that
 * zsur_im2col reads from (c, b, y, x).  dcols FP32 [C*9][B*H*W]. */
zsur_status zsur_col2im(const float *dcols, int C, int B, int H, int W, int dil, float *dx, void *stream);

/* Leaky activation backward: dz[i] = dy[i] * (y[i] > 0 ? 1 : slope) (in
 * place on dy allowed), and a bf16 copy into dzb (may be NULL). */
zsur_status zsur_act_grad(const float *y, const float *dy, float *dz, uint16_t *dzb, size_t n, float slope,
                          void *stream);

/* out[m] = sum_n x[m*N + n] (FP32, fixed order: 64 slices per row summed
 * in order); partial holds at least 64*M floats.  M <= 65535. */
zsur_status zsur_rowsum(const float *x, int M, int N, float *out, float *partial, void *stream);

/* Mean squared error: d[i] = 2 (p[i] - t[i]) / n, loss[0] = sum (p - t)^2 / n
 * (two-pass, fixed order; `partial` holds at least 1024 floats). */
zsur_status zsur_mse(const float *p, const float *t, size_t n, float *d, float *loss, float *partial,
                     void *stream);

/* FP32 -> bf16 (round to nearest even). */
zsur_status zsur_to_bf16(const float *x, uint16_t *y, size_t n, void *stream);

/* One Adam step (t >= 1): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr mhat / (sqrt(vhat) + eps); pb (may be NULL) gets bf16(p). */
zsur_status zsur_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                      float eps, int t, uint16_t *pb, void *stream);

const char *zsur_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ZSUR_H */
