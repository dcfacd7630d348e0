// Kernels of the learned coarse propagator Psi(u) = u + f(u) (gfx950).
//
// Layout: activations are NHWC BF16, [field][y][x][32]; a pixel's 32 channels
// are 64 contiguous bytes, so one 16-byte load gives 8 channels of a pixel.
// The 32 -> 32 convolutions run on MFMA (v_mfma_f32_16x16x32_bf16): per 3x3
// tap, A = the tap's 16x32 weight block (output channel x input channel),
// B = 32 input channels of 16 neighbouring pixels, D = 16 output channels of
// the 16 pixels in FP32.  Each wave keeps the 18 weight fragments of its layer
// in registers and walks 16-pixel row segments.  The 1 -> 32 and 32 -> 1
// layers, the weight gradients (FP32 sums of exact BF16 products), the loss
// and Adam run on the vector ALUs.
//
// Arithmetic (the same points of rounding as the CPU oracle in bf16 mode):
//   x0 = bf16(x); z1 = b1 + sum_t W1[t] x0(p+t); a1 = bf16(relu(z1))
//   z2 = b2 + sum_t W2[t] a1(p+t) (MFMA, FP32); a2 = bf16(relu(z2)); a3 likewise
//   f  = b4 + sum_t W4[t] . a3(p+t) (FP32)
// weights used in BF16; biases FP32.  Back-propagation rounds the signals of
// layers 3, 2, 1 to BF16 after the ReLU mask.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "atm_cnn.hpp"
#include "atm_device.hpp"

namespace atm {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16r(float v) { return (float)(__bf16)v; }

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// layer 1 (1 -> 32), VALU: forward (bias + ReLU) or Jacobian-vector product
// (no bias, ReLU mask of a stored activation)
// ---------------------------------------------------------------------------


__global__ __launch_bounds__(256) void l1_kernel(L1Args a)
{
    const int64_t npix = (int64_t)a.h * a.w;
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= a.nb * npix) return;
    const int64_t b = gid / npix, p = gid % npix;
    const int y = (int)(p / a.w), x = (int)(p % a.w);
    const int64_t f = map_field(a.xmap, b);
    float xin[TAPS];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) {
        const int yy = wrap(y + t / 3 - 1, a.h), xx = wrap(x + t % 3 - 1, a.w);
        const int64_t i = f * a.x_stride + (int64_t)yy * a.w + xx;
        const float v = a.x_f64 ? (float)static_cast<const double*>(a.x)[i] : static_cast<const float*>(a.x)[i];
        xin[t] = bf16r(v);
    }
    const __bf16* mref = a.ref ? a.ref + (map_field(a.refmap, b) * npix + p) * C : nullptr;
    __bf16* o = a.out + gid * C;
#pragma unroll
    for (int c0 = 0; c0 < C; c0 += 8) {
        bf16x8 v;
        bf16x8 m;
        if (mref) m = *reinterpret_cast<const bf16x8*>(mref + c0);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float z = a.b1 ? a.b1[c0 + c] : 0.0f;
#pragma unroll
            for (int t = 0; t < TAPS; ++t) z += (float)a.w1[t * C + c0 + c] * xin[t];
            if (mref)
                z = ((float)m[c] > 0.0f) ? z : 0.0f;
            else
                z = z > 0.0f ? z : 0.0f;
            v[c] = (__bf16)z;
        }
        *reinterpret_cast<bf16x8*>(o + c0) = v;
    }
}

// ---------------------------------------------------------------------------
// 32 -> 32 convolution on MFMA
// ---------------------------------------------------------------------------


__global__ __launch_bounds__(256) void conv32_kernel(ConvArgs a)
{
    const int lane = threadIdx.x & 63;
    const int col = lane & 15;  // pixel of the tile (B and D), output channel row of A
    const int kq = lane >> 4;   // 8-channel group of the K dimension
    // weight fragments of all taps: A[t][mb] = W[t][16 mb + col][8 kq .. 8 kq + 7]
    bf16x8 wa[TAPS][2];
#pragma unroll
    for (int t = 0; t < TAPS; ++t)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
            wa[t][mb] = *reinterpret_cast<const bf16x8*>(a.wpk + (t * C + 16 * mb + col) * C + 8 * kq);
    float bias[2][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) bias[mb][r] = a.bias ? a.bias[16 * mb + 4 * kq + r] : 0.0f;
    const int tpr = a.w / 16;
    const int64_t npix = (int64_t)a.h * a.w;
    const int64_t ntiles = a.nb * a.h * tpr;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles; tile += nwaves) {
        const int64_t b = tile / ((int64_t)a.h * tpr);
        const int64_t rem = tile % ((int64_t)a.h * tpr);
        const int y = (int)(rem / tpr);
        const int x0 = (int)(rem % tpr) * 16;
        const __bf16* in = a.in + b * npix * C;
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < TAPS; ++t) {
            const int yy = wrap(y + t / 3 - 1, a.h);
            const int xx = wrap(x0 + col + t % 3 - 1, a.w);
            const bf16x8 bv = *reinterpret_cast<const bf16x8*>(in + ((int64_t)yy * a.w + xx) * C + 8 * kq);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t][0], bv, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t][1], bv, acc1, 0, 0, 0);
        }
        // D[out channel 16 mb + 4 kq + r][pixel col]
        const int64_t pix = (int64_t)y * a.w + x0 + col;
        __bf16* o = a.out + (b * npix + pix) * C + 4 * kq;
        const __bf16* mr = a.bias ? nullptr : a.ref + (map_field(a.refmap, b) * npix + pix) * C + 4 * kq;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const f32x4 acc = mb ? acc1 : acc0;
            bf16x4 v;
            bf16x4 m;
            if (mr) m = *reinterpret_cast<const bf16x4*>(mr + 16 * mb);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float z = acc[r];
                if (mr)
                    z = ((float)m[r] > 0.0f) ? z : 0.0f;
                else {
                    z += bias[mb][r];
                    z = z > 0.0f ? z : 0.0f;
                }
                v[r] = (__bf16)z;
            }
            *reinterpret_cast<bf16x4*>(o + 16 * mb) = v;
        }
    }
}

// ---------------------------------------------------------------------------
// layer 4 (32 -> 1), VALU, with the epilogues of its three uses
// ---------------------------------------------------------------------------



__global__ __launch_bounds__(256) void l4_kernel(L4Args a)
{
    __shared__ float red[4];
    const int64_t npix = (int64_t)a.h * a.w;
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float d2 = 0.0f;
    if (gid < a.nb * npix) {
        const int64_t b = gid / npix, p = gid % npix;
        const int y = (int)(p / a.w), x = (int)(p % a.w);
        const __bf16* in = a.in + b * npix * C;
        float f = a.b4 ? a.b4[0] : 0.0f;
#pragma unroll
        for (int t = 0; t < TAPS; ++t) {
            const int yy = wrap(y + t / 3 - 1, a.h), xx = wrap(x + t % 3 - 1, a.w);
            const __bf16* src = in + ((int64_t)yy * a.w + xx) * C;
#pragma unroll
            for (int c0 = 0; c0 < C; c0 += 8) {
                const bf16x8 v = *reinterpret_cast<const bf16x8*>(src + c0);
#pragma unroll
                for (int c = 0; c < 8; ++c) f += (float)a.w4[t * C + c0 + c] * (float)v[c];
            }
        }
        if (a.epi == EPI_F32) {
            a.out[gid] = (a.add ? a.add[gid] : 0.0f) + f;
        } else if (a.epi == EPI_TRAIN) {
            const float xv = a.frames[map_field(a.xmap, b) * npix + p];
            const float yv = a.frames[map_field(a.ymap, b) * npix + p];
            const float d = xv + f - yv;
            a.g4[gid] = a.two_over_n * d;
            d2 = d * d;
        } else if (a.epi == EPI_WINDOW) {
            const int64_t j = map_field(a.smap, b) + 1;
            const int64_t ei = map_field(a.emap, b) * npix + p;
            a.e[ei] = (a.e[ei] + (double)f) + a.tau[j * npix + p];
        } else {
            const int64_t j = b + 1;
            const double vj = a.usol[(j * a.m) * npix + p];
            const double psi = a.usol[((j - 1) * a.m) * npix + p] + (double)f;
            a.tau[j * npix + p] = (vj - psi) + (a.ysol[j * npix + p] - vj);
        }
    }
    if (a.epi == EPI_TRAIN) {
        // fixed-order block sum of d^2
        float v = d2;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) a.loss_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// back-propagation through layer 4: g3(p)[c] = bf16([a3(p)[c] > 0] sum_t W4[t][c] g4(p - t))

__global__ __launch_bounds__(256) void l4_back_kernel(L4BArgs a)
{
    const int64_t npix = (int64_t)a.h * a.w;
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= a.nb * npix) return;
    const int64_t b = gid / npix, p = gid % npix;
    const int y = (int)(p / a.w), x = (int)(p % a.w);
    float g[TAPS];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) {
        const int yy = wrap(y - (t / 3 - 1), a.h), xx = wrap(x - (t % 3 - 1), a.w);
        g[t] = a.g4[b * npix + (int64_t)yy * a.w + xx];
    }
#pragma unroll
    for (int c0 = 0; c0 < C; c0 += 8) {
        const bf16x8 m = *reinterpret_cast<const bf16x8*>(a.a3 + gid * C + c0);
        bf16x8 v;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float s = 0.0f;
#pragma unroll
            for (int t = 0; t < TAPS; ++t) s += (float)a.w4[t * C + c0 + c] * g[t];
            v[c] = (__bf16)(((float)m[c] > 0.0f) ? s : 0.0f);
        }
        *reinterpret_cast<bf16x8*>(a.g3 + gid * C + c0) = v;
    }
}

// ---------------------------------------------------------------------------
// weight gradients: each workgroup sums over a contiguous range of grid rows
// (all fields stacked) and writes one partial row; a fixed-order reduction
// over the kGradBlocks rows follows
// ---------------------------------------------------------------------------


__device__ __forceinline__ void row_range(const DWArgs& a, int64_t& r0, int64_t& r1)
{
    const int64_t rows = a.nb * a.h;
    const int64_t per = (rows + kGradBlocks - 1) / kGradBlocks;
    r0 = (int64_t)blockIdx.x * per;
    r1 = r0 + per < rows ? r0 + per : rows;
}

// 32 -> 32 layers: dW[t][o][i] = sum_p g(p)[o] a(p + t)[i], db[o] = sum_p g(p)[o].
// 256 threads: o = tid % 32, input channels 4 (tid / 32) .. + 3, all nine taps.
__global__ __launch_bounds__(256) void dw32_kernel(DWArgs a, int off_w, int off_b)
{
    extern __shared__ float lds[];  // g row [w][32], a rows [3][w][32]
    float* gl = lds;
    float* al = lds + a.w * C;
    const int o = threadIdx.x & 31;
    const int i0 = 4 * (threadIdx.x >> 5);
    float acc[TAPS][4];
#pragma unroll
    for (int t = 0; t < TAPS; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] = 0.0f;
    float accb = 0.0f;
    int64_t r0, r1;
    row_range(a, r0, r1);
    const int64_t npix = (int64_t)a.h * a.w;
    for (int64_t row = r0; row < r1; ++row) {
        const int64_t b = row / a.h;
        const int y = (int)(row % a.h);
        __syncthreads();
        for (int idx = threadIdx.x; idx < a.w * C; idx += 256)
            gl[idx] = (float)a.g[(b * npix + (int64_t)y * a.w) * C + idx];
        for (int idx = threadIdx.x; idx < 3 * a.w * C; idx += 256) {
            const int dy = idx / (a.w * C) - 1;
            const int rest = idx % (a.w * C);
            al[idx] = (float)a.a[(b * npix + (int64_t)wrap(y + dy, a.h) * a.w) * C + rest];
        }
        __syncthreads();
        for (int x = 0; x < a.w; ++x) {
            const float gv = gl[x * C + o];
            accb += gv;
#pragma unroll
            for (int t = 0; t < TAPS; ++t) {
                const int xx = wrap(x + t % 3 - 1, a.w);
                const float4 av = *reinterpret_cast<const float4*>(al + ((t / 3) * a.w + xx) * C + i0);
                acc[t][0] += gv * av.x;
                acc[t][1] += gv * av.y;
                acc[t][2] += gv * av.z;
                acc[t][3] += gv * av.w;
            }
        }
    }
    float* pr = a.part + (int64_t)blockIdx.x * N_PARAMS;
#pragma unroll
    for (int t = 0; t < TAPS; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) pr[off_w + (t * C + o) * C + i0 + r] = acc[t][r];
    if (i0 == 0) pr[off_b + o] = accb;
}

// layer 1: dW1[t][c] = sum_p g1(p)[c] x0(p + t), db1[c] = sum_p g1(p)[c]; 320 threads (t = tid / 32, 9 = bias)
__global__ __launch_bounds__(320) void dw1_kernel(DWArgs a)
{
    extern __shared__ float lds[];  // g row [w][32], x rows [3][w]
    float* gl = lds;
    float* xl = lds + a.w * C;
    const int c = threadIdx.x & 31;
    const int t = threadIdx.x >> 5;
    float acc = 0.0f;
    int64_t r0, r1;
    row_range(a, r0, r1);
    const int64_t npix = (int64_t)a.h * a.w;
    for (int64_t row = r0; row < r1; ++row) {
        const int64_t b = row / a.h;
        const int y = (int)(row % a.h);
        __syncthreads();
        for (int idx = threadIdx.x; idx < a.w * C; idx += 320)
            gl[idx] = (float)a.g[(b * npix + (int64_t)y * a.w) * C + idx];
        const int64_t f = map_field(a.xmap, b);
        for (int idx = threadIdx.x; idx < 3 * a.w; idx += 320) {
            const int dy = idx / a.w - 1;
            xl[idx] = bf16r(a.frames[f * npix + (int64_t)wrap(y + dy, a.h) * a.w + idx % a.w]);
        }
        __syncthreads();
        if (t < TAPS) {
            for (int x = 0; x < a.w; ++x) acc += gl[x * C + c] * xl[(t / 3) * a.w + wrap(x + t % 3 - 1, a.w)];
        } else {
            for (int x = 0; x < a.w; ++x) acc += gl[x * C + c];
        }
    }
    float* pr = a.part + (int64_t)blockIdx.x * N_PARAMS;
    if (t < TAPS)
        pr[OFF_W1 + t * C + c] = acc;
    else
        pr[OFF_B1 + c] = acc;
}

// layer 4: dW4[t][i] = sum_p g4(p) a3(p + t)[i], db4 = sum_p g4(p); 320 threads (t = tid / 32, 9 = bias)
__global__ __launch_bounds__(320) void dw4_kernel(DWArgs a)
{
    extern __shared__ float lds[];  // g4 row [w], a3 rows [3][w][32]
    float* gl = lds;
    float* al = lds + a.w;
    const int i = threadIdx.x & 31;
    const int t = threadIdx.x >> 5;
    float acc = 0.0f;
    int64_t r0, r1;
    row_range(a, r0, r1);
    const int64_t npix = (int64_t)a.h * a.w;
    for (int64_t row = r0; row < r1; ++row) {
        const int64_t b = row / a.h;
        const int y = (int)(row % a.h);
        __syncthreads();
        for (int idx = threadIdx.x; idx < a.w; idx += 320) gl[idx] = a.g4[b * npix + (int64_t)y * a.w + idx];
        for (int idx = threadIdx.x; idx < 3 * a.w * C; idx += 320) {
            const int dy = idx / (a.w * C) - 1;
            al[idx] = (float)a.a[(b * npix + (int64_t)wrap(y + dy, a.h) * a.w) * C + idx % (a.w * C)];
        }
        __syncthreads();
        if (t < TAPS) {
            for (int x = 0; x < a.w; ++x) acc += gl[x] * al[((t / 3) * a.w + wrap(x + t % 3 - 1, a.w)) * C + i];
        } else if (i == 0) {
            for (int x = 0; x < a.w; ++x) acc += gl[x];
        }
    }
    float* pr = a.part + (int64_t)blockIdx.x * N_PARAMS;
    if (t < TAPS)
        pr[OFF_W4 + t * C + i] = acc;
    else if (i == 0)
        pr[OFF_B4] = acc;
}

// grad[k] = sum over the partial rows in a fixed order
__global__ __launch_bounds__(256) void grad_reduce_kernel(const float* part, float* grad)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N_PARAMS) return;
    float s = 0.0f;
    for (int r = 0; r < kGradBlocks; ++r) s += part[(int64_t)r * N_PARAMS + k];
    grad[k] = s;
}

__global__ __launch_bounds__(256) void loss_reduce_kernel(const float* part, int64_t n, float inv_n, float* loss)
{
    __shared__ float red[4];
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) loss[0] = ((red[0] + red[1]) + (red[2] + red[3])) * inv_n;
}

// Adam (Kingma and Ba) on the FP32 parameters
__global__ __launch_bounds__(256) void adam_kernel(float* params, const float* grad, float* m, float* v, float lr,
                                                   float b1, float b2, float c1, float c2, float eps)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N_PARAMS) return;
    const float g = grad[k];
    const float mk = b1 * m[k] + (1.0f - b1) * g;
    const float vk = b2 * v[k] + (1.0f - b2) * g * g;
    m[k] = mk;
    v[k] = vk;
    params[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// BF16 copies of the weights: forward layouts, and the adjoint layout of the 32 -> 32 layers
// (Wb[t'][i][o] = W[8 - t'][o][i]: the transposed convolution as a forward one)
__global__ __launch_bounds__(256) void pack_kernel(const float* params, __bf16* pk)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= PK_N) return;
    float v;
    if (k < PK_W2F) {
        v = params[OFF_W1 + k];
    } else if (k < PK_W3F) {
        v = params[OFF_W2 + (k - PK_W2F)];
    } else if (k < PK_W2B) {
        v = params[OFF_W3 + (k - PK_W3F)];
    } else if (k < PK_W4) {
        const bool l2 = k < PK_W3B;
        const int q = k - (l2 ? PK_W2B : PK_W3B);
        const int tb = q / (C * C), i = (q / C) % C, o = q % C;
        v = params[(l2 ? OFF_W2 : OFF_W3) + ((TAPS - 1 - tb) * C + o) * C + i];
    } else {
        v = params[OFF_W4 + (k - PK_W4)];
    }
    pk[k] = (__bf16)v;
}

// FAS windows of the learned coarse solve start at w_p = v_s + r_s, s = max(0, p - k + 1), v_s = u_{sm},
// r_0 = 0, r_s = y_s - u_{sm}; they end with e_p = w_p - v_p
__global__ __launch_bounds__(256) void window_init_kernel(double* e, const double* y, const double* u, int64_t NT,
                                                          int64_t n, int m, int k)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (NT + 1) * n) return;
    const int64_t p = gid / n, i = gid % n;
    const int64_t s = p - k + 1 > 0 ? p - k + 1 : 0;
    const double vs = u[(s * m) * n + i];
    e[gid] = (s == 0) ? vs : vs + (y[s * n + i] - vs);
}

__global__ __launch_bounds__(256) void window_final_kernel(double* e, const double* u, int64_t NT, int64_t n, int m)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (NT + 1) * n) return;
    const int64_t p = gid / n, i = gid % n;
    e[gid] = e[gid] - u[(p * m) * n + i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

void launch_window_init(double* e, const double* y, const double* u, int64_t NT, int64_t n, int m, int k,
                        hipStream_t s)
{
    hipLaunchKernelGGL(window_init_kernel, dim3((unsigned)(((NT + 1) * n + 255) / 256)), dim3(256), 0, s, e, y, u, NT,
                       n, m, k);
}

void launch_window_final(double* e, const double* u, int64_t NT, int64_t n, int m, hipStream_t s)
{
    hipLaunchKernelGGL(window_final_kernel, dim3((unsigned)(((NT + 1) * n + 255) / 256)), dim3(256), 0, s, e, u, NT, n,
                       m);
}

static unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void launch_pack(const float* params, __bf16* pk, hipStream_t s)
{
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(PK_N, 256)), dim3(256), 0, s, params, pk);
}

void launch_l1(const L1Args& a, hipStream_t s)
{
    hipLaunchKernelGGL(l1_kernel, dim3(blocks_for(a.nb * a.h * a.w, 256)), dim3(256), 0, s, a);
}

void launch_conv32(const ConvArgs& a, hipStream_t s)
{
    const int64_t ntiles = a.nb * a.h * (a.w / 16);
    int64_t nblk = (ntiles + 3) / 4;
    if (nblk > 4096) nblk = 4096;  // each wave walks several tiles with its weight fragments in registers
    hipLaunchKernelGGL(conv32_kernel, dim3((unsigned)nblk), dim3(256), 0, s, a);
}

void launch_l4(const L4Args& a, hipStream_t s)
{
    hipLaunchKernelGGL(l4_kernel, dim3(blocks_for(a.nb * a.h * a.w, 256)), dim3(256), 0, s, a);
}

void launch_l4_back(const L4BArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(l4_back_kernel, dim3(blocks_for(a.nb * a.h * a.w, 256)), dim3(256), 0, s, a);
}

void launch_dw32(const DWArgs& a, int off_w, int off_b, hipStream_t s)
{
    const size_t lds = (size_t)4 * a.w * C * sizeof(float);
    hipLaunchKernelGGL(dw32_kernel, dim3(kGradBlocks), dim3(256), lds, s, a, off_w, off_b);
}

void launch_dw1(const DWArgs& a, hipStream_t s)
{
    const size_t lds = (size_t)(a.w * C + 3 * a.w) * sizeof(float);
    hipLaunchKernelGGL(dw1_kernel, dim3(kGradBlocks), dim3(320), lds, s, a);
}

void launch_dw4(const DWArgs& a, hipStream_t s)
{
    const size_t lds = (size_t)(a.w + 3 * a.w * C) * sizeof(float);
    hipLaunchKernelGGL(dw4_kernel, dim3(kGradBlocks), dim3(320), lds, s, a);
}

void launch_grad_reduce(const float* part, float* grad, hipStream_t s)
{
    hipLaunchKernelGGL(grad_reduce_kernel, dim3(blocks_for(N_PARAMS, 256)), dim3(256), 0, s, part, grad);
}

void launch_loss_reduce(const float* part, int64_t n, float inv_n, float* loss, hipStream_t s)
{
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(256), 0, s, part, n, inv_n, loss);
}

void launch_adam(float* params, const float* grad, float* m, float* v, int step, float lr, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(N_PARAMS, 256)), dim3(256), 0, s, params, grad, m, v, lr, b1, b2,
                       c1, c2, 1e-8f);
}

}  // namespace cnn
}  // namespace atm
