// Learned coarse propagator Psi(u) = u + f(u): a four-layer 3x3 convolutional
// network on the periodic grid (1 -> 32 -> 32 -> 32 -> 1 channels, ReLU after
// the first three layers), BF16 weights and activations, FP32 accumulation.
// Shared by the CNN kernels (atm_cnn.hip) and the host API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace atm {
namespace cnn {

constexpr int C = 32;     // hidden channels
constexpr int TAPS = 9;   // 3x3 stencil, tap t = (dy + 1) * 3 + (dx + 1)
// FP32 parameter vector
constexpr int OFF_W1 = 0;                    // [9][32]      (tap, out)
constexpr int OFF_B1 = OFF_W1 + TAPS * C;    // [32]
constexpr int OFF_W2 = OFF_B1 + C;           // [9][32][32]  (tap, out, in)
constexpr int OFF_B2 = OFF_W2 + TAPS * C * C;
constexpr int OFF_W3 = OFF_B2 + C;
constexpr int OFF_B3 = OFF_W3 + TAPS * C * C;
constexpr int OFF_W4 = OFF_B3 + C;           // [9][32]      (tap, in)
constexpr int OFF_B4 = OFF_W4 + TAPS * C;    // [1]
constexpr int N_PARAMS = OFF_B4 + 1;         // 19105
// BF16 copies (element offsets in the packed array)
constexpr int PK_W1 = 0;                     // [9][32]
constexpr int PK_W2F = PK_W1 + TAPS * C;     // forward  [9][out][in]
constexpr int PK_W3F = PK_W2F + TAPS * C * C;
constexpr int PK_W2B = PK_W3F + TAPS * C * C;  // adjoint [9][in][out] with the taps reversed
constexpr int PK_W3B = PK_W2B + TAPS * C * C;
constexpr int PK_W4 = PK_W3B + TAPS * C * C;  // [9][32]
constexpr int PK_N = PK_W4 + TAPS * C;
constexpr int kGradBlocks = 512;  // workgroups of the weight-gradient reductions (one partial row each)

// How a batch index b selects a field of a stacked array.
struct FieldMap {
    int mode;            // 0: off + b; 1: index[b]; 2: window state max(0, t + b - k + 1) + t - 1
    int t, k;
    int64_t off;
    const int32_t* index;
};

__host__ __device__ inline int64_t map_field(const FieldMap& m, int64_t b)
{
    if (m.mode == 1) return m.index[b];
    if (m.mode == 2) {
        const int64_t p = m.t + b;
        const int64_t s = p - m.k + 1 > 0 ? p - m.k + 1 : 0;
        return s + m.t - 1;
    }
    return m.off + b;
}


// kernel arguments (atm_cnn.hip)

enum { EPI_F32 = 0, EPI_TRAIN = 1, EPI_WINDOW = 2, EPI_TAU = 3 };

struct L1Args {
    int64_t nb;
    int h, w;
    const void* x;  // stacked input fields, FP32 or FP64
    int x_f64;
    int64_t x_stride;  // elements between fields
    FieldMap xmap;
    const __bf16* w1;  // packed [9][32]
    const float* b1;   // forward only
    const __bf16* ref;  // masks: stacked activations [field][h][w][32] (nullptr: ReLU)
    FieldMap refmap;
    __bf16* out;  // [nb][h][w][32]
};

struct ConvArgs {
    int64_t nb;
    int h, w;
    const __bf16* in;   // [nb][h][w][32]
    __bf16* out;        // [nb][h][w][32]
    const __bf16* wpk;  // [9][32 out][32 in]
    const float* bias;  // forward: bias + ReLU; nullptr: mask by ref
    const __bf16* ref;  // stacked activations for the mask
    FieldMap refmap;
};

struct L4Args {
    int64_t nb;
    int h, w;
    const __bf16* in;  // a3 (forward) or the product signal (JVP), [nb][h][w][32]
    const __bf16* w4;  // packed [9][32]
    const float* b4;   // forward only
    int epi;
    // EPI_F32: out[b][p] = (add ? add[b][p] : 0) + f
    float* out;
    const float* add;
    // EPI_TRAIN: d = x + f - y; g4 = 2 d / N; per-block sum of d^2
    const float* frames;
    FieldMap xmap, ymap;
    float* g4;
    float* loss_part;
    float two_over_n;
    // EPI_WINDOW (FAS window step): w (FP64, in/out) = (w + f) + tau_j, w = e[emap(b)], j = smap(b) + 1
    // EPI_TAU: tau_j = (v_j - (v_{j-1} + f)) + (y_j - v_j), v_j = u_{jm}, j = b + 1
    double* e;
    FieldMap emap, smap;
    double* tau;
    const double* ysol;
    const double* usol;
    int m;
};

struct L4BArgs {
    int64_t nb;
    int h, w;
    const float* g4;
    const __bf16* w4;
    const __bf16* a3;
    __bf16* g3;
};

struct DWArgs {
    int64_t nb;
    int h, w;
    const __bf16* g;   // back-propagated signal at the layer's output, [nb][h][w][32] (layer 4: FP32 g4)
    const float* g4;
    const __bf16* a;   // the layer's input activations [nb][h][w][32]
    const float* frames;  // layer 1: the input fields x (x0 = bf16(x))
    FieldMap xmap;
    float* part;  // [kGradBlocks][N_PARAMS]
};

void launch_pack(const float* params, __bf16* pk, hipStream_t s);
void launch_l1(const L1Args& a, hipStream_t s);
void launch_conv32(const ConvArgs& a, hipStream_t s);
void launch_l4(const L4Args& a, hipStream_t s);
void launch_l4_back(const L4BArgs& a, hipStream_t s);
void launch_dw32(const DWArgs& a, int off_w, int off_b, hipStream_t s);
void launch_dw1(const DWArgs& a, hipStream_t s);
void launch_dw4(const DWArgs& a, hipStream_t s);
void launch_grad_reduce(const float* part, float* grad, hipStream_t s);
void launch_loss_reduce(const float* part, int64_t n, float inv_n, float* loss, hipStream_t s);
void launch_adam(float* params, const float* grad, float* m, float* v, int step, float lr, hipStream_t s);
void launch_window_init(double* e, const double* y, const double* u, int64_t NT, int64_t n, int m, int k,
                        hipStream_t s);
void launch_window_final(double* e, const double* u, int64_t NT, int64_t n, int m, hipStream_t s);

}  // namespace cnn
}  // namespace atm
