// C-ABI of the learned coarse propagator: forward, Jacobian-vector product,
// gradients and one Adam training step (see include/atm.h).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "../../include/atm.h"
#include "atm_cnn.hpp"
#include "atm_kernels.hpp"

namespace {

using namespace atm::cnn;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

atm_status cnn_fail(atm_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
atm_status cnn_fail(atm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    atm::set_last_error(buf);
    return st;
}

#define CNN_HIP(call)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return cnn_fail(ATM_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

atm_status check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cnn_fail(ATM_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    return ATM_OK;
}

struct CnnLayout {
    size_t pk, a1, a2, a3, ga, gb, g4, part, grad, lpart, loss, idx, total;
};

int64_t loss_blocks(int64_t npx) { return (npx + 255) / 256; }

CnnLayout cnn_layout(int64_t nb, int64_t h, int64_t w)
{
    const size_t npx = (size_t)(nb * h * w);
    const size_t act = npx * C * 2;
    CnnLayout L;
    size_t off = 0;
    L.pk = off;
    off += align_up(PK_N * 2);
    L.a1 = off;
    off += align_up(act);
    L.a2 = off;
    off += align_up(act);
    L.a3 = off;
    off += align_up(act);
    L.ga = off;
    off += align_up(act);
    L.gb = off;
    off += align_up(act);
    L.g4 = off;
    off += align_up(npx * 4);
    L.part = off;
    off += align_up((size_t)kGradBlocks * N_PARAMS * 4);
    L.grad = off;
    off += align_up(N_PARAMS * 4);
    L.lpart = off;
    off += align_up((size_t)loss_blocks((int64_t)npx) * 4);
    L.loss = off;
    off += align_up(4);
    L.idx = off;
    off += align_up((size_t)nb * 2 * 4);
    L.total = off;
    return L;
}

atm_status cnn_validate(int32_t batch, int32_t h, int32_t w)
{
    if (batch < 1) return cnn_fail(ATM_ERR_INVALID_ARG, "batch must be >= 1");
    if (h < 1) return cnn_fail(ATM_ERR_INVALID_ARG, "h must be >= 1");
    if (w < 16 || w % 16 != 0 || w > 128)
        return cnn_fail(ATM_ERR_UNSUPPORTED, "w must be a multiple of 16 in [16, 128] (got %d)", w);
    return ATM_OK;
}

struct Bufs {
    __bf16 *pk, *a1, *a2, *a3, *ga, *gb;
    float *g4, *part, *grad, *lpart, *loss;
    int32_t* idx;
};

atm_status cnn_bufs(int32_t batch, int32_t h, int32_t w, void* ws, size_t ws_bytes, Bufs& B)
{
    atm_status st = cnn_validate(batch, h, w);
    if (st) return st;
    const CnnLayout L = cnn_layout(batch, h, w);
    if (!ws) return cnn_fail(ATM_ERR_INVALID_ARG, "null workspace");
    if (((uintptr_t)ws) % kAlign) return cnn_fail(ATM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return cnn_fail(ATM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
    char* b = (char*)ws;
    B.pk = (__bf16*)(b + L.pk);
    B.a1 = (__bf16*)(b + L.a1);
    B.a2 = (__bf16*)(b + L.a2);
    B.a3 = (__bf16*)(b + L.a3);
    B.ga = (__bf16*)(b + L.ga);
    B.gb = (__bf16*)(b + L.gb);
    B.g4 = (float*)(b + L.g4);
    B.part = (float*)(b + L.part);
    B.grad = (float*)(b + L.grad);
    B.lpart = (float*)(b + L.lpart);
    B.loss = (float*)(b + L.loss);
    B.idx = (int32_t*)(b + L.idx);
    return ATM_OK;
}

FieldMap fmap_off(int64_t off)
{
    FieldMap m;
    memset(&m, 0, sizeof(m));
    m.mode = 0;
    m.off = off;
    return m;
}

FieldMap fmap_index(const int32_t* idx)
{
    FieldMap m = fmap_off(0);
    m.mode = 1;
    m.index = idx;
    return m;
}

// forward pass of a batch whose input fields are given by (x, x_f64, xmap); activations into B.a1..a3
void forward_batch(const float* params, const Bufs& B, int64_t nb, int h, int w, const void* x, int x_f64,
                   FieldMap xmap, hipStream_t s)
{
    const int64_t npix = (int64_t)h * w;
    L1Args l1;
    memset(&l1, 0, sizeof(l1));
    l1.nb = nb;
    l1.h = h;
    l1.w = w;
    l1.x = x;
    l1.x_f64 = x_f64;
    l1.x_stride = npix;
    l1.xmap = xmap;
    l1.w1 = B.pk + PK_W1;
    l1.b1 = params + OFF_B1;
    l1.out = B.a1;
    launch_l1(l1, s);
    ConvArgs cv;
    memset(&cv, 0, sizeof(cv));
    cv.nb = nb;
    cv.h = h;
    cv.w = w;
    cv.in = B.a1;
    cv.out = B.a2;
    cv.wpk = B.pk + PK_W2F;
    cv.bias = params + OFF_B2;
    launch_conv32(cv, s);
    cv.in = B.a2;
    cv.out = B.a3;
    cv.wpk = B.pk + PK_W3F;
    cv.bias = params + OFF_B3;
    launch_conv32(cv, s);
}

atm_status copy_indices(const Bufs& B, const int32_t* idx_x, const int32_t* idx_y, int32_t batch, int32_t n_frames,
                        hipStream_t s)
{
    for (int32_t i = 0; i < batch; ++i) {
        if (idx_x[i] < 0 || idx_x[i] >= n_frames || idx_y[i] < 0 || idx_y[i] >= n_frames)
            return cnn_fail(ATM_ERR_INVALID_ARG, "frame index %d of the batch is outside [0, %d)", i, n_frames);
    }
    // pageable host memory: the copy has taken the data when the call returns
    CNN_HIP(hipMemcpyAsync(B.idx, idx_x, (size_t)batch * 4, hipMemcpyHostToDevice, s));
    CNN_HIP(hipMemcpyAsync(B.idx + batch, idx_y, (size_t)batch * 4, hipMemcpyHostToDevice, s));
    return ATM_OK;
}

// loss and gradients of one batch into B.grad and B.loss
atm_status gradients_batch(const float* params, const Bufs& B, const float* frames, int32_t batch, int32_t h,
                           int32_t w, hipStream_t s)
{
    const int64_t nb = batch;
    const int64_t npix = (int64_t)h * w;
    launch_pack(params, B.pk, s);
    forward_batch(params, B, nb, h, w, frames, 0, fmap_index(B.idx), s);
    L4Args l4;
    memset(&l4, 0, sizeof(l4));
    l4.nb = nb;
    l4.h = h;
    l4.w = w;
    l4.in = B.a3;
    l4.w4 = B.pk + PK_W4;
    l4.b4 = params + OFF_B4;
    l4.epi = EPI_TRAIN;
    l4.frames = frames;
    l4.xmap = fmap_index(B.idx);
    l4.ymap = fmap_index(B.idx + batch);
    l4.g4 = B.g4;
    l4.loss_part = B.lpart;
    l4.two_over_n = (float)(2.0 / (double)(nb * npix));
    launch_l4(l4, s);
    launch_loss_reduce(B.lpart, loss_blocks(nb * npix), (float)(1.0 / (double)(nb * npix)), B.loss, s);
    // back-propagation
    L4BArgs lb;
    lb.nb = nb;
    lb.h = h;
    lb.w = w;
    lb.g4 = B.g4;
    lb.w4 = B.pk + PK_W4;
    lb.a3 = B.a3;
    lb.g3 = B.ga;
    launch_l4_back(lb, s);
    DWArgs dw;
    memset(&dw, 0, sizeof(dw));
    dw.nb = nb;
    dw.h = h;
    dw.w = w;
    dw.part = B.part;
    dw.g4 = B.g4;
    dw.a = B.a3;
    launch_dw4(dw, s);
    dw.g = B.ga;  // g3
    dw.a = B.a2;
    launch_dw32(dw, OFF_W3, OFF_B3, s);
    ConvArgs cv;
    memset(&cv, 0, sizeof(cv));
    cv.nb = nb;
    cv.h = h;
    cv.w = w;
    cv.in = B.ga;  // g3 -> g2 = bf16(mask(a2) convT(g3, W3))
    cv.out = B.gb;
    cv.wpk = B.pk + PK_W3B;
    cv.ref = B.a2;
    cv.refmap = fmap_off(0);
    launch_conv32(cv, s);
    dw.g = B.gb;  // g2
    dw.a = B.a1;
    launch_dw32(dw, OFF_W2, OFF_B2, s);
    cv.in = B.gb;  // g2 -> g1
    cv.out = B.ga;
    cv.wpk = B.pk + PK_W2B;
    cv.ref = B.a1;
    launch_conv32(cv, s);
    dw.g = B.ga;  // g1
    dw.frames = frames;
    dw.xmap = fmap_index(B.idx);
    launch_dw1(dw, s);
    launch_grad_reduce(B.part, B.grad, s);
    return check_launch();
}

}  // namespace

extern "C" {

int32_t atm_cnn_param_count(void) { return N_PARAMS; }

size_t atm_cnn_workspace_bytes(int32_t batch, int32_t h, int32_t w)
{
    if (batch < 1 || h < 1 || w < 16 || w % 16 != 0 || w > 128) return 0;
    return cnn_layout(batch, h, w).total;
}

atm_status atm_cnn_forward(const float* params, const float* x, int32_t batch, int32_t h, int32_t w, float* f_out,
                           void* ws, size_t ws_bytes, void* stream)
{
    Bufs B;
    atm_status st = cnn_bufs(batch, h, w, ws, ws_bytes, B);
    if (st) return st;
    if (!params || !x || !f_out) return cnn_fail(ATM_ERR_INVALID_ARG, "null params, x or f_out");
    hipStream_t s = (hipStream_t)stream;
    launch_pack(params, B.pk, s);
    forward_batch(params, B, batch, h, w, x, 0, fmap_off(0), s);
    L4Args l4;
    memset(&l4, 0, sizeof(l4));
    l4.nb = batch;
    l4.h = h;
    l4.w = w;
    l4.in = B.a3;
    l4.w4 = B.pk + PK_W4;
    l4.b4 = params + OFF_B4;
    l4.epi = EPI_F32;
    l4.out = f_out;
    launch_l4(l4, s);
    return check_launch();
}

atm_status atm_cnn_jvp(const float* params, const float* v, const float* e, int32_t batch, int32_t h, int32_t w,
                       float* out, void* ws, size_t ws_bytes, void* stream)
{
    Bufs B;
    atm_status st = cnn_bufs(batch, h, w, ws, ws_bytes, B);
    if (st) return st;
    if (!params || !v || !e || !out) return cnn_fail(ATM_ERR_INVALID_ARG, "null params, v, e or out");
    hipStream_t s = (hipStream_t)stream;
    launch_pack(params, B.pk, s);
    forward_batch(params, B, batch, h, w, v, 0, fmap_off(0), s);  // activations (masks) at v
    L1Args l1;
    memset(&l1, 0, sizeof(l1));
    l1.nb = batch;
    l1.h = h;
    l1.w = w;
    l1.x = e;
    l1.x_stride = (int64_t)h * w;
    l1.xmap = fmap_off(0);
    l1.w1 = B.pk + PK_W1;
    l1.ref = B.a1;
    l1.refmap = fmap_off(0);
    l1.out = B.ga;
    launch_l1(l1, s);
    ConvArgs cv;
    memset(&cv, 0, sizeof(cv));
    cv.nb = batch;
    cv.h = h;
    cv.w = w;
    cv.in = B.ga;
    cv.out = B.gb;
    cv.wpk = B.pk + PK_W2F;
    cv.ref = B.a2;
    cv.refmap = fmap_off(0);
    launch_conv32(cv, s);
    cv.in = B.gb;
    cv.out = B.ga;
    cv.wpk = B.pk + PK_W3F;
    cv.ref = B.a3;
    launch_conv32(cv, s);
    L4Args l4;
    memset(&l4, 0, sizeof(l4));
    l4.nb = batch;
    l4.h = h;
    l4.w = w;
    l4.in = B.ga;
    l4.w4 = B.pk + PK_W4;
    l4.epi = EPI_F32;
    l4.out = out;
    l4.add = e;
    launch_l4(l4, s);
    return check_launch();
}

atm_status atm_cnn_gradients(const float* params, const float* frames, int32_t n_frames, const int32_t* idx_x,
                             const int32_t* idx_y, int32_t batch, int32_t h, int32_t w, float* grad_out,
                             float* loss_out, void* ws, size_t ws_bytes, void* stream)
{
    Bufs B;
    atm_status st = cnn_bufs(batch, h, w, ws, ws_bytes, B);
    if (st) return st;
    if (!params || !frames || !idx_x || !idx_y || !grad_out)
        return cnn_fail(ATM_ERR_INVALID_ARG, "null params, frames, indices or grad_out");
    hipStream_t s = (hipStream_t)stream;
    if ((st = copy_indices(B, idx_x, idx_y, batch, n_frames, s))) return st;
    if ((st = gradients_batch(params, B, frames, batch, h, w, s))) return st;
    CNN_HIP(hipMemcpyAsync(grad_out, B.grad, N_PARAMS * 4, hipMemcpyDeviceToDevice, s));
    if (loss_out) CNN_HIP(hipMemcpyAsync(loss_out, B.loss, 4, hipMemcpyDeviceToDevice, s));
    return ATM_OK;
}

atm_status atm_cnn_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                              const float* frames, int32_t n_frames, const int32_t* idx_x, const int32_t* idx_y,
                              int32_t batch, int32_t h, int32_t w, float* loss_out, void* ws, size_t ws_bytes,
                              void* stream)
{
    Bufs B;
    atm_status st = cnn_bufs(batch, h, w, ws, ws_bytes, B);
    if (st) return st;
    if (!params || !adam_m || !adam_v || !frames || !idx_x || !idx_y)
        return cnn_fail(ATM_ERR_INVALID_ARG, "null params, Adam moments, frames or indices");
    if (step < 1) return cnn_fail(ATM_ERR_INVALID_ARG, "step counts from 1");
    if (!(lr > 0.0f)) return cnn_fail(ATM_ERR_INVALID_ARG, "lr must be > 0");
    hipStream_t s = (hipStream_t)stream;
    if ((st = copy_indices(B, idx_x, idx_y, batch, n_frames, s))) return st;
    if ((st = gradients_batch(params, B, frames, batch, h, w, s))) return st;
    launch_adam(params, B.grad, adam_m, adam_v, step, lr, s);
    if (loss_out) CNN_HIP(hipMemcpyAsync(loss_out, B.loss, 4, hipMemcpyDeviceToDevice, s));
    return check_launch();
}

}  // extern "C"
