// Kernels for 2D grids larger than the on-chip strip layout (up to 1024 points per row).
//
// One 1024-thread workgroup per interval or window, as for the small grids, but
// the Krylov vectors of the step's linear solve live in a per-task scratch in
// global memory (they stay in L2 / the MALL: 65536 points x 4 vectors is 1 MB
// in FP32).  A thread owns column x = tid % nx of rows ty, ty + TY, ... (TY =
// 1024 / nx rows per pass): row accesses are coalesced, and the west/east
// neighbours of a thread are fixed for the whole kernel.  Reductions go through
// LDS in a fixed order (bitwise reproducible).  The same step forms as the
// small grids: FP64 direct steps (x0 = previous slice), FP32 defect-correction
// steps with FP64 update (precision 1), FP64 coarse steps.
#include "atm_device.hpp"
#include "atm_kernels.hpp"
#include "atm_pairsync.hpp"
#include "atm_spectral.hpp"

namespace atm {

constexpr int kBlockL = 1024;
constexpr int kWavesL = kBlockL / 64;

struct LCol {
    int x, ty, TY;
    bool act;
    int xw, xe;  // west / east neighbour columns (-1: zero boundary)
};

__device__ __forceinline__ LCol make_col(const Grid2D& g)
{
    LCol c;
    const int TY = kBlockL / g.nx;
    c.TY = TY;
    c.x = threadIdx.x % g.nx;
    c.ty = threadIdx.x / g.nx;
    c.act = c.ty < TY;
    c.xw = c.x > 0 ? c.x - 1 : (g.periodic ? g.nx - 1 : -1);
    c.xe = c.x < g.nx - 1 ? c.x + 1 : (g.periodic ? 0 : -1);
    return c;
}

// M v at (x, y), v a full field in global memory
template <typename T>
__device__ __forceinline__ T stencil_g(const Grid2D& g, const StepCoef& c, const LCol& col, const T* __restrict__ v,
                                       int y)
{
    const int64_t row = (int64_t)y * g.nx;
    const int yn = y > 0 ? y - 1 : (g.periodic ? g.ny - 1 : -1);
    const int ys = y < g.ny - 1 ? y + 1 : (g.periodic ? 0 : -1);
    const T cen = v[row + col.x];
    const T w = col.xw >= 0 ? v[row + col.xw] : (T)0;
    const T e = col.xe >= 0 ? v[row + col.xe] : (T)0;
    const T up = yn >= 0 ? v[(int64_t)yn * g.nx + col.x] : (T)0;
    const T dn = ys >= 0 ? v[(int64_t)ys * g.nx + col.x] : (T)0;
    return stencil_value(c, up, cen, dn, w, e);
}

// The rows of a thread (y = ty, ty + TY, ...).  A plain loop over them waits out one memory
// latency per row, so the passes of the CG below take the rows in batches of kRowBatch: every load
// of a batch is issued before any is used (the vectors are distinct, __restrict__), and the sums
// keep the row order.  The loops outside the CG iterations are unrolled by the same factor.
constexpr int kRowBatch = 4;
#define FOR_ROWS(col, g, y) for (int y = (col).ty; (col).act && y < (g).ny; y += (col).TY)
#define FOR_BATCH(col, g, y0) for (int y0 = (col).ty; (col).act && y0 < (g).ny; y0 += kRowBatch * (col).TY)

// the five stencil inputs of row y (zero outside a Dirichlet boundary)
template <typename T>
struct Nb {
    T cen, w, e, up, dn;
};

// Offsets within one slice are 32-bit (a slice holds at most 1024 x 1024 points), so that a load is
// a uniform base plus one offset register.
__device__ __forceinline__ uint32_t pt(const Grid2D& g, const LCol& col, int y)
{
    return (uint32_t)y * (uint32_t)g.nx + (uint32_t)col.x;
}

template <typename T>
__device__ __forceinline__ Nb<T> load_nb(const Grid2D& g, const LCol& col, const T* __restrict__ v, int y)
{
    const uint32_t row = (uint32_t)y * (uint32_t)g.nx;
    const int yn = y > 0 ? y - 1 : (g.periodic ? g.ny - 1 : -1);
    const int ys = y < g.ny - 1 ? y + 1 : (g.periodic ? 0 : -1);
    Nb<T> b;
    b.cen = v[row + (uint32_t)col.x];
    b.w = col.xw >= 0 ? v[row + (uint32_t)col.xw] : (T)0;
    b.e = col.xe >= 0 ? v[row + (uint32_t)col.xe] : (T)0;
    b.up = yn >= 0 ? v[(uint32_t)yn * (uint32_t)g.nx + (uint32_t)col.x] : (T)0;
    b.dn = ys >= 0 ? v[(uint32_t)ys * (uint32_t)g.nx + (uint32_t)col.x] : (T)0;
    return b;
}

// Jacobi-preconditioned CG (constant diagonal: plain CG on the scaled direction) for M x = b with
// the vectors in global memory.  On entry x = x0, r = b.  Same stopping rule and failure flag as
// the on-chip solver.  Returns the iteration count.
template <typename T>
__device__ int cg_large(const Grid2D& g, const StepCoef& c, const LCol& col, T* __restrict__ x, T* __restrict__ r,
                        T* __restrict__ p, T* __restrict__ q, double* red, int& slot, double rtol2, int maxit,
                        int* fail, double bb_floor = 0.0)
{
    constexpr int U = kRowBatch;
    double bb = 0.0, rr = 0.0;
    // r = b - M x0, p = r (the stencil reads x at neighbours; r and p only at the thread's own points)
    FOR_BATCH(col, g, y0)
    {
        Nb<T> nb[U];
        T b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int y = y0 + u * col.TY;
            if (y < g.ny) {
                nb[u] = load_nb(g, col, x, y);
                b[u] = r[pt(g, col, y)];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int y = y0 + u * col.TY;
            if (y < g.ny) {
                const uint32_t i = pt(g, col, y);
                bb += (double)b[u] * (double)b[u];
                const T ri = b[u] - stencil_value(c, nb[u].up, nb[u].cen, nb[u].dn, nb[u].w, nb[u].e);
                rr += (double)ri * (double)ri;
                r[i] = ri;
                p[i] = ri;
            }
        }
    }
    block_sum2(bb, rr, red, slot, kWavesL);
    const bool bzero = !(bb > bb_floor);
    const double thresh = rtol2 * bb;
    double gamma = rr;
    int it = 0;
    while (!bzero && rr > thresh && it < maxit) {
        // q = M p, (p, q)
        double pq = 0.0;
        FOR_BATCH(col, g, y0)
        {
            Nb<T> nb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int y = y0 + u * col.TY;
                if (y < g.ny) nb[u] = load_nb(g, col, p, y);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int y = y0 + u * col.TY;
                if (y < g.ny) {
                    const T v = stencil_value(c, nb[u].up, nb[u].cen, nb[u].dn, nb[u].w, nb[u].e);
                    q[pt(g, col, y)] = v;
                    pq += (double)nb[u].cen * (double)v;
                }
            }
        }
        pq = block_sum1(pq, red, slot, kWavesL);
        const T alpha = (T)(gamma / pq);
        // x += alpha p, r -= alpha q
        rr = 0.0;
        FOR_BATCH(col, g, y0)
        {
            T xv[U], pv[U], rv[U], qv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int y = y0 + u * col.TY;
                if (y < g.ny) {
                    const uint32_t i = pt(g, col, y);
                    xv[u] = x[i];
                    pv[u] = p[i];
                    rv[u] = r[i];
                    qv[u] = q[i];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int y = y0 + u * col.TY;
                if (y < g.ny) {
                    const uint32_t i = pt(g, col, y);
                    x[i] = xv[u] + alpha * pv[u];
                    const T ri = rv[u] - alpha * qv[u];
                    r[i] = ri;
                    rr += (double)ri * (double)ri;
                }
            }
        }
        rr = block_sum1(rr, red, slot, kWavesL);
        const T beta = (T)(rr / gamma);
        gamma = rr;
        // p = r + beta p
        FOR_BATCH(col, g, y0)
        {
            T rv[U], pv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int y = y0 + u * col.TY;
                if (y < g.ny) {
                    const uint32_t i = pt(g, col, y);
                    rv[u] = r[i];
                    pv[u] = p[i];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int y = y0 + u * col.TY;
                if (y < g.ny) p[pt(g, col, y)] = rv[u] + beta * pv[u];
            }
        }
        __syncthreads();
        ++it;
    }
    if (!bzero && rr > thresh && threadIdx.x == 0) atomicOr(fail, 1);
    if (bzero) {
        FOR_ROWS(col, g, y) x[pt(g, col, y)] = (T)0;
        __syncthreads();
    }
    return it;
}

// per-task scratch: five n-vectors of doubles (FP32 solves use the first halves)
struct LScratch {
    double* base;
    int64_t n;
    __device__ double* vec(int64_t task, int k) const { return base + (task * 5 + k) * n; }
    __device__ double* flat(int64_t i) const { return base + i * n; }  // vector i of the whole scratch
};

// one FP64 step v <- Phi_c(v) in place (v global), using CG vectors x, r, p, q
__device__ __forceinline__ long long step_large64(const KArgs& a, const StepCoef& c, double rtol2, const LCol& col,
                                                  double* __restrict__ v, double* __restrict__ x,
                                                  double* __restrict__ r, double* __restrict__ p,
                                                  double* __restrict__ q, double* red, int& slot)
{
    const Grid2D& g = a.g;
    FOR_ROWS(col, g, y)
    {
        const int64_t i = (int64_t)y * g.nx + col.x;
        x[i] = v[i];
        r[i] = explicit_part(c, v[i]);
    }
    __syncthreads();
    const int its = cg_large<double>(g, c, col, x, r, p, q, red, slot, rtol2, a.maxit, a.fail);
    FOR_ROWS(col, g, y)
    {
        const int64_t i = (int64_t)y * g.nx + col.x;
        v[i] = x[i];
    }
    __syncthreads();
    return its;
}

// FP64 sweep (precision 0) over interval j; the state of the step is the slice just written to u (or y)
__global__ __launch_bounds__(kBlockL) void sweep_large_kernel(KArgs a, LScratch sc)
{
    __shared__ double red[4 * kWavesL];
    int slot = 0;
    const int64_t j = blockIdx.x;
    const Grid2D& g = a.g;
    const LCol col = make_col(g);
    const int64_t n = a.n;
    double* v = sc.vec(j, 4);
    bool same = true;
    FOR_ROWS(col, g, y)
    {
        const int64_t i = (int64_t)y * g.nx + col.x;
        const double c0 = sweep_start(a, j, i);
        same = same && !(c0 != a.u[(j * a.m) * n + i]);
        if (a.mode != 0) a.u[(j * a.m) * n + i] = c0;
        v[i] = c0;
    }
    const int64_t total = (j < a.NT) ? a.m : (a.nt - a.NT * a.m);
    if (a.skip_unchanged && __syncthreads_and(same)) {
        if (a.skip_y_src && j < a.NT) FOR_ROWS(col, g, y)
            {
                const int64_t i = (int64_t)y * g.nx + col.x;
                a.y[(j + 1) * n + i] = a.skip_y_src[(j + 1) * n + i];
            }
        if (threadIdx.x == 0 && total > 0) atomicAdd(&a.hdr->skipped, (unsigned long long)total);
        return;
    }
    __syncthreads();
    long long its = 0;
    for (int64_t t = 1; t <= total; ++t) {
        its += step_large64(a, a.fine, a.rtol2, col, v, sc.vec(j, 0), sc.vec(j, 1), sc.vec(j, 2), sc.vec(j, 3), red,
                            slot);
        double* __restrict__ dst = (t < a.m) ? a.u + (j * a.m + t) * n : a.y + (j + 1) * n;
        const double* __restrict__ vs = v;
        FOR_ROWS(col, g, y)
        {
            const int64_t i = (int64_t)y * g.nx + col.x;
            dst[i] = vs[i];
        }
    }
    count_cg(a, its);
}

// FP32 defect-correction sweep (precision 1): rho = psi(v_{i-1}) - M s_i (FP64), M d = rho by FP32 CG,
// v_i = s_i + d (FP64); starting values as in the on-chip mixed sweep
__global__ __launch_bounds__(kBlockL) void sweep_large_mixed_kernel(KArgs a, LScratch sc)
{
    __shared__ double red[4 * kWavesL];
    int slot = 0;
    const int64_t j = blockIdx.x;
    const Grid2D& g = a.g;
    const LCol col = make_col(g);
    const int64_t n = a.n;
    float* __restrict__ x = reinterpret_cast<float*>(sc.vec(j, 0));
    float* __restrict__ r = reinterpret_cast<float*>(sc.vec(j, 1));
    float* __restrict__ p = reinterpret_cast<float*>(sc.vec(j, 2));
    float* __restrict__ q = reinterpret_cast<float*>(sc.vec(j, 3));
    double* __restrict__ prev = sc.vec(j, 4);
    FOR_ROWS(col, g, y)
    {
        const int64_t i = (int64_t)y * g.nx + col.x;
        const double c0 = sweep_start(a, j, i);
        if (a.mode != 0) a.u[(j * a.m) * n + i] = c0;
        prev[i] = c0;
    }
    __syncthreads();
    const int64_t total = (j < a.NT) ? a.m : (a.nt - a.NT * a.m);
    long long its = 0;
    for (int64_t t = 1; t <= total; ++t) {
        const bool ystep = (t == a.m);
        const double* xo_;
        if (!ystep)
            xo_ = a.u + (j * a.m + t) * n;
        else
            xo_ = (a.mode == 0 ? a.u + ((j + 1) * a.m) * n : (a.mode == 1 ? a.y : a.aux) + (j + 1) * n);
        const double* __restrict__ xo = xo_;
        double* __restrict__ dst = ystep ? a.y + (j + 1) * n : a.u + (j * a.m + t) * n;
        double psi2 = 0.0;
        FOR_ROWS(col, g, y)
        {
            const int64_t i = (int64_t)y * g.nx + col.x;
            const double ps = explicit_part(a.fine, prev[i]);
            psi2 += ps * ps;
            const double rho = ps - stencil_g(g, a.fine, col, xo, y);
            r[i] = (float)rho;
            x[i] = 0.0f;
        }
        psi2 = block_sum1(psi2, red, slot, kWavesL);  // its barrier also orders the stores above
        its += cg_large<float>(g, a.fine, col, x, r, p, q, red, slot, a.rtol2_mixed, a.maxit, a.fail,
                               defect_floor2(a.fine) * psi2);
        FOR_ROWS(col, g, y)
        {
            const int64_t i = (int64_t)y * g.nx + col.x;
            const double vnew = xo[i] + (double)x[i];
            prev[i] = vnew;
            dst[i] = vnew;
        }
        __syncthreads();
    }
    count_cg(a, its);
}

// C[M x N] = A[M x K] B[K x N] (row-major, leading dimensions lda, ldb, ldc) by the whole workgroup
// on v_mfma_f64_16x16x4f64 (lane l holds A[l%16][l/16] and B[l/16][l%16]; result item t of lane l is
// C[4t + l/16][l%16]).  Each wave takes 32 x 32 blocks of C (2 x 2 tiles) in turn; the k loop reads
// four k-steps of fragments before their products.  Entries beyond M, N, K read as zero and are not
// written; C[i][j] is stored as epi(i, j, value).  AT: A is passed as its transpose [K x M] (leading
// dimension lda), so that a fragment reads 16 consecutive entries of a row.
template <bool AT = false, typename F>
__device__ __forceinline__ void gemm_f64(const double* __restrict__ A, int lda, const double* __restrict__ B,
                                         int ldb, double* __restrict__ C, int ldc, int M, int N, int K, F&& epi)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int bm = (M + 31) / 32, bn = (N + 31) / 32;
    for (int blk = wave; blk < bm * bn; blk += kWavesL) {
        const int i0 = (blk / bn) * 32, j0 = (blk % bn) * 32;
        f64x4 acc[2][2];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int s = 0; s < 2; ++s) acc[r][s] = f64x4{0.0, 0.0, 0.0, 0.0};
        const int ia = i0 + li, ib = i0 + 16 + li, ja = j0 + li, jb = j0 + 16 + li;
        for (int k0 = 0; k0 < K; k0 += 16) {
            double fa[4][2], fb[4][2];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + 4 * q + lk;
                const bool kin = k < K;
                fa[q][0] = (kin && ia < M) ? (AT ? A[(int64_t)k * lda + ia] : A[(int64_t)ia * lda + k]) : 0.0;
                fa[q][1] = (kin && ib < M) ? (AT ? A[(int64_t)k * lda + ib] : A[(int64_t)ib * lda + k]) : 0.0;
                fb[q][0] = (kin && ja < N) ? B[(int64_t)k * ldb + ja] : 0.0;
                fb[q][1] = (kin && jb < N) ? B[(int64_t)k * ldb + jb] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 2; ++r)
#pragma unroll
                    for (int s = 0; s < 2; ++s)
                        acc[r][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[q][r], fb[q][s], acc[r][s], 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int i = i0 + 16 * r + 4 * t + lk, j = j0 + 16 * s + li;
                    if (i < M && j < N) C[(int64_t)i * ldc + j] = epi(i, j, acc[r][s][t]);
                }
    }
}

// The same product for M and K multiples of 64 and N = 64 NT (NT <= 4), MFMA-bound: 64-row blocks of
// C, each computed by 16 waves (wave w: the 16 rows 16 (w / 4) .. of the block and the N / 4 columns
// (w % 4) N / 4 .., NT tiles of 16 x 16), over k-chunks of 16 whose A block and B rows ([k][col], pitch
// kBP) are staged in LDS, two buffers: the next chunk's loads are in flight while the current chunk's
// MFMAs run.  The A block is kept as the global A is read -- [k][row] (pitch kAPT) when A is given
// transposed, [row][k] (pitch kAPN) otherwise -- so that its stores take consecutive addresses.  The
// pitches put the 32 lanes of a fragment read (16 consecutive entries at k and 16 at k + 1) on distinct
// banks of the 64-bank LDS: 16 mod 32 doubles for the [k][..] layouts, 2 mod 32 for [row][k].  The k
// order of every output's sum is that of gemm_f64.
// CB / CC: B is read, C written, through device-coherent accesses (data shared by a pair).  STORE
// false: C is not written (the epilogue consumes the products).
constexpr int kKC = 16;
constexpr int kAPT = 64 + 16;
constexpr int kAPN = kKC + 2;
constexpr int kBP = 256 + 16;
constexpr int kABuf = kKC * kAPT > 64 * kAPN ? kKC * kAPT : 64 * kAPN;  // doubles of the A block
constexpr int kGemmBuf = kABuf + kKC * kBP;                             // doubles of one buffer
constexpr int kGemmLds = 2 * kGemmBuf;
template <int NT, bool AT = false, bool CB = false, bool CC = false, bool STORE = true, typename F>
__device__ __forceinline__ void gemm_f64_tiled(const double* __restrict__ A, int lda, const double* __restrict__ B,
                                               int ldb, double* __restrict__ C, int ldc, int M, int K, double* lds,
                                               F&& epi)
{
    constexpr int N = 64 * NT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int rt = wave >> 2, cg = wave & 3;
    const int nkc = K / kKC;
    for (int i0 = 0; i0 < M; i0 += 64) {
        f64x4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
        double ra, rb[NT];
        // element of the A block and of the B rows this thread moves: A (k, row), B (k, col)
        const int ak = AT ? (tid >> 6) : (tid & 15), ar = AT ? (tid & 63) : (tid >> 4);
        auto load = [&](int k0) {
            ra = AT ? A[(int64_t)(k0 + ak) * lda + i0 + ar] : A[(int64_t)(i0 + ar) * lda + k0 + ak];
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                const int e = tid + q * kBlockL;
                const int64_t o = (int64_t)(k0 + e / N) * ldb + e % N;
                rb[q] = CB ? pair::get(B + o) : B[o];
            }
        };
        auto stage = [&](int buf) {
            double* As = lds + buf * kGemmBuf;
            double* Bs = As + kABuf;
            As[AT ? ak * kAPT + ar : ar * kAPN + ak] = ra;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                const int e = tid + q * kBlockL;
                Bs[(e / N) * kBP + e % N] = rb[q];
            }
        };
        load(0);
        stage(0);
        __syncthreads();
        for (int kc = 0; kc < nkc; ++kc) {
            const int buf = kc & 1;
            if (kc + 1 < nkc) load((kc + 1) * kKC);
            const double* As = lds + buf * kGemmBuf;
            const double* Bs = As + kABuf;
#pragma unroll
            for (int q = 0; q < kKC / 4; ++q) {
                const int k = 4 * q + lk;
                const double fa = AT ? As[k * kAPT + rt * 16 + li] : As[(rt * 16 + li) * kAPN + k];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const double fb = Bs[k * kBP + cg * (N / 4) + t * 16 + li];
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, fb, acc[t], 0, 0, 0);
                }
            }
            if (kc + 1 < nkc) stage(buf ^ 1);
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + rt * 16 + 4 * u + lk, j = cg * (N / 4) + t * 16 + li;
                const double v = epi(i, j, acc[t][u]);
                if constexpr (!STORE)
                    (void)v;
                else if constexpr (CC)
                    pair::put(C + (int64_t)i * ldc + j, v);
                else
                    C[(int64_t)i * ldc + j] = v;
            }
    }
}

// C = A B: the tiled product with NT column tiles per wave (N = 64 NT), or gemm_f64 for NT = 0
template <int NT, bool AT = false, typename F>
__device__ __forceinline__ void gemm_f64_any(const double* __restrict__ A, int lda, const double* __restrict__ B,
                                             int ldb, double* __restrict__ C, int ldc, int M, int N, int K, double* lds,
                                             F&& epi)
{
    if constexpr (NT > 0)
        gemm_f64_tiled<NT, AT>(A, lda, B, ldb, C, ldc, M, K, lds, epi);
    else
        gemm_f64<AT>(A, lda, B, ldb, C, ldc, M, N, K, epi);
}

// the tiled products' column tiles per wave for an nx x ny grid (0: they do not apply)
inline int spectral_nt(int nx, int ny)
{
    if (ny % 64 || nx % 64 || nx > 256) return 0;
    return nx / 64 >= 2 ? nx / 64 : 0;
}

// one Psi substep w <- M^-1 psi(w) (coarse coefficients) by the eigenbasis solve; t0, t1 scratch; lds
// (kGemmLds doubles) for the tiled products (NT > 0)
template <int NT>
__device__ __forceinline__ void spectral_step(const KArgs& a, const LCol& col, double* __restrict__ w,
                                              double* __restrict__ t0, double* __restrict__ t1, double* lds)
{
    const Grid2D& g = a.g;
    const SpecTables T = spec_tables(a);
    const int nx = g.nx, ny = g.ny;
    auto same = [](int, int, double v) { return v; };
    FOR_ROWS(col, g, y)
    {
        const int64_t i = (int64_t)y * nx + col.x;
        t0[i] = explicit_part(a.coarse, w[i]);
    }
    __syncthreads();
    gemm_f64_any<NT, true>(T.qy, ny, t0, nx, t1, nx, ny, nx, ny, lds, same);  // Qy^T b (read through Qy)
    __syncthreads();
    const double cx2 = 2.0 * a.coarse.cx, cy2 = 2.0 * a.coarse.cy;
    gemm_f64_any<NT>(t1, nx, T.qx, nx, t0, nx, ny, nx, nx, lds,           // (.. Qx) ./ mu
                 [&](int i, int j, double v) { return v / (1.0 + (cx2 * T.ex[j] + cy2 * T.ey[i])); });
    __syncthreads();
    gemm_f64_any<NT, true>(T.qyt, ny, t0, nx, t1, nx, ny, nx, ny, lds, same); // Qy .. (read through Qy^T)
    __syncthreads();
    gemm_f64_any<NT>(t1, nx, T.qxt, nx, w, nx, ny, nx, nx, lds, same);    // .. Qx^T
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ long long psi_large(const KArgs& a, const LCol& col, double* w, const LScratch& sc,
                                               int64_t task, double* red, int& slot, double* lds)
{
    long long its = 0;
    for (int q = 0; q < a.substeps; ++q) {
        if (NT > 0 || a.spectral)
            spectral_step<NT>(a, col, w, sc.vec(task, 0), sc.vec(task, 1), lds);
        else if constexpr (NT == 0)
            its += step_large64(a, a.coarse, a.rtol2_coarse, col, w, sc.vec(task, 0), sc.vec(task, 1),
                                sc.vec(task, 2), sc.vec(task, 3), red, slot);
    }
    return its;
}

// window p (linear or FAS form), FP64; NT > 0: Psi in the eigenbasis by the tiled products
template <int NT>
__global__ __launch_bounds__(kBlockL) void coarse_large_kernel(KArgs a, LScratch sc)
{
    __shared__ double red[4 * kWavesL];
    __shared__ double gl[NT > 0 ? kGemmLds : 1];
    int slot = 0;
    const int64_t p = blockIdx.x;
    const int64_t s0 = p - a.k + 1 > 0 ? p - a.k + 1 : 0;
    const Grid2D& g = a.g;
    const LCol col = make_col(g);
    const int64_t n = a.n;
    double* __restrict__ w = sc.vec(p, 4);
    FOR_ROWS(col, g, y)
    {
        const int64_t i = (int64_t)y * g.nx + col.x;
        const double r = cpoint_residual(a, s0, i);
        w[i] = a.fas ? a.u[(s0 * a.m) * n + i] + r : r;
    }
    __syncthreads();
    long long its = 0;
    for (int64_t jj = s0 + 1; jj <= p; ++jj) {
        its += psi_large<NT>(a, col, w, sc, p, red, slot, gl);
        FOR_ROWS(col, g, y)
        {
            const int64_t i = (int64_t)y * g.nx + col.x;
            w[i] = w[i] + (a.fas ? a.tau[jj * n + i] : cpoint_residual(a, jj, i));
        }
        __syncthreads();
    }
    FOR_ROWS(col, g, y)
    {
        const int64_t i = (int64_t)y * g.nx + col.x;
        a.e[p * n + i] = a.fas ? w[i] - a.u[(p * a.m) * n + i] : w[i];
    }
    count_cg(a, its);
}

// tau_j = (v_j - Psi(v_{j-1})) + r_j, one workgroup per j = 1..N_T
template <int NT>
__global__ __launch_bounds__(kBlockL) void tau_large_kernel(KArgs a, LScratch sc)
{
    __shared__ double red[4 * kWavesL];
    __shared__ double gl[NT > 0 ? kGemmLds : 1];
    int slot = 0;
    const int64_t j = blockIdx.x + 1;
    const Grid2D& g = a.g;
    const LCol col = make_col(g);
    const int64_t n = a.n;
    double* w = sc.vec(j, 4);
    FOR_ROWS(col, g, y)
    {
        const int64_t i = (int64_t)y * g.nx + col.x;
        w[i] = a.u[((j - 1) * a.m) * n + i];
    }
    __syncthreads();
    const long long its = psi_large<NT>(a, col, w, sc, j, red, slot, gl);
    FOR_ROWS(col, g, y)
    {
        const int64_t i = (int64_t)y * g.nx + col.x;
        const double vj = a.u[(j * a.m) * n + i];
        a.tau[j * n + i] = (vj - w[i]) + cpoint_residual(a, j, i);
    }
    count_cg(a, its);
}

// ---------------------------------------------------------------------------
// Windows and FAS right-hand sides on two CUs each (eigenbasis Psi, tiled products)
// ---------------------------------------------------------------------------
// One window's state (256 x 256 FP64, 512 KB) lives in global memory anyway, so splitting a window
// over two workgroups costs only their meetings: each half computes the rows r0 .. r0 + ny/2 of
// every product of the eigenbasis solve.  Of the four products, the two that apply Qy^T or Qy need
// every row of their right operand, the other two only the half's own rows, so a Psi substep has
// two meetings: after the explicit part is formed and after the scaled forward transform.  The
// operands written by one half and read by the other go through device-coherent stores and loads;
// a half raises its counter after its stores have completed and waits (bounded) for its partner's.
// The k order of every sum is that of the one-workgroup kernels, so the results are identical.

struct WinPair {
    unsigned* epoch;  // [pairs][2] meeting counters, zero before the launch
    int pairs;        // workgroup pairs in the grid (a multiple of 8)
    int spin_cap;     // polls of the partner's counter before giving up
};

// meeting k of the two halves; false (every thread) if the partner did not arrive within the cap
__device__ __forceinline__ bool pair_meet(const WinPair& wp, int pr, int half, unsigned k, int* ok)
{
    pair::drain();
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_store(wp.epoch + 2 * pr + half, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int seen = 0;
        for (int spin = 0; spin < wp.spin_cap && !seen; ++spin)
            seen = __hip_atomic_load(wp.epoch + 2 * pr + (half ^ 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= k;
        *ok = seen;
    }
    __syncthreads();
    return *ok != 0;
}

// one Psi substep w <- M^-1 psi(w) on the rows r0 .. r0 + rows of w; t0, t2 shared by the pair, t1
// private rows; false if a meeting failed
template <int NT>
__device__ __forceinline__ bool spectral_step_pair(const KArgs& a, const SpecTables& T, double* __restrict__ w,
                                                   double* __restrict__ t0, double* __restrict__ t1,
                                                   double* __restrict__ t2, double* lds, int r0, int rows,
                                                   const WinPair& wp, int pr, int half, unsigned& k, int* ok)
{
    const int nx = a.g.nx, ny = a.g.ny;
    const int64_t o = (int64_t)r0 * nx;
    auto same = [](int, int, double v) { return v; };
    for (int e = threadIdx.x; e < rows * nx; e += kBlockL) pair::put(t0 + o + e, explicit_part(a.coarse, w[o + e]));
    if (!pair_meet(wp, pr, half, ++k, ok)) return false;
    gemm_f64_tiled<NT, true, true>(T.qy + r0, ny, t0, nx, t1 + o, nx, rows, ny, lds, same);  // Qy^T b
    __syncthreads();
    const double cx2 = 2.0 * a.coarse.cx, cy2 = 2.0 * a.coarse.cy;
    gemm_f64_tiled<NT, false, false, true>(t1 + o, nx, T.qx, nx, t2 + o, nx, rows, nx, lds,  // (.. Qx) ./ mu
                                           [&](int i, int j, double v) {
                                               return v / (1.0 + (cx2 * T.ex[j] + cy2 * T.ey[r0 + i]));
                                           });
    if (!pair_meet(wp, pr, half, ++k, ok)) return false;
    gemm_f64_tiled<NT, true, true>(T.qyt + r0, ny, t2, nx, t1 + o, nx, rows, ny, lds, same);  // Qy ..
    __syncthreads();
    gemm_f64_tiled<NT>(t1 + o, nx, T.qxt, nx, w + o, nx, rows, nx, lds, same);  // .. Qx^T
    __syncthreads();
    return true;
}

// The tasks of the paired kernels: windows p = 0 .. N_T (linear or FAS form), or the FAS right-hand
// sides tau_j = (v_j - Psi(v_{j-1})) + r_j, j = 1 .. N_T.
enum PairTask { kWinTask = 0, kTauTask = 1 };

// Pair q takes the tasks q, q + pairs, ... of its kind.
template <int NT, int MODE>
__global__ __launch_bounds__(kBlockL) void coarse_pair_kernel(KArgs a, LScratch sc, WinPair wp)
{
    __shared__ double gl[kGemmLds];
    __shared__ int ok;
    constexpr bool WIN = MODE == kWinTask;
    const int pr = pair::pair_of(blockIdx.x), half = pair::half_of(blockIdx.x);
    const int nx = a.g.nx, rows = a.g.ny / 2, r0 = half * rows;
    const int64_t n = a.n, o = (int64_t)r0 * nx, cnt = (int64_t)rows * nx;
    const SpecTables T = spec_tables(a);
    unsigned k = 0;
    bool alive = true;
    for (int64_t task = (WIN ? 0 : 1) + pr; alive && task <= a.NT; task += wp.pairs) {
        double* __restrict__ w = sc.vec(task, 4);
        double* t0 = sc.vec(task, 0);
        double* t1 = sc.vec(task, 1);
        double* t2 = sc.vec(task, 2);
        const int64_t s0 = !WIN ? task - 1 : (task - a.k + 1 > 0 ? task - a.k + 1 : 0);
        for (int64_t e = threadIdx.x; e < cnt; e += kBlockL) {
            const int64_t i = o + e;
            if (!WIN)
                w[i] = a.u[(s0 * a.m) * n + i];
            else {
                const double r = cpoint_residual(a, s0, i);
                w[i] = a.fas ? a.u[(s0 * a.m) * n + i] + r : r;
            }
        }
        __syncthreads();
        for (int64_t jj = s0 + 1; alive && jj <= task; ++jj) {
            for (int q = 0; alive && q < a.substeps; ++q)
                alive = spectral_step_pair<NT>(a, T, w, t0, t1, t2, gl, r0, rows, wp, pr, half, k, &ok);
            if (!alive || !WIN) break;
            for (int64_t e = threadIdx.x; e < cnt; e += kBlockL) {
                const int64_t i = o + e;
                w[i] = w[i] + (a.fas ? a.tau[jj * n + i] : cpoint_residual(a, jj, i));
            }
            __syncthreads();
        }
        if (!alive) break;
        for (int64_t e = threadIdx.x; e < cnt; e += kBlockL) {
            const int64_t i = o + e;
            if (MODE == kTauTask)
                a.tau[task * n + i] = (a.u[(task * a.m) * n + i] - w[i]) + cpoint_residual(a, task, i);
            else
                a.e[task * n + i] = a.fas ? w[i] - a.u[(task * a.m) * n + i] : w[i];
        }
        __syncthreads();
    }
    if (!alive && threadIdx.x == 0) atomicOr(a.fail, kFailPairTimeout);
}

// ---------------------------------------------------------------------------
// The paired windows with Psi's eigenbasis solve on the BF16 matrix cores (coarse_solver 2)
// ---------------------------------------------------------------------------
// A window carries e (the correction; FAS form: e = w - v) in FP32 in its global scratch (the products
// are accurate to about 1e-5 of e, FP32 keeps 6e-8).  Every substep forms its explicit part in FP64 --
// the FAS form the difference of the explicit parts at v + e and at v, e + react (e - e (3 v^2 + 3 v e
// + e^2)), so that the products' error scales with e and vanishes with it -- splits it into BF16 planes
// hi + lo and applies M^-1 by the four products of the eigenbasis solve, each taken as hi*hi + hi*lo +
// lo*hi on v_mfma_f32_16x16x32_bf16 with FP32 sums (about 16 significant bits per operand: Psi to
// about 1e-5 relative, which changes the two-level convergence rate and never the fixed point).  v
// passes through Psi's substeps as well:
// v^(0) = v_{j-1} is the C-point, v^(1 .. s-1) its trajectory through Psi's substeps, computed once per
// coarse solve by the same kernel (TRAJ) with the same products and stored in FP32 (v enters only the
// explicit parts' difference, multiplied by e, so its own 1e-5 does not reach the fixed point).
//
// Every product is OutT[j][i] = sum_k A[i][k] BT[j][k] with A [M][K] and BT [N][K] stored
// k-contiguous (BF16 hi and lo planes), so that each lane reads 8 consecutive k of a fragment and
// writes 4 consecutive entries of an OutT row, which is the layout the next product reads:
//   t1[i][x]  = sum_y  bT[x][y]  QyT[r0+i][y]        Qy^T b        (M = nx, N = rows, K = ny)
//   t2T[x][i] = sum_x' t1[i][x'] QxT[x][x'] / mu     (.. Qx) ./ mu (M = rows, N = nx, K = nx)
//   t1[i][x]  = sum_y  t2T[x][y] Qy[r0+i][y]         Qy ..         (M = nx, N = rows, K = ny)
//   e[i][x]   = sum_x' Qx[x][x'] t1[i][x']           .. Qx^T       (M = nx, N = rows, K = nx)
// with i the half's rows r0 + i.  bT and t2T are shared by the pair (device-coherent 8-byte stores
// and loads, a meeting after each is complete), t1 is the half's own.

constexpr int kBfKC = 32;                      // k per chunk: one MFMA
constexpr int kBfPitch = kBfKC + 8;            // BF16 per LDS row of a chunk (80 bytes)
constexpr int kBfRowsMax = 384;                // A rows + BT rows of the largest product (256 + 128)
constexpr int kBfBuf = kBfRowsMax * 2 * kBfPitch;  // BF16 of one chunk buffer, both planes
constexpr int kBfTP = 128 + 8;                 // BF16 pitch of the explicit part's transpose tile

struct BfOp {
    const __bf16* hi;
    const __bf16* lo;
    int ld;  // leading dimension (BF16)
};

__device__ __forceinline__ uint64_t get64(const __bf16* p)
{
    return __hip_atomic_load(reinterpret_cast<uint64_t*>(const_cast<__bf16*>(p)), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// Loads at a uniform global base plus a 32-bit byte offset (one scalar pair and one vector register,
// global rather than generic addressing)
typedef __attribute__((address_space(1))) const char gbyte;
__device__ __forceinline__ uint64_t gget64(const __bf16* base, uint32_t off)
{
    return __hip_atomic_load((__attribute__((address_space(1))) uint64_t*)((gbyte*)base + off), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4_t gload16(const __bf16* base, uint32_t off)
{
    return *(__attribute__((address_space(1))) const u32x4_t*)((gbyte*)base + off);
}
__device__ __forceinline__ void put64(__bf16* p, uint64_t v)
{
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// four FP32 values as BF16 hi and lo parts, packed 4 x 16 bits
__device__ __forceinline__ void split4(const f32x4_t& v, uint64_t& hi, uint64_t& lo)
{
    bf16x4_t h, l;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const __bf16 b = (__bf16)v[r];
        h[r] = b;
        l[r] = (__bf16)(v[r] - (float)b);
    }
    hi = __builtin_bit_cast(uint64_t, h);
    lo = __builtin_bit_cast(uint64_t, l);
}

// OutT[j][i] = out(i, j, sum_k A[i][k] BT[j][k]) (out receives four consecutive i from i) for M = 64 TM,
// N = 64 TN, K a multiple of 32.  16 waves in a 4 x 4 grid, wave (wm, wn) owning rows 16 TM wm .. and
// columns 16 TN wn .. (TM x TN tiles of 16 x 16).  Per k-chunk of 32 the A rows and BT rows of both
// planes are staged in LDS (two buffers: the next chunk's global loads are in flight while the
// current chunk's MFMAs run); the 80-byte row pitch puts the 16-byte fragment reads of 16
// consecutive rows on distinct banks.  ACOH: A is read through device-coherent loads.
template <int TM, int TN, bool ACOH, typename O>
__device__ __forceinline__ void bf_gemm(const BfOp A, const BfOp B, int K, __bf16* lds, O&& out)
{
    constexpr int M = 64 * TM, N = 64 * TN, R = M + N;
    static_assert(R <= kBfRowsMax, "chunk buffer too small");
    static_assert(M % 16 == 0, "a wave's rows within one operand");
    // A chunk is loaded in wave pieces of 16 rows x 4 16-byte segments of one plane (planes outermost):
    // the operand and plane of a piece are alike on its wave, so its base address is scalar and a
    // lane's address is that base plus a 32-bit offset.
    constexpr int WP = R / 16 * 2;  // wave pieces of a chunk
    constexpr int PER = (WP + kWavesL - 1) / kWavesL;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int wm = wave >> 2, wn = wave & 3;
    uint64_t ld0[PER], ld1[PER];
    // each piece's base (scalar, chosen once) and the lane's offset in it at k = 0
    const __bf16* pbase[PER];
    uint32_t poff[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int wp = q * kWavesL + wave;
        const int plane = wp / (R / 16), rb = wp % (R / 16);
        const bool isa = rb * 16 < M;
        const __bf16* b = isa ? (plane ? A.lo : A.hi) : (plane ? B.lo : B.hi);
        const uint64_t bb = reinterpret_cast<uint64_t>(b);
        const uint32_t blo = __builtin_amdgcn_readfirstlane((uint32_t)bb), bhi = __builtin_amdgcn_readfirstlane((uint32_t)(bb >> 32));
        pbase[q] = reinterpret_cast<const __bf16*>(((uint64_t)bhi << 32) | blo);
        const int ld = isa ? A.ld : B.ld;
        const int r = (isa ? rb * 16 : rb * 16 - M) + (lane >> 2);
        poff[q] = (uint32_t)(r * ld + 8 * (lane & 3)) * 2u;
    }
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int wp = q * kWavesL + wave;
            if (wp < WP) {
                const bool isa = wp % (R / 16) * 16 < M;
                const uint32_t off = poff[q] + (uint32_t)k0 * 2u;
                if (ACOH && isa) {
                    ld0[q] = gget64(pbase[q], off);
                    ld1[q] = gget64(pbase[q], off + 8u);
                } else {
                    const u32x4_t v = gload16(pbase[q], off);
                    ld0[q] = (uint64_t)v.x | ((uint64_t)v.y << 32);
                    ld1[q] = (uint64_t)v.z | ((uint64_t)v.w << 32);
                }
            }
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int wp = q * kWavesL + wave;
            if (wp < WP) {
                const int plane = wp / (R / 16), row = wp % (R / 16) * 16 + (lane >> 2), seg = lane & 3;
                uint4 v;
                v.x = (uint32_t)ld0[q];
                v.y = (uint32_t)(ld0[q] >> 32);
                v.z = (uint32_t)ld1[q];
                v.w = (uint32_t)(ld1[q] >> 32);
                *reinterpret_cast<uint4*>(lds + buf * kBfBuf + (plane * R + row) * kBfPitch + 8 * seg) = v;
            }
        }
    };
    f32x4_t acc[TM][TN];
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const int nk = K / kBfKC;
    load(0);
    stage(0);
    __syncthreads();
#pragma unroll 1
    for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nk) load((kc + 1) * kBfKC);
        const __bf16* Lh = lds + buf * kBfBuf;
        const __bf16* Ll = Lh + R * kBfPitch;
        bf16x8_t bh[TN], bl[TN];
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            const int o = (M + wn * 16 * TN + 16 * tn + li) * kBfPitch + 8 * lk;
            bh[tn] = *reinterpret_cast<const bf16x8_t*>(Lh + o);
            bl[tn] = *reinterpret_cast<const bf16x8_t*>(Ll + o);
        }
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
            const int o = (wm * 16 * TM + 16 * tm + li) * kBfPitch + 8 * lk;
            const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(Lh + o);
            const bf16x8_t al = *reinterpret_cast<const bf16x8_t*>(Ll + o);
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) {
                acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[tn], acc[tm][tn], 0, 0, 0);
                acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[tn], acc[tm][tn], 0, 0, 0);
                acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[tn], acc[tm][tn], 0, 0, 0);
            }
        }
        if (kc + 1 < nk) stage(buf ^ 1);
        __syncthreads();
    }
    // item r of the lane: row 4 lk + r, column li of its tile
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn)
            out(wm * 16 * TM + 16 * tm + 4 * lk, wn * 16 * TN + 16 * tn + li, acc[tm][tn]);
}

// the window's tasks p = q, q + pairs, ... on pair q; nx = 64 NXT, half rows ny / 2 = 64 RT.  TRAJ: the
// tasks j = 1 .. N_T instead: v_{j-1} = u_{(j-1)m} carried through Psi's first s - 1 substeps (the plain
// explicit part, the same products), each substep's result stored in a.traj
template <int NXT, int RT, bool TRAJ = false>
__global__ __launch_bounds__(kBlockL) void coarse_pair_bf_kernel(KArgs a, LScratch sc, WinPair wp)
{
    __shared__ __align__(16) __bf16 lds[2 * kBfBuf];
    __shared__ int ok;
    constexpr int NX = 64 * NXT, ROWS = 64 * RT, NY = 2 * ROWS;
    const int pr = pair::pair_of(blockIdx.x), half = pair::half_of(blockIdx.x);
    const int r0 = half * ROWS;
    const int64_t n = a.n, o = (int64_t)r0 * NX, cnt = (int64_t)ROWS * NX;
    const int tid = threadIdx.x;
    const SpecTables T = spec_tables(a);
    // the eigenvalue factors of the two directions as FP32, in LDS for the products' epilogue (read
    // there once per output tile, where global loads would each wait out a memory latency)
    __shared__ float eig[NX + NY];
    for (int e = tid; e < NX + NY; e += kBlockL) eig[e] = (float)(e < NX ? T.ex[e] : T.ey[e - NX]);
    __syncthreads();
    const BfOp qyt{bf_table(a, 0, 0) + r0 * NY, bf_table(a, 0, 1) + r0 * NY, NY};
    const BfOp qxt{bf_table(a, 1, 0), bf_table(a, 1, 1), NX};
    const BfOp qy{bf_table(a, 2, 0) + r0 * NY, bf_table(a, 2, 1) + r0 * NY, NY};
    const BfOp qx{bf_table(a, 3, 0), bf_table(a, 3, 1), NX};
    const float cx2 = (float)(2.0 * a.coarse.cx), cy2 = (float)(2.0 * a.coarse.cy);
    const double react = a.coarse.react;
    unsigned k = 0;
    bool alive = true;
    for (int64_t task = (TRAJ ? 1 : 0) + pr; alive && task <= a.NT; task += wp.pairs) {
        float* __restrict__ w = reinterpret_cast<float*>(sc.vec(task, 4));
        __bf16* bt = reinterpret_cast<__bf16*>(sc.vec(task, 0));  // bT [NX][NY], hi then lo plane
        __bf16* t1 = reinterpret_cast<__bf16*>(sc.vec(task, 1));  // t1 [NY][NX] (the half's rows)
        __bf16* t2 = reinterpret_cast<__bf16*>(sc.vec(task, 2));  // t2T [NX][NY]
        const BfOp opb{bt, bt + n, NY}, opt2{t2, t2 + n, NY};
        const BfOp opt1{t1 + o, t1 + n + o, NX};
        const int64_t s0 = TRAJ ? task - 1 : (task - a.k + 1 > 0 ? task - a.k + 1 : 0);
        for (int64_t e = tid; e < cnt; e += kBlockL)
            w[o + e] = TRAJ ? (float)a.u[(s0 * a.m) * n + o + e] : (float)cpoint_residual(a, s0, o + e);
        __syncthreads();
        // C[x][i] -> t1[i][x .. x+3] (the half's rows)
        auto to_t1 = [&](int x, int i, f32x4_t v) {
            uint64_t h, l;
            split4(v, h, l);
            *reinterpret_cast<uint64_t*>(t1 + o + (int64_t)i * NX + x) = h;
            *reinterpret_cast<uint64_t*>(t1 + n + o + (int64_t)i * NX + x) = l;
        };
        for (int64_t jj = s0 + 1; alive && jj <= task; ++jj) {
            for (int q = 0; alive && q < (TRAJ ? a.substeps - 1 : a.substeps); ++q) {
                const bool fas = !TRAJ && a.fas != 0;
                const double* v64 = (fas && q == 0) ? a.u + ((jj - 1) * a.m) * n : nullptr;
                const float* v32 = (fas && q > 0) ? a.traj + ((jj - 1) * (a.substeps - 1) + q - 1) * n : nullptr;
                // the explicit part in FP64, split, and transposed through LDS into bT[x][r0 ..], in
                // two passes of 128 columns
                for (int c0 = 0; c0 < NX; c0 += 128) {
                    const int cols = NX - c0 < 128 ? NX - c0 : 128;
                    // ROWS * cols is a multiple of 4 kBlockL: batches of four points per thread, every
                    // load of a batch issued before any is used
                    for (int b0 = tid; b0 < ROWS * cols; b0 += 4 * kBlockL) {
                        double ew[4], vw[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int e = b0 + u * kBlockL, y = e / cols, x = c0 + e % cols;
                            const int64_t i = o + (int64_t)y * NX + x;
                            ew[u] = (double)w[i];
                            vw[u] = v64 ? v64[i] : (v32 ? (double)v32[i] : 0.0);
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int e = b0 + u * kBlockL, y = e / cols, x = e % cols;
                            const double ee = ew[u], vv = vw[u];
                            const double b = fas ? ee + react * (ee - ee * (3.0 * vv * vv + 3.0 * vv * ee + ee * ee))
                                                 : explicit_part(a.coarse, ee);
                            const __bf16 h = (__bf16)b;
                            lds[x * kBfTP + y] = h;
                            lds[(128 + x) * kBfTP + y] = (__bf16)(b - (double)h);
                        }
                    }
                    __syncthreads();
                    for (int e = tid; e < cols * (ROWS / 4) * 2; e += kBlockL) {
                        const int plane = e / (cols * (ROWS / 4)), rest = e % (cols * (ROWS / 4));
                        const int x = rest / (ROWS / 4), y4 = 4 * (rest % (ROWS / 4));
                        const uint64_t val = *reinterpret_cast<const uint64_t*>(lds + (plane * 128 + x) * kBfTP + y4);
                        put64(bt + plane * n + (int64_t)(c0 + x) * NY + r0 + y4, val);
                    }
                    __syncthreads();
                }
                if (!(alive = pair_meet(wp, pr, half, ++k, &ok))) break;
                bf_gemm<NXT, RT, true>(opb, qyt, NY, lds, to_t1);  // Qy^T b
                __syncthreads();
                bf_gemm<RT, NXT, false>(opt1, qxt, NX, lds, [&](int i, int x, f32x4_t c) {  // (.. Qx) ./ mu
                    const float ex = eig[x];
#pragma unroll
                    for (int r = 0; r < 4; ++r) c[r] = c[r] / (1.0f + (cx2 * ex + cy2 * eig[NX + r0 + i + r]));
                    uint64_t h, l;
                    split4(c, h, l);
                    put64(t2 + (int64_t)x * NY + r0 + i, h);
                    put64(t2 + n + (int64_t)x * NY + r0 + i, l);
                });
                if (!(alive = pair_meet(wp, pr, half, ++k, &ok))) break;
                bf_gemm<NXT, RT, true>(opt2, qy, NY, lds, to_t1);  // Qy ..
                __syncthreads();
                bf_gemm<NXT, RT, false>(qx, opt1, NX, lds, [&](int x, int i, f32x4_t c) {  // .. Qx^T
                    *reinterpret_cast<f32x4_t*>(w + o + (int64_t)i * NX + x) = c;
                    if (TRAJ)
                        *reinterpret_cast<f32x4_t*>(a.traj + ((task - 1) * (a.substeps - 1) + q) * n + o +
                                                    (int64_t)i * NX + x) = c;
                });
                __syncthreads();
            }
            if (!alive || TRAJ) break;
            for (int64_t e = tid; e < cnt; e += kBlockL)
                w[o + e] = (float)((double)w[o + e] + cpoint_residual(a, jj, o + e));
            __syncthreads();
        }
        if (!alive) break;
        if (!TRAJ) {
            for (int64_t e = tid; e < cnt; e += kBlockL) a.e[task * n + o + e] = (double)w[o + e];
            __syncthreads();
        }
    }
    if (!alive && tid == 0) atomicOr(a.fail, kFailPairTimeout);
}

__global__ void clear_counters_kernel(unsigned* c, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c[i] = 0u;
}

// sequential stepping in one workgroup
__global__ __launch_bounds__(kBlockL) void seq_large_kernel(KArgs a, LScratch sc)
{
    __shared__ double red[4 * kWavesL];
    int slot = 0;
    const Grid2D& g = a.g;
    const LCol col = make_col(g);
    const int64_t n = a.n;
    double* v = sc.vec(0, 4);
    FOR_ROWS(col, g, y) v[(int64_t)y * g.nx + col.x] = a.u[(int64_t)y * g.nx + col.x];
    __syncthreads();
    long long its = 0;
    for (int64_t t = 1; t <= a.nt; ++t) {
        its += step_large64(a, a.fine, a.rtol2, col, v, sc.vec(0, 0), sc.vec(0, 1), sc.vec(0, 2), sc.vec(0, 3), red,
                            slot);
        FOR_ROWS(col, g, y)
        {
            const int64_t i = (int64_t)y * g.nx + col.x;
            a.u[t * n + i] = v[i];
        }
    }
    count_cg(a, its);
}

// ||M^-1 rho||^2 per interval (the paper-form residual of the exact step), FP64
__global__ __launch_bounds__(kBlockL) void step_residual_large_kernel(KArgs a, LScratch sc)
{
    __shared__ double red[4 * kWavesL];
    int slot = 0;
    const int64_t j = blockIdx.x;
    const Grid2D& g = a.g;
    const LCol col = make_col(g);
    const int64_t n = a.n;
    double* __restrict__ x = sc.vec(j, 0);
    double* __restrict__ r = sc.vec(j, 1);
    const int64_t total = (j < a.NT) ? a.m : (a.nt - a.NT * a.m);
    double acc = 0.0;
    long long its = 0;
    if (a.spectral) {
        // |M^-1 rho|^2 = |(Qy^T rho Qx) ./ mu|^2 (fine coefficients), the sum taken over each
        // thread's entries in a fixed order
        const SpecTables T = spec_tables(a);
        const double cx2 = 2.0 * a.fine.cx, cy2 = 2.0 * a.fine.cy;
        for (int64_t t = 1; t <= total; ++t) {
            const int64_t i0 = j * a.m + t;
            FOR_ROWS(col, g, y)
            {
                const int64_t i = (int64_t)y * g.nx + col.x;
                r[i] = explicit_part(a.fine, a.u[(i0 - 1) * n + i]) - stencil_g(g, a.fine, col, a.u + i0 * n, y);
            }
            __syncthreads();
            gemm_f64<true>(T.qy, g.ny, r, g.nx, x, g.nx, g.ny, g.nx, g.ny, [](int, int, double v) { return v; });
            __syncthreads();
            gemm_f64(x, g.nx, T.qx, g.nx, r, g.nx, g.ny, g.nx, g.nx, [&](int i, int jj, double v) {
                const double c = v / (1.0 + (cx2 * T.ex[jj] + cy2 * T.ey[i]));
                acc += c * c;
                return c;
            });
            __syncthreads();
        }
    }
    for (int64_t t = 1; t <= (a.spectral ? 0 : total); ++t) {
        const int64_t i0 = j * a.m + t;
        FOR_ROWS(col, g, y)
        {
            const int64_t i = (int64_t)y * g.nx + col.x;
            r[i] = explicit_part(a.fine, a.u[(i0 - 1) * n + i]) - stencil_g(g, a.fine, col, a.u + i0 * n, y);
            x[i] = 0.0;
        }
        __syncthreads();
        its += cg_large<double>(g, a.fine, col, x, r, sc.vec(j, 2), sc.vec(j, 3), red, slot, a.rtol2, a.maxit, a.fail);
        FOR_ROWS(col, g, y)
        {
            const int64_t i = (int64_t)y * g.nx + col.x;
            acc += x[i] * x[i];
        }
        __syncthreads();
    }
    double unused = 0.0;
    block_sum2(acc, unused, red, slot, kWavesL);
    if (threadIdx.x == 0) a.partials[j] = acc;
    count_cg(a, its);
}

static LScratch scratch_of(const KArgs& a) { return LScratch{a.large_scratch, a.n}; }

// ||M^-1 rho_i||^2 in the eigenbasis with the tiled products, the fine steps i = 1 .. nt split into
// gridDim.x contiguous runs (one workgroup each, all CUs busy): rho_i = psi(u_{i-1}) - M u_i, then
// |(Qy^T rho Qx) ./ mu|^2 (fine coefficients), each thread summing its entries in a fixed order.
// Two scratch vectors per workgroup.  The square grid's products are taken transposed, X^T = rho^T Qy
// and (X^T)^T Qx, so that the workgroup's own vectors are the left operands, read once per product
// (the right operands, Qy and Qx, are shared by all workgroups and stay in L2); the second product's
// entries are summed, not stored.
template <int NT>
__global__ __launch_bounds__(kBlockL) void step_residual_spec_kernel(KArgs a, LScratch sc)
{
    __shared__ double red[4 * kWavesL];
    __shared__ double gl[kGemmLds];
    int slot = 0;
    const int64_t b = blockIdx.x, nb = gridDim.x;
    const int64_t i_lo = 1 + (a.nt * b) / nb, i_hi = (a.nt * (b + 1)) / nb;  // steps i_lo .. i_hi
    const Grid2D& g = a.g;
    const LCol col = make_col(g);
    const int64_t n = a.n;
    double* __restrict__ r = sc.flat(2 * b);
    double* __restrict__ x = sc.flat(2 * b + 1);
    const SpecTables T = spec_tables(a);
    const double cx2 = 2.0 * a.fine.cx, cy2 = 2.0 * a.fine.cy;
    auto same = [](int, int, double v) { return v; };
    double acc = 0.0;
    for (int64_t i0 = i_lo; i0 <= i_hi; ++i0) {
        FOR_ROWS(col, g, y)
        {
            const int64_t i = (int64_t)y * g.nx + col.x;
            r[i] = explicit_part(a.fine, a.u[(i0 - 1) * n + i]) - stencil_g(g, a.fine, col, a.u + i0 * n, y);
        }
        __syncthreads();
        auto scaled = [&](int i, int jj, double v) {
            const double c = v / (1.0 + (cx2 * T.ex[jj] + cy2 * T.ey[i]));
            acc += c * c;
            return c;
        };
        if (g.nx == g.ny) {
            gemm_f64_tiled<NT, true>(r, g.nx, T.qy, g.ny, x, g.ny, g.nx, g.ny, gl, same);      // x = (Qy^T rho)^T
            __syncthreads();
            gemm_f64_tiled<NT, true, false, false, false>(x, g.ny, T.qx, g.nx, r, g.nx, g.ny, g.nx, gl, scaled);
        } else {
            gemm_f64_tiled<NT, true>(T.qy, g.ny, r, g.nx, x, g.nx, g.ny, g.ny, gl, same);
            __syncthreads();
            gemm_f64_tiled<NT>(x, g.nx, T.qx, g.nx, r, g.nx, g.ny, g.nx, gl, scaled);
        }
        __syncthreads();
    }
    double unused = 0.0;
    block_sum2(acc, unused, red, slot, kWavesL);
    if (threadIdx.x == 0) a.partials[b] = acc;
}

__global__ __launch_bounds__(256) void sum_partials_large_kernel(KArgs a, int64_t count)
{
    __shared__ double red[2 * 2 * 4];
    int slot = 0;
    double acc = 0.0, unused = 0.0;
    for (int64_t b = threadIdx.x; b < count; b += 256) acc += a.partials[b];
    block_sum2(acc, unused, red, slot, 4);
    if (threadIdx.x == 0) {
        a.hdr->norm2 = acc;
        publish_header(a);
    }
}

hipError_t launch_sweep_large(const KArgs& a, int64_t n_tasks, bool mixed, hipStream_t s)
{
    if (mixed) {
        const int pairs = a.large_scratch ? sweep_pair_pairs(a, n_tasks) : 0;
        if (pairs > 0) return launch_sweep_pair(a, pairs, s);
    }
    if (mixed)
        hipLaunchKernelGGL(sweep_large_mixed_kernel, dim3(n_tasks), dim3(kBlockL), 0, s, a, scratch_of(a));
    else
        hipLaunchKernelGGL(sweep_large_kernel, dim3(n_tasks), dim3(kBlockL), 0, s, a, scratch_of(a));
    return hipGetLastError();
}

// the paired window kernels of an nx x ny grid with NT-tile products, and the pairs to launch (0: the
// one-workgroup kernels take the grid).  pre: the kernel that runs before the windows (FP64 FAS
// right-hand sides, or the trajectory of v for the BF16 windows; null when none is needed).
struct CoarsePair {
    const void* pre;
    const void* win;
    int pairs;
};

template <int NT, bool TRAJ = false>
static const void* bf_window_kernel(int rt)
{
    if (rt == 1) return (const void*)coarse_pair_bf_kernel<NT, 1, TRAJ>;
    if (rt == 2) return (const void*)coarse_pair_bf_kernel<NT, 2, TRAJ>;
    return nullptr;
}

static CoarsePair coarse_pair(const KArgs& a)
{
    CoarsePair cp{nullptr, nullptr, 0};
    const int nt = a.spectral ? spectral_nt(a.g.nx, a.g.ny) : 0;
    if (a.g.ny % 128) return cp;  // halves of whole 64-row blocks
    if (a.spectral == 2) {
        // nx of 128, 192 or 256 points, halves of 64 or 128 rows
        const int rt = a.g.ny / 128;
        if (nt == 4) cp.win = bf_window_kernel<4>(rt);
        if (nt == 3) cp.win = bf_window_kernel<3>(rt);
        if (nt == 2) cp.win = bf_window_kernel<2>(rt);
        if (a.fas && a.substeps > 1) {
            if (nt == 4) cp.pre = bf_window_kernel<4, true>(rt);
            if (nt == 3) cp.pre = bf_window_kernel<3, true>(rt);
            if (nt == 2) cp.pre = bf_window_kernel<2, true>(rt);
        }
    } else {
        if (nt == 4) cp = {(const void*)coarse_pair_kernel<4, kTauTask>, (const void*)coarse_pair_kernel<4, kWinTask>, 0};
        if (nt == 3) cp = {(const void*)coarse_pair_kernel<3, kTauTask>, (const void*)coarse_pair_kernel<3, kWinTask>, 0};
        if (nt == 2) cp = {(const void*)coarse_pair_kernel<2, kTauTask>, (const void*)coarse_pair_kernel<2, kWinTask>, 0};
        if (!a.fas) cp.pre = nullptr;
    }
    if (!cp.win) return cp;
    int resident = resident_blocks(cp.win, kBlockL);
    if (cp.pre) {
        const int rp = resident_blocks(cp.pre, kBlockL);
        if (rp < resident) resident = rp;
    }
    int pairs = (resident / 2) / 8 * 8;
    const int64_t want = (a.NT + 1 + 7) / 8 * 8;
    if (pairs > want) pairs = (int)want;
    cp.pairs = pairs >= 8 ? pairs : 0;
    return cp;
}

int coarse_pair_pairs(const KArgs& a) { return coarse_pair(a).pairs; }

hipError_t launch_coarse_large(const KArgs& a, hipStream_t s)
{
    if (a.spectral) launch_spectral_tables(a, s);
    const CoarsePair cp = coarse_pair(a);
    if (a.spectral == 2 && cp.pairs == 0) return hipErrorNotSupported;  // no one-workgroup BF16 form
    if (cp.pairs > 0) {
        // the meeting counters in the fourth vector of task 0, which no paired task uses
        WinPair wp;
        wp.epoch = reinterpret_cast<unsigned*>(a.large_scratch + 3 * a.n);
        wp.pairs = cp.pairs;
        wp.spin_cap = 1 << 21;
        KArgs ka = a;
        LScratch sc = scratch_of(a);
        void* args[] = {&ka, &sc, &wp};
        if (cp.pre && a.NT >= 1) {
            hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(256), 0, s, wp.epoch, 2 * cp.pairs);
            hipError_t e = hipLaunchCooperativeKernel(cp.pre, dim3(2 * cp.pairs), dim3(kBlockL), args, 0, s);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(256), 0, s, wp.epoch, 2 * cp.pairs);
        return hipLaunchCooperativeKernel(cp.win, dim3(2 * cp.pairs), dim3(kBlockL), args, 0, s);
    }
    const int nt = a.spectral ? spectral_nt(a.g.nx, a.g.ny) : 0;
    switch (nt) {
        case 4:
            if (a.fas && a.NT >= 1) hipLaunchKernelGGL(tau_large_kernel<4>, dim3(a.NT), dim3(kBlockL), 0, s, a, scratch_of(a));
            hipLaunchKernelGGL(coarse_large_kernel<4>, dim3(a.NT + 1), dim3(kBlockL), 0, s, a, scratch_of(a));
            break;
        case 3:
            if (a.fas && a.NT >= 1) hipLaunchKernelGGL(tau_large_kernel<3>, dim3(a.NT), dim3(kBlockL), 0, s, a, scratch_of(a));
            hipLaunchKernelGGL(coarse_large_kernel<3>, dim3(a.NT + 1), dim3(kBlockL), 0, s, a, scratch_of(a));
            break;
        case 2:
            if (a.fas && a.NT >= 1) hipLaunchKernelGGL(tau_large_kernel<2>, dim3(a.NT), dim3(kBlockL), 0, s, a, scratch_of(a));
            hipLaunchKernelGGL(coarse_large_kernel<2>, dim3(a.NT + 1), dim3(kBlockL), 0, s, a, scratch_of(a));
            break;
        default:
            if (a.fas && a.NT >= 1) hipLaunchKernelGGL(tau_large_kernel<0>, dim3(a.NT), dim3(kBlockL), 0, s, a, scratch_of(a));
            hipLaunchKernelGGL(coarse_large_kernel<0>, dim3(a.NT + 1), dim3(kBlockL), 0, s, a, scratch_of(a));
    }
    return hipGetLastError();
}

void launch_sequential_large(const KArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(seq_large_kernel, dim3(1), dim3(kBlockL), 0, s, a, scratch_of(a));
}

static int64_t step_residual_large_blocks(const KArgs& a, int64_t n_tasks, const void* fn)
{
    // the eigenbasis form over the whole chip: one round of resident workgroups (a second, partial
    // round would double the time), two scratch vectors and one partial each
    if (!fn) return n_tasks;
    int64_t blocks = 2 * (a.NT + 1) < kResidBlocks ? 2 * (a.NT + 1) : kResidBlocks;  // (N_T + 1) * 5 vectors
    const int64_t resident = resident_blocks(fn, kBlockL);
    if (resident > 0 && blocks > resident) blocks = resident;
    if (blocks > a.nt) blocks = a.nt;
    return blocks > 0 ? blocks : n_tasks;
}

void launch_step_residual_large(const KArgs& a, int64_t n_tasks, hipStream_t s)
{
    if (a.spectral) launch_spectral_tables(a, s);
    const int nt = a.spectral ? spectral_nt(a.g.nx, a.g.ny) : 0;
    const void* fn = nt == 4 ? (const void*)step_residual_spec_kernel<4>
                   : nt == 3 ? (const void*)step_residual_spec_kernel<3>
                   : nt == 2 ? (const void*)step_residual_spec_kernel<2> : nullptr;
    const int64_t blocks = step_residual_large_blocks(a, n_tasks, fn);
    if (nt == 4)
        hipLaunchKernelGGL(step_residual_spec_kernel<4>, dim3(blocks), dim3(kBlockL), 0, s, a, scratch_of(a));
    else if (nt == 3)
        hipLaunchKernelGGL(step_residual_spec_kernel<3>, dim3(blocks), dim3(kBlockL), 0, s, a, scratch_of(a));
    else if (nt == 2)
        hipLaunchKernelGGL(step_residual_spec_kernel<2>, dim3(blocks), dim3(kBlockL), 0, s, a, scratch_of(a));
    else
        hipLaunchKernelGGL(step_residual_large_kernel, dim3(blocks), dim3(kBlockL), 0, s, a, scratch_of(a));
    hipLaunchKernelGGL(sum_partials_large_kernel, dim3(1), dim3(256), 0, s, a, blocks);
}

}  // namespace atm
