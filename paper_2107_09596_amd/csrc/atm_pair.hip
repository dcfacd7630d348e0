// FP32-fine / FP64-residual relaxation sweeps (precision 1) on 2D grids beyond the on-chip strip
// layout, with two CUs per coarse interval.
//
// The CG state of one fine step of a 256 x 256 grid (x, r, p and M p in FP32: 1 MB) does not fit
// on one CU (512 KB of registers, 160 KB of LDS), so each interval is taken by a pair of 512-thread
// workgroups, each owning half of the rows: x, r and M p of its half in registers (a thread holds
// R consecutive rows of one column; on the 256 x 256 grid the last rows of x go to the LDS that p
// leaves free and to a coalesced global buffer), the search direction p of its half in LDS with one
// ghost row above and below.  128 intervals then use all 256 CUs.
//
// The two halves meet once per CG iteration.  After the stencil pass each half publishes, through
// a mailbox in global memory, three partial sums -- (p, M p), (r, M p), (M p, M p) -- and the true
// (r, r) of its current residual, plus its first and last rows of r and its first two and last two
// rows of p.  From these, both halves form the same step lengths (the sums are added in the order
// half 0, half 1), the new residual norm by (r - a q, r - a q) = (r, r) - 2 a (r, q) + a^2 (q, q),
// and each half recomputes its partner's boundary rows of the new p with the same expressions the
// partner evaluates: the ghost rows of the next iteration need no second exchange.  The mathematics
// is plain CG (the iterates of Jacobi-PCG with the constant diagonal); only the grouping of the
// sums and the residual-norm recurrence differ from the one-workgroup solver.
//
// Handshake: the mailbox rows and sums are written with device-coherent stores (they bypass the
// non-coherent caches).  The rows are stored where a pass starts (their values are known then), and
// every thread waits for its stores to complete before the workgroup sums its partials; one wave
// then stores the four sums, which are themselves the signal: the partner polls them with coherent
// loads until none holds the empty mark (a NaN pattern no arithmetic produces), and after taking
// them writes the mark back, freeing the slot for the handshake after next.  Every wait is bounded:
// a half that waits longer than the spin cap sets the header's pair-timeout flag and leaves, and its
// partner then times out too, so the kernel always ends.  The grid is launched cooperatively (every workgroup resident),
// pairs sit on one XCD (blocks b and b ^ 8), and each pair takes intervals pair, pair + pairs, ...
#include "atm_device.hpp"
#include "atm_kernels.hpp"
#include "atm_pairsync.hpp"

namespace atm {
namespace pair {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kParts = 4;  // (p, q), (r, q), (q, q), (r, r)
constexpr int kTimeoutFlag = kFailPairTimeout;

// floats of the boundary packs of one half: first rows (r, p, p of the next row) and last rows (r, p,
// p of the row before), NX each, plus a spare row for the row groups between them, padded to a
// multiple of the workgroup so that every thread copies the same number
constexpr int pack_floats(int nx) { return (7 * nx + kThreads - 1) / kThreads * kThreads; }

struct PairArgs {
    float* mail;      // [2 parities][pairs][2 halves][slot] mailbox, sums marked empty before the launch
    int pairs;        // workgroup pairs in the grid (a multiple of 8)
    int slot;         // floats per mailbox slot: pack_floats(NX), then kParts doubles
    int pack;         // pack_floats(NX): where the sums of a slot start
    int spin_cap;     // polls of the partner's counter before giving up
    float* xg;        // rows of x kept in global memory: [2 x pairs workgroups][x_global_rows][kThreads]
};

// A 32-bit offset hidden from the optimiser, so that the row offsets of the unrolled strip loops are
// recomputed where they are used instead of being hoisted out of the time loop (one register each);
// a load is then a uniform base plus one offset register.
__device__ __forceinline__ uint32_t opq(uint32_t v)
{
    __asm__ volatile("" : "+v"(v));
    return v;
}

// the same for a value alike on every lane, kept in a scalar register
__device__ __forceinline__ uint32_t opqs(uint32_t v)
{
    __asm__ volatile("" : "+s"(v));
    return v;
}

// No instruction; memory accesses are not moved across it by the compiler.  Placed every few rows
// of the unrolled strip passes so that the loads of all rows are not issued at once (they would
// hold one register each).
__device__ __forceinline__ void row_fence() { __asm__ volatile("" ::: "memory"); }

// a value every lane of the wave holds alike, kept in scalar registers
__device__ __forceinline__ float uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// The FP32 step operator at one point: M v = d v - cx (w + e) - cy (up + dn).  Both halves
// evaluate every boundary point through this one expression.
__device__ __forceinline__ float stencil32(float d, float cx, float cy, float up, float cen, float dn, float w, float e)
{
    return d * cen - cx * (w + e) - cy * (up + dn);
}

// one CG update at a point: r' = r - a q, p' = r' + b p
__device__ __forceinline__ void cg_update(float a, float b, float q, float p, float& r, float& pn)
{
    r = r - a * q;
    pn = r + b * p;
}

// Sum kParts doubles over the workgroup (wave sums, then the 16 wave totals in a fixed order).
// Every thread returns the totals.
__device__ __forceinline__ void block_sum4(double (&v)[kParts], double* red, int& slot)
{
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < kParts; ++q) v[q] = wave_sum(v[q]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* base = red + slot * kParts * kWaves;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < kParts; ++q) base[q * kWaves + wave] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kParts; ++q) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += base[q * kWaves + w];
        v[q] = s;
    }
    slot ^= 1;
    __builtin_amdgcn_sched_barrier(0);
}

// The per-launch constants of one half.
template <int NX, int R>
struct Half {
    static constexpr int G = kThreads / NX;  // row groups of a half
    static constexpr int H = G * R;          // rows of a half
    int x, g, half, pair;
    int xw, xe;         // west / east columns (-1: zero boundary)
    int row0;           // first global row of this thread
    bool top_ghost, bot_ghost;  // the ghost row above / below the half comes from the partner
    bool periodic;
};

// v at global row Y (wrapped on the periodic grid, zero beyond a Dirichlet edge), column x
template <int NX, int R>
__device__ __forceinline__ double row_val(const double* v, const Half<NX, R>& h, int Y, int x)
{
    constexpr int ny = 2 * Half<NX, R>::H;
    if (Y < 0 || Y >= ny) {
        if (!h.periodic) return 0.0;
        Y = Y < 0 ? Y + ny : Y - ny;
    }
    return v[opq((uint32_t)Y * NX + x)];
}

// The FP64 part of a step boundary, over the half's points in row order (coalesced, and free of the
// per-thread CG arrays): for each point the value v the next step starts from and the defect of that
// step, rho = psi(v) - M s with s the stored iterate of the step, written as FP32 into the p rows of
// LDS, where the next step's CG takes it as r = p.  v comes from two loads (vin: global index o, LDS
// index li) and a combination that may store (vout).  A thread takes kBatch points at a time and
// issues every load of the batch before the first store, so that a batch costs one memory latency
// (a store may alias the loads of the next batch: v is written over its own input in place).  The
// arithmetic of every point is that of the defect in the one-workgroup solver.
constexpr int kBatch = 8;
// element i of one slice, addressed as a uniform base plus a 32-bit byte offset (one register)
__device__ __forceinline__ const double& at(const double* base, uint32_t i)
{
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + i * 8u);
}
__device__ __forceinline__ double& at(double* base, uint32_t i)
{
    return *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + i * 8u);
}
struct V2 {
    double a, b;
};
template <int NX, int R, typename VIN, typename VOUT>
__device__ __forceinline__ double defect_pass(const StepCoef& c, const Half<NX, R>& h, float* P, const double* __restrict__ s,
                                            VIN&& vin, VOUT&& vout)
{
    constexpr int H = Half<NX, R>::H, PW = NX + 2, NY = 2 * H;
    constexpr int RS = kThreads / NX;  // rows between a thread's points
    static_assert(H % (kBatch * RS) == 0, "whole batches per half");
    const int col = threadIdx.x % NX;
    // the neighbour columns at wrapped (always valid) addresses, zero beyond a Dirichlet edge
    const int cw = col > 0 ? col - 1 : NX - 1, ce = col < NX - 1 ? col + 1 : 0;
    const bool wm = col > 0 || h.periodic, em = col < NX - 1 || h.periodic;
    double psi2 = 0.0;  // this thread's share of |psi(v)|^2
    for (int rb = threadIdx.x / NX; rb < H; rb += kBatch * RS) {
        const int r0 = (int)opq((uint32_t)rb);  // the offsets are formed here, not held across the CG
        V2 in[kBatch];
        double cen[kBatch], up[kBatch], dn[kBatch], w[kBatch], ea[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int row = r0 + b * RS, Y = h.half * H + row;
            const uint32_t o = (uint32_t)Y * NX + col;
            const int yu = Y > 0 ? Y - 1 : NY - 1, yd = Y < NY - 1 ? Y + 1 : 0;
            in[b] = vin(o, (row + 1) * PW + col + 1);
            cen[b] = at(s, o);
            up[b] = at(s, (uint32_t)yu * NX + col);
            dn[b] = at(s, (uint32_t)yd * NX + col);
            w[b] = at(s, (uint32_t)Y * NX + cw);
            ea[b] = at(s, (uint32_t)Y * NX + ce);
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int row = r0 + b * RS, Y = h.half * H + row;
            const uint32_t o = (uint32_t)Y * NX + col;
            const int li = (row + 1) * PW + col + 1;
            const double v = vout(in[b], o, li);
            const double u_ = (Y > 0 || h.periodic) ? up[b] : 0.0, d_ = (Y < NY - 1 || h.periodic) ? dn[b] : 0.0;
            const double w_ = wm ? w[b] : 0.0, e_ = em ? ea[b] : 0.0;
            const double ps = explicit_part(c, v);
            psi2 += ps * ps;
            P[li] = (float)(ps - stencil_value(c, u_, cen[b], d_, w_, e_));
        }
    }
    return psi2;
}

// the partner's mailbox slot of handshake k and the packs in it: first rows (r, p, p of the next
// row), last rows (r, p, p of the row before)
__device__ __forceinline__ const float* partner_slot(const PairArgs& pa, int pair, int half, unsigned k)
{
    return pa.mail + ((size_t)((k & 1) * pa.pairs + pair) * 2 + (half ^ 1)) * pa.slot;
}
__device__ __forceinline__ float* own_slot(const PairArgs& pa, int pair, int half, unsigned k)
{
    return pa.mail + ((size_t)((k & 1) * pa.pairs + pair) * 2 + half) * pa.slot;
}

// the mark of a sum not yet written: a signalling-NaN pattern, which no arithmetic produces
constexpr unsigned long long kEmpty = 0x7FF4DEADBEEF0001ull;
__device__ __forceinline__ bool is_empty(double v) { return __builtin_bit_cast(unsigned long long, v) == kEmpty; }

// Exchange the partial sums and wait for the partner.  The caller has written its mailbox rows.
// Returns false (all threads) if the partner did not arrive within the spin cap.
template <int NX, int R>
__device__ __forceinline__ bool handshake(const PairArgs& pa, const Half<NX, R>& h, unsigned k, double (&tot)[kParts],
                                          double* red, int& slot, double (*parts)[kParts], int* flag)
{
    constexpr int PK = pack_floats(NX);
    drain();  // this thread's pack stores
    block_sum4(tot, red, slot);  // its barrier follows every thread's drain
    // wave 0 publishes and waits, all its lanes alike (same addresses, same values): a branch taken by
    // whole waves, so the rest of the kernel sees no divergent control flow here
    if (__builtin_amdgcn_readfirstlane(threadIdx.x) < 64) {
        double* mine = reinterpret_cast<double*>(own_slot(pa, h.pair, h.half, k) + PK);
        double* theirs = reinterpret_cast<double*>(const_cast<float*>(partner_slot(pa, h.pair, h.half, k)) + PK);
#pragma unroll
        for (int q = 0; q < kParts; ++q) put(mine + q, tot[q]);
        // the decision and the values are taken from one lane, so the wave agrees on them
        int ok = 0;
        double v[kParts];
        for (int spin = 0; spin < pa.spin_cap && !ok; ++spin) {
            ok = 1;
#pragma unroll
            for (int q = 0; q < kParts; ++q) {
                v[q] = uniform(get(theirs + q));
                ok = is_empty(v[q]) ? 0 : ok;
            }
        }
        if (ok) {
#pragma unroll
            for (int q = 0; q < kParts; ++q) {
                parts[h.half][q] = tot[q];
                parts[h.half ^ 1][q] = v[q];
                put(theirs + q, __builtin_bit_cast(double, kEmpty));
            }
        }
        *flag = ok;
    }
    __syncthreads();
    if (!*flag) return false;
#pragma unroll
    for (int q = 0; q < kParts; ++q) tot[q] = parts[0][q] + parts[1][q];
    return true;
}

// Rows of x a thread keeps in LDS rather than registers: the 256 x 256 grid's R = 64 rows of x, r and
// M p fill the registers of a thread; LDS beyond p and the sums holds 14 of them.
constexpr int x_lds_rows(int nx, int r) { return (nx == 256 && r == 64) ? 14 : 0; }
// Rows of x kept in global memory (coalesced, one row of the workgroup's threads after another) on the
// same grid: 16 more, which the update pass loads as one batch half-way through its rows, where the
// compiler would otherwise spill about as many and reload them one at a time.
constexpr int x_global_rows(int nx, int r) { return (nx == 256 && r == 64) ? 16 : 0; }
constexpr int kXgMax = 16;
constexpr int kXgLoadRow = 16;  // the update pass's row before which the batch is issued
constexpr int kStencilBatch = 8;  // rows of the stencil pass whose LDS loads are issued together

template <int NX, int R>
__global__ __launch_bounds__(kThreads) void sweep_pair_mixed_kernel(KArgs a, PairArgs pa)
{
    using HF = Half<NX, R>;
    constexpr int G = HF::G, H = HF::H;
    // p of the half in LDS: local rows 0 .. H+1 (0 and H+1 are the ghost rows from the partner), each
    // of NX + 2 columns (columns 0 and NX+1: zero for Dirichlet, copies of the opposite edge when
    // periodic), so that a thread's stencil reads are constant offsets from one base address
    constexpr int PW = NX + 2;
    // row H+2: writes of the row groups without a ghost row (none when a half has two row groups)
    constexpr int PROWS = G > 2 ? H + 3 : H + 2;
    __shared__ float P[PROWS * PW];
    // the last XL rows of x of every thread, in the LDS that p leaves free (fewer registers to spill)
    constexpr int XL = x_lds_rows(NX, R);
    __shared__ float XS[XL > 0 ? XL * kThreads : 1];
    // rows XR .. R - XL - 1 of x in global memory, rows from R - XL in LDS, the first XR in registers
    constexpr int XG = x_global_rows(NX, R), XR = R - XL - XG;
    static_assert(XG <= kXgMax && (XG == 0 || kXgLoadRow <= XR) && R % 8 == 0, "x rows");
    // (a uniform base and a 32-bit offset formed where it is used: one register per access, not one
    // 64-bit address per row held across the time loop)
    float* const XGb = XG > 0 ? pa.xg + (size_t)blockIdx.x * XG * kThreads : nullptr;
    const uint32_t tid4 = threadIdx.x * 4u;
    auto xg = [&](int j) -> float& {
        return *reinterpret_cast<float*>(reinterpret_cast<char*>(XGb) + (opq((uint32_t)j * (kThreads * 4u)) + tid4));
    };
    __shared__ double red[2 * kParts * kWaves];
    __shared__ double parts[2][kParts];
    __shared__ int flag;
    int slot = 0;

    HF h;
    h.x = threadIdx.x % NX;
    // the row group, alike on every lane of a wave (a wave's 64 threads lie in one row of NX columns),
    // kept in a scalar register with everything that depends on it alone
    static_assert(NX % 64 == 0, "a wave within one row group");
    h.g = (int)__builtin_amdgcn_readfirstlane(threadIdx.x / NX);
    h.half = half_of(blockIdx.x);
    h.pair = pair_of(blockIdx.x);
    h.periodic = a.g.periodic != 0;
    h.xw = h.x > 0 ? h.x - 1 : (h.periodic ? NX - 1 : -1);
    h.xe = h.x < NX - 1 ? h.x + 1 : (h.periodic ? 0 : -1);
    h.row0 = h.half * H + h.g * R;
    h.top_ghost = h.periodic || h.half == 1;
    h.bot_ghost = h.periodic || h.half == 0;
    const int64_t n = a.n;
    const StepCoef& c = a.fine;
    const float d32 = (float)c.d, cx32 = (float)c.cx, cy32 = (float)c.cy;
    const bool first_group = h.g == 0, last_group = h.g == G - 1;
    float* const Pr = P + (h.g * R + 1) * PW + h.x + 1;  // this thread's first row
    // its west and east neighbours through bases of their own, pointing at the wrapped column on the
    // periodic grid and at the zero column 0 at a Dirichlet edge (opaque, so that the two reads of a
    // row are not merged into one paired read, whose short offsets would need a base register per row)
    const float* const Pw = P + opq((uint32_t)((h.g * R + 1) * PW + h.xw + 1));
    const float* const Pe = P + opq((uint32_t)((h.g * R + 1) * PW + (h.xe >= 0 ? h.xe + 1 : 0)));
    // where this thread's ghost-row value goes: above its first row (first group), below its last row
    // (last group), else the spare row H+2; and its pack rows (first group: r, p, p of rows 0 and 1;
    // last group: r, p, p of rows R-1 and R-2; other groups: the spare pack row 6 of the mailbox slot)
    float* const Pg = first_group ? Pr - PW : (last_group ? Pr + R * PW : P + (H + 2) * PW + h.x + 1);
    const int pk0 = first_group ? h.x : (last_group ? 3 * NX + h.x : 6 * NX + h.x);
    const int pk_step = (first_group || last_group) ? NX : 0;
    const int prow_a = last_group ? (R - 1) * PW : 0, prow_b = last_group ? (R - 2) * PW : PW;
    unsigned k = 0;  // handshakes so far
    long long its_total = 0;
    bool alive = true;

    for (int q = threadIdx.x; q < (H + 2) * PW; q += kThreads) P[q] = 0.0f;
    __syncthreads();

    float xv[R], rv[R], qv[R];
    double psi_part = 0.0;  // this thread's share of |psi(v_{t-1})|^2 of the current defect

    for (int64_t j = h.pair; j <= a.NT && alive; j += pa.pairs) {
        const int64_t total = (j < a.NT) ? a.m : (a.nt - a.NT * a.m);
        // the starting value c_j (written to u_{jm} in modes 1 and 2) and the defect of the first step
        // rho_1 = psi(c_j) - M s_1, s_1 the value stored at the first point of the interval (into LDS)
        const double* xo = a.u + (j * a.m + 1) * n;  // s_t of the next step (valid while total >= 1)
        {
            double* uc = a.u + (j * a.m) * n;
            const double* ax = (a.mode != 0 && a.aux) ? a.aux + j * n : nullptr;
            const bool use_aux = a.mode == 1 || (a.mode == 2 && j > 0);
            auto start_in = [&](uint32_t o, int) { return V2{at(uc, o), use_aux ? at(ax, o) : 0.0}; };
            auto start_out = [&](const V2& in, uint32_t o, int) {
                const double c0 = !use_aux ? in.a : (a.mode == 1 ? in.a + in.b : in.b);
                if (a.mode != 0) at(uc, o) = c0;
                return c0;
            };
            if (total >= 1)
                psi_part = defect_pass<NX, R>(c, h, P, xo, start_in, start_out);
            else if (a.mode != 0)
                for (int e = threadIdx.x; e < H * NX; e += kThreads) {
                    const uint32_t o = (uint32_t)(h.half * H) * NX + e;
                    start_out(start_in(o, 0), o, 0);
                }
        }
        __syncthreads();
        for (int64_t t = 1; t <= total && alive; ++t) {
            // ---- FP32 CG for M d = rho from d = 0: x = 0, p = r (rho in the p rows of LDS) ----
            double rr_part = 0.0;  // this thread's share of (r, r) of the current residual
            {
                float chunk = 0.0f;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    if (i < XR)
                        xv[i] = 0.0f;
                    else if (i < R - XL)
                        xg(i - XR) = 0.0f;
                    else
                        XS[(i - (R - XL)) * kThreads + threadIdx.x] = 0.0f;
                    rv[i] = Pr[i * PW];
                    chunk += rv[i] * rv[i];
                    if ((i & 7) == 7 || i == R - 1) {
                        rr_part += (double)chunk;
                        chunk = 0.0f;
                    }
                }
            }
            ++k;
            {
                float* ms = own_slot(pa, h.pair, h.half, k) + pk0;
                const float ra = last_group ? rv[R - 1] : rv[0], rb = last_group ? rv[R - 2] : rv[1];
                put(ms, ra);
                put(ms + pk_step, ra);
                put(ms + 2 * pk_step, rb);
            }
            double tot[kParts] = {psi_part, 0.0, 0.0, rr_part};
            if (!handshake<NX, R>(pa, h, k, tot, red, slot, parts, &flag)) {
                alive = false;
                break;
            }
            {
                // ghost rows of p = r: the partner's last row above, its first row below
                const float* ps = partner_slot(pa, h.pair, h.half, k);
                const bool from_partner = first_group ? h.top_ghost : h.bot_ghost;
                const float v = get(ps + (first_group ? 4 * NX : NX) + h.x);
                *Pg = from_partner ? v : 0.0f;
            }
            __syncthreads();
            const double bb = uniform(tot[3]);
            int it = 0;
            // b = 0 (d = 0 is exact), or a defect at the rounding level of its own FP64 evaluation
            bool converged = !(bb > 0.0) || !(bb > defect_floor2(c) * uniform(tot[0]));
            // The CG runs on the unit right-hand side rho / |rho| (its sums stay clear of FP32's
            // underflow however small the defect) and d = |rho| x.  Both halves scale by the same factor
            // of the pair's total, so the ghost rows (the partner's unscaled r) scale to the partner's
            // own values.
            const double sig = converged ? 1.0 : sqrt(bb);
            const float inv = uniform((float)(1.0 / sig)), sig32 = uniform((float)sig);
            const double thresh = a.rtol2_mixed;
            if (!converged) {
                float chunk = 0.0f;
                rr_part = 0.0;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    rv[i] = rv[i] * inv;
                    Pr[i * PW] = rv[i];
                    chunk += rv[i] * rv[i];
                    if ((i & 7) == 7 || i == R - 1) {
                        rr_part += (double)chunk;
                        chunk = 0.0f;
                    }
                }
                *Pg = *Pg * inv;
                __syncthreads();
            }
            while (!converged && it < a.maxit) {
                // the boundary packs, r and p before the update, stored first (their latency is hidden
                // by the pass)
                {
                    float* ms = own_slot(pa, h.pair, h.half, k + 1) + pk0;
                    put(ms, last_group ? rv[R - 1] : rv[0]);
                    put(ms + pk_step, Pr[prow_a]);
                    put(ms + 2 * pk_step, Pr[prow_b]);
                }
                // pass 1: q = M p and the partial sums
                double sums[kParts] = {0.0, 0.0, 0.0, rr_part};
                {
                    // the rows go PB at a time, every LDS load of the PB rows issued before the first is used
                    constexpr int PB = kStencilBatch;
                    static_assert(R % PB == 0 && 8 % PB == 0, "whole batches");
                    float cpq = 0.0f, crq = 0.0f, cqq = 0.0f;
                    float up = Pr[-PW], cen = Pr[0];
#pragma unroll
                    for (int i0 = 0; i0 < R; i0 += PB) {
                        float dns[PB], ws[PB], es[PB];
#pragma unroll
                        for (int b = 0; b < PB; ++b) {
                            dns[b] = Pr[(i0 + b + 1) * PW];
                            ws[b] = Pw[(i0 + b) * PW];
                            es[b] = Pe[(i0 + b) * PW];
                        }
                        row_fence();
#pragma unroll
                        for (int b = 0; b < PB; ++b) {
                            const int i = i0 + b;
                            const float dn = dns[b];
                            const float q = stencil32(d32, cx32, cy32, up, cen, dn, ws[b], es[b]);
                            qv[i] = q;
                            cpq += cen * q;
                            crq += rv[i] * q;
                            cqq += q * q;
                            if ((i & 7) == 7 || i == R - 1) {
                                sums[0] += (double)cpq;
                                sums[1] += (double)crq;
                                sums[2] += (double)cqq;
                                cpq = crq = cqq = 0.0f;
                            }
                            up = cen;
                            cen = dn;
                        }
                        row_fence();
                    }
                }
                ++k;
                if (!handshake<NX, R>(pa, h, k, sums, red, slot, parts, &flag)) {
                    alive = false;
                    break;
                }
                const double rr = uniform(sums[3]);
                const double alpha = uniform(rr / sums[0]);
                const double rr_new = uniform(rr - 2.0 * alpha * sums[1] + alpha * alpha * sums[2]);
                const double beta = rr_new / rr;
                const float a32 = uniform((float)alpha), b32 = uniform((float)beta);
                // the partner's boundary row next to this thread's group, as the partner computes it:
                // above the first group the partner's last row (its r and p, the row before it, and this
                // half's first row below it), below the last group its first row (this half's last row
                // above it, the row after it below); written to the ghost rows after every thread has
                // formed its q from the old ones.  Its inputs are loaded here, before the update pass, and
                // used after it, which hides their latency; this thread's own boundary value of p is
                // taken before the pass overwrites it.
                const bool top = first_group;
                const float* ps = partner_slot(pa, h.pair, h.half, k) + (top ? 3 * NX : 0);
                const float g_r = get(ps + h.x), g_p0 = get(ps + NX + h.x), g_p1 = get(ps + 2 * NX + h.x);
                // (the west and east columns as 32-bit byte offsets from the uniform slot address, formed
                // here from the thread index rather than held across the loop; wrapped columns, which the
                // Dirichlet edge then ignores)
                const uint32_t xc = opq(threadIdx.x) % NX;
                const uint32_t ow = (NX + (xc > 0 ? xc - 1 : NX - 1)) * 4u, oe = (NX + (xc < NX - 1 ? xc + 1 : 0)) * 4u;
                const float g_wr = get(reinterpret_cast<const float*>(reinterpret_cast<const char*>(ps) + ow));
                const float g_er = get(reinterpret_cast<const float*>(reinterpret_cast<const char*>(ps) + oe));
                const float g_own = Pr[opqs(top ? 0u : (uint32_t)((R - 1) * PW))];
                // pass 2: x += a p, r -= a q, p = r + b p (each thread reads and writes only its own points
                // of p), this thread's share of the new (r, r), and the ghost rows.  The rows go eight at a
                // time, every load of p of the eight issued before the first is used.
                {
                    float crr = 0.0f;
                    rr_part = 0.0;
                    float xgv[XG > 0 ? XG : 1];
#pragma unroll
                    for (int i0 = 0; i0 < R; i0 += 8) {
                        float pcs[8];
#pragma unroll
                        for (int b = 0; b < 8; ++b) pcs[b] = Pr[(i0 + b) * PW];
                        if (XG > 0 && i0 == kXgLoadRow) {
#pragma unroll
                            for (int j = 0; j < XG; ++j) xgv[j] = xg(j);
                        }
                        row_fence();
#pragma unroll
                        for (int b = 0; b < 8; ++b) {
                            const int i = i0 + b;
                            const float pc = pcs[b];
                            if (i < XR)
                                xv[i] = xv[i] + a32 * pc;
                            else if (i < R - XL)
                                xg(i - XR) = xgv[i - XR] + a32 * pc;
                            else {
                                float& xl = XS[(i - (R - XL)) * kThreads + threadIdx.x];
                                xl = xl + a32 * pc;
                            }
                            float pn;
                            cg_update(a32, b32, qv[i], pc, rv[i], pn);
                            Pr[i * PW] = pn;
                            crr += rv[i] * rv[i];
                        }
                        rr_part += (double)crr;
                        crr = 0.0f;
                        row_fence();
                    }
                    const float w = h.xw >= 0 ? g_wr : 0.0f, e = h.xe >= 0 ? g_er : 0.0f;
                    const float q = top ? stencil32(d32, cx32, cy32, g_p1, g_p0, g_own, w, e)
                                        : stencil32(d32, cx32, cy32, g_own, g_p0, g_p1, w, e);
                    float r = g_r, ghost;
                    cg_update(a32, b32, q, g_p0, r, ghost);
                    *Pg = (top ? h.top_ghost : h.bot_ghost) ? ghost : 0.0f;
                }
                __syncthreads();
                ++it;
                converged = !(rr_new > thresh);
            }
            if (!alive) break;
            its_total += it;
            if (!converged) atomicOr(a.fail, 1);
            // ---- v_t = s_t + d in FP64; the defect of the next step ----
            // d goes to the p rows of LDS (p is no longer needed), then a row-order pass forms v_t and
            // the next defect in its place
#pragma unroll
            for (int i = 0; i < R; ++i)
                Pr[i * PW] = sig32 * (i < XR ? xv[i] : (i < R - XL ? xg(i - XR) : XS[(i - (R - XL)) * kThreads + threadIdx.x]));
            __syncthreads();
            const bool ystep = (t == a.m);
            const double* so = xo;
            double* dst = ystep ? a.y + (j + 1) * n : a.u + (j * a.m + t) * n;
            const double* xn = nullptr;
            auto upd_in = [&](uint32_t o, int li) { return V2{at(so, o), (double)P[li]}; };
            auto upd_out = [&](const V2& in, uint32_t o, int) {
                const double v = in.a + in.b;
                at(dst, o) = v;
                return v;
            };
            if (t < total) {
                xn = (t + 1 < a.m) ? a.u + (j * a.m + t + 1) * n
                                   : (a.mode == 0 ? a.u + ((j + 1) * a.m) * n : (a.mode == 1 ? a.y : a.aux) + (j + 1) * n);
                psi_part = defect_pass<NX, R>(c, h, P, xn, upd_in, upd_out);
            } else {
                for (int e = threadIdx.x; e < H * NX; e += kThreads) {
                    const uint32_t o = (uint32_t)(h.half * H) * NX + e;
                    const int li = (e / NX + 1) * PW + e % NX + 1;
                    upd_out(upd_in(o, li), o, li);
                }
            }
            __syncthreads();
            xo = xn;
        }
    }
    if (!alive && threadIdx.x == 0) atomicOr(a.fail, kTimeoutFlag);
    if (h.half == 0) count_cg(a, its_total);
}

// mark every sum of the mailbox empty (the slots of both parities, pairs and halves)
__global__ void reset_mailbox_kernel(PairArgs pa)
{
    const int slots = 2 * pa.pairs * 2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < slots * kParts; i += gridDim.x * blockDim.x) {
        double* sums = reinterpret_cast<double*>(pa.mail + (size_t)(i / kParts) * pa.slot + pa.pack);
        sums[i % kParts] = __builtin_bit_cast(double, kEmpty);
    }
}

}  // namespace pair
}  // namespace atm

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace atm {

namespace {

constexpr int kSpinCap = 1 << 21;  // polls of the partner's counter (about a second) before giving up
constexpr size_t xg_offset_pad = 64;  // floats between the mailbox and the rows of x in global memory

struct PairShape {
    void* fn;  // the kernel instantiation, null when the grid has none
};

// the instantiation for an nx x ny grid: two halves of ny/2 rows, 512 / nx row groups of R rows
PairShape pair_shape(int nx, int ny)
{
    PairShape p{nullptr};
    if (ny % 2) return p;
    const int half = ny / 2;
    if (nx == 256 && half == 128) p.fn = (void*)pair::sweep_pair_mixed_kernel<256, 64>;
    if (nx == 256 && half == 64) p.fn = (void*)pair::sweep_pair_mixed_kernel<256, 32>;
    if (nx == 128 && half == 128) p.fn = (void*)pair::sweep_pair_mixed_kernel<128, 32>;
    return p;
}

}  // namespace

int resident_blocks(const void* fn, int threads)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess) return 0;
    return per_cu * cus;
}

int sweep_pair_pairs(const KArgs& a, int64_t n_tasks)
{
    const PairShape ps = pair_shape(a.g.nx, a.g.ny);
    if (!ps.fn || !a.large || a.is1d) return 0;
    const int resident = resident_blocks(ps.fn, pair::kThreads);
    int pairs = (resident / 2) / 8 * 8;
    const int64_t want = (n_tasks + 7) / 8 * 8;
    if (pairs > want) pairs = (int)want;
    if (pairs < 8) return 0;
    // the mailbox in the large-grid scratch (free while the sweep runs)
    const size_t slot = ((size_t)pair::pack_floats(a.g.nx) + 2 * pair::kParts + 63) / 64 * 64;
    const size_t need = (2 * (size_t)pairs * 2 * slot + xg_offset_pad + 2 * (size_t)pairs * pair::kXgMax * pair::kThreads) * sizeof(float);
    const size_t have = (size_t)(a.NT + 1) * 5 * (size_t)a.n * sizeof(double);
    return need <= have ? pairs : 0;
}

hipError_t launch_sweep_pair(const KArgs& a, int pairs, hipStream_t s)
{
    const PairShape ps = pair_shape(a.g.nx, a.g.ny);
    pair::PairArgs pa;
    pa.pairs = pairs;
    pa.slot = (int)(((size_t)pair::pack_floats(a.g.nx) + 2 * pair::kParts + 63) / 64 * 64);
    pa.pack = pair::pack_floats(a.g.nx);
    pa.spin_cap = kSpinCap;
    pa.mail = reinterpret_cast<float*>(a.large_scratch);
    pa.xg = pa.mail + 2 * (size_t)pairs * 2 * pa.slot + xg_offset_pad;
    hipLaunchKernelGGL(pair::reset_mailbox_kernel, dim3(8), dim3(256), 0, s, pa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    KArgs ka = a;
    void* args[] = {&ka, &pa};
    return hipLaunchCooperativeKernel(ps.fn, dim3(2 * pairs), dim3(pair::kThreads), args, 0, s);
}

}  // namespace atm
