// trbt_chase.hip -- banded-to-tridiagonal reduction by bulge chasing on AMD
// Instinct MI355X (gfx950): the step that produces the Householder
// reflectors the back-transformation consumes (Sec. 2.2.1, Eq. 2stage_fwd2,
// Eq. householder).
//
// The reduction.  B is Hermitian with semi-bandwidth b, held in lower band
// storage.  Stage s (0-based, s = 0 .. n-3) runs S_s steps.  Step (s, j)
// acts on rows [r0, r0+len), r0 = s+1+j*b, len = min(b, n-r0):
//   * it annihilates column c below row r0 (c = s for j = 0, else the first
//     column of the bulge the previous step created, c = r0-b) with a
//     reflector H = I - tau v v^H built from that column segment
//     (H^H x = beta e1, beta real, v[0] = 1), stored in generation order;
//   * it applies the similarity B <- H^H B H to the rest of rows/columns
//     [r0, r0+len).
// Its nonzero footprint (traced exactly on the sequential order) is:
// column c and, for j > 0, columns c+1 .. r0-1 on rows [r0, r0+len) (the
// "left block", updated from the left only); the lower triangle of the
// diagonal block [r0, r0+len)^2 (updated from both sides); and the rows
// [r0+len, r0+len+b) of columns [r0, r0+len) (the "right block", updated
// from the right: this is where the next bulge appears).  All of it lies
// within 2b-1 of the diagonal, so the band is kept with 2b stored diagonals.
//
// Parallel schedule (the pipelined stages of Sec. 2.2.1's bulge chasing).
// In the sequential order every step of stage s-1 precedes every step of
// stage s.  The footprint of (s, j) meets those of stage s-1 only for steps
// j' <= j+2, and its overlap with (s-1, j+2) is one entry: the right block's
// last, which is the leading entry of the column (s-1, j+2) annihilates.  So
// (s, j) runs once (s-1, 0 .. j+1) are done, leaves the last row of its
// right block for a tail that waits for (s-1, j+2), and finishes it with the
// corner's new value; stages form a pipeline two steps apart.  (Exhaustive
// checks of this schedule against the traced sequential footprints, over
// stage distances 1-5 and ragged ends, find no other overlap.)  Each stage is
// run start to finish by one workgroup (stages are dealt in increasing order
// from a ticket counter), which publishes its progress after every step
// and waits for its predecessor's, the band being read and written with
// device-coherent accesses (so neither side needs a fence over the whole
// cache).  A stage only ever waits on a stage whose ticket was taken earlier
// by a workgroup that is running, so the wait always ends; it is bounded
// anyway (a wall-clock limit that sets an error flag and makes every
// workgroup leave).
//
// A step's right block is exactly the next step's column c and left block,
// and no other step touches it in between, so it stays in registers and is
// stored once, by the next step.
//
// One step on one workgroup of 16 waves, lane = row of the block, block
// columns dealt round-robin over the waves by their offset (from c for the
// left block, from r0 for the others):
//   1. all waves load their columns of the right and diagonal blocks (the
//      left block and column c come from the registers of the previous
//      step, or column c from memory for j = 0); the diagonal block is also
//      mirrored into LDS as a dense Hermitian matrix;
//   2. wave 0 builds the reflector (one wave-wide sum of squares), writes
//      (v, tau) and the annihilated column;
//   3. left block: y <- y - conj(tau) v (v^H y) per column (wave-wide sums,
//      all of a wave's columns reduced together); right block: partial
//      products z = M v; diagonal block: partial products p = A v;
//   4. z and p summed over the waves in fixed order; w = tau p -
//      (|tau|^2/2)(v^H p) v; right block M <- M - tau z v^H; diagonal block
//      A <- A - w v^H - v w^H (the two-sided product written as a rank-2
//      update, which is H^H A H expanded), lower triangle stored.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "trbt.h"
#include "trbt_device.h"
#include "trbt_lanes.h"

namespace {

constexpr int CH_BMAX = 64;        // largest semi-bandwidth of the chase
constexpr int CH_NW = 16;          // waves per workgroup
constexpr int CH_PITCH = CH_BMAX + 1;          // LDS pitch of the diagonal block
constexpr int CH_MAX_WG = 512;     // persistent workgroups at most
constexpr int64_t CH_HDR = 256;    // workspace header: ticket, error flag
// a progress wait gives up after this many ticks of the 100 MHz wall clock
// (10 s): far beyond any step's duration
constexpr uint64_t CH_WAIT_TICKS = 1000000000ull;

struct cx {
    double re, im;
};

template <bool C>
__device__ inline cx cadd(cx a, cx b)
{
    if constexpr (C) return {a.re + b.re, a.im + b.im};
    else return {a.re + b.re, 0.0};
}

template <bool C>
__device__ inline cx cmul(cx a, cx b)   // a b
{
    if constexpr (C) return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    else return {a.re * b.re, 0.0};
}

template <bool C>
__device__ inline cx cmulc(cx a, cx b)   // conj(a) b
{
    if constexpr (C) return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
    else return {a.re * b.re, 0.0};
}

template <bool C>
__device__ inline cx cmul_cb(cx a, cx b)   // a conj(b)
{
    if constexpr (C) return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
    else return {a.re * b.re, 0.0};
}

template <bool C>
__device__ inline cx csub(cx a, cx b)
{
    if constexpr (C) return {a.re - b.re, a.im - b.im};
    else return {a.re - b.re, 0.0};
}

template <bool C>
__device__ inline cx ldx(const double* p)
{
    if constexpr (C) return {p[0], p[1]};
    else return {p[0], 0.0};
}

template <bool C>
__device__ inline void stx(double* p, cx v)
{
    p[0] = v.re;
    if constexpr (C) p[1] = v.im;
}

// Device-coherent (agent-scope relaxed atomic) access to the band: every
// entry a step reads may have been written by another stage's workgroup on
// another CU (and another XCD's L2), and every entry it writes may be read
// by one; ordering comes from the progress counters (see the step's end).
template <bool C>
__device__ inline cx ldx_coh(const double* p)
{
    double* q = const_cast<double*>(p);
    cx v;
    v.re = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v.im = C ? __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
    return v;
}

template <bool C>
__device__ inline void stx_coh(double* p, cx v)
{
    __hip_atomic_store(p, v.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if constexpr (C) __hip_atomic_store(p + 1, v.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool C>
__device__ inline cx shfl_x(cx v, int src)
{
    cx r;
    r.re = __shfl(v.re, src, 64);
    r.im = C ? __shfl(v.im, src, 64) : 0.0;
    return r;
}

// sums over the 64 lanes of N values at once (every lane gets every sum):
// within rows by DPP, then across the four rows by two lane swaps; the N
// values are independent and interleave
template <bool C, int N>
__device__ inline void wave_sums(cx (&v)[N])
{
#pragma unroll
    for (int t = 0; t < N; ++t) {
        v[t].re = row_sum(v[t].re);
        if constexpr (C) v[t].im = row_sum(v[t].im);
    }
#pragma unroll
    for (int t = 0; t < N; ++t) {
        v[t].re = swap_add<16>(v[t].re);
        if constexpr (C) v[t].im = swap_add<16>(v[t].im);
    }
#pragma unroll
    for (int t = 0; t < N; ++t) {
        v[t].re = swap_add<32>(v[t].re);
        if constexpr (C) v[t].im = swap_add<32>(v[t].im);
    }
}

__device__ inline double wave_sum1(double x) { return wave_sum(x); }

// Band copy with 2b stored diagonals (the fill of the chase), zeroed
// counters.  bd[(d + k*2b) * E] = B(k+d, k).
template <bool C>
__global__ void k_chase_init(int64_t n, int b, const double* __restrict__ ab, int64_t ldab,
                             double* __restrict__ bd, int* __restrict__ prog,
                             int* __restrict__ ctl)
{
    constexpr int E = C ? 2 : 1;
    const int64_t LD = 2 * (int64_t)b;
    const int64_t total = n * LD;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += stride) {
        const int64_t k = x / LD, d = x - k * LD;
        cx v = {0.0, 0.0};
        if (d <= b && k + d < n) v = ldx<C>(ab + (d + k * ldab) * E);
        if (d == 0) v.im = 0.0;   // a Hermitian matrix has a real diagonal
        stx<C>(bd + x * E, v);
    }
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) prog[x] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 2) ctl[threadIdx.x] = 0;
}

// thread 0 of the workgroup: wait until *p >= need or the error flag is set
// or the time limit passes; returns false on failure (and sets the flag)
__device__ inline bool chase_wait(const int* p, int need, int* ctl)
{
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
        if (__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() - t0 > CH_WAIT_TICKS) {
            __hip_atomic_store(&ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
}

template <bool C, int NW>
__global__ __launch_bounds__(64 * NW) void k_chase(int64_t n, int b,
                                                        double* __restrict__ bd,
                                                        double* __restrict__ hv,
                                                        double* __restrict__ ht,
                                                        int* __restrict__ prog,
                                                        int* __restrict__ ctl)
{
    constexpr int E = C ? 2 : 1;
    const int64_t LD = 2 * (int64_t)b;
    const int64_t nst = n - 2;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    __shared__ double As[CH_BMAX * CH_PITCH * E];   // diagonal block, column-major, dense
    __shared__ double vs[CH_BMAX * E];
    constexpr int COLS = CH_BMAX / NW;   // block columns per wave
    __shared__ double zs[NW][CH_BMAX * E], ps[NW][CH_BMAX * E];
    __shared__ double tau_s[2];
    __shared__ int64_t s_sh;
    __shared__ int fail_sh;
    // tail waits of this workgroup that wave 0 has seen end (the other
    // waves' tail waits read it here instead of polling global memory).  It
    // only grows over the kernel (every wave counts the same tail waits in
    // `tick`), so a wave that reads it late still finds a value at least
    // its own count.
    __shared__ int64_t seen_sh;
    if (threadIdx.x == 0) seen_sh = 0;
    int64_t tick = 0;

    auto at = [&](int64_t i, int64_t k) { return bd + ((i - k) + k * LD) * E; };
    // the same address as column base + row offset: B(i, k) is at
    // bd + k CS + i E, and the columns a wave holds are NW apart
    const int64_t CS = (LD - 1) * E, SNW = NW * CS;

    for (;;) {
        if (threadIdx.x == 0) {
            const bool bad = __hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_sh = bad ? nst : (int64_t)atomicAdd(&ctl[0], 1);
        }
        __syncthreads();
        const int64_t s64 = s_sh;
        __syncthreads();   // every thread has read the ticket before the next one is taken
        if (s64 >= nst) return;
        // row, column, stage and step indices fit 32 bits (n <= 2^30)
        const int s = (int)s64, nn = (int)n;
        const int S = (int)sweeps_in_stage(n, b, s);
        const int Sp = s > 0 ? (int)sweeps_in_stage(n, b, s - 1) : 0;
        int64_t kref = stage_offset(n, b, s);
        // the previous step's right block, kept in registers: it is exactly
        // this step's column c and left block (rows [r0, r0+len), columns
        // c .. c+b-1, dealt over the waves by column offset like the right
        // block), and no other step touches it in between (the one shared
        // entry, its last, was finished in the previous step's tail)
        cx car[COLS];
        for (int j = 0; j < S; ++j, ++kref) {
            // (s-1, 0 .. j+1) done: for j > 0 the previous step's tail already
            // waited for that
            if (s > 0 && j == 0) {
                if (threadIdx.x == 0) {
                    fail_sh = !chase_wait(&prog[s - 1], j + 2 < Sp ? j + 2 : Sp, ctl);
                }
                __syncthreads();
                if (fail_sh) return;
            }
            const int r0 = s + 1 + j * b;
            const int len = nn - r0 < b ? nn - r0 : b;
            const int rest = nn - r0 - len;
            const int nr = rest < b ? rest : b;                 // right-block rows
            const int c = j == 0 ? s : r0 - b;
            const bool has_next = j + 1 < S;                    // else the right block is stored here
            // the right block's last entry (row r0+2b-1, column r0+b-1) is
            // the leading entry of the column step (s-1, j+2) annihilates:
            // its row is finished in the tail, after that step
            const bool corner = len == b && nr == b;
            const bool crow = corner && lane == b - 1;          // this lane holds that row
            // this wave's first block column (k = r0 + w; for the left block
            // k = c + w) and the lane's rows (r0 + lane, r0 + len + lane)
            double* const cw = bd + (int64_t)(r0 + w) * CS;
            double* const cl = bd + (int64_t)(c + w) * CS;
            const int64_t rd = (int64_t)(r0 + lane) * E, rr = (int64_t)(r0 + len + lane) * E;

            // 1. loads (column c + m, m = w + NW t: x for m = 0, the left
            // block for m >= 1 -- carried over for j > 0)
            cx x = {0.0, 0.0};
            if (w == 0) {
                if (j > 0) x = car[0];
                else if (lane < len) x = ldx_coh<C>(bd + (int64_t)c * CS + rd);
            }
            cx yl[COLS], yr[COLS], ad[COLS];
            // every lane issues every load (from a valid dummy address where
            // it has no entry), so the loads of all columns are in flight
            // together instead of one masked load and its wait at a time
#pragma unroll
            for (int t = 0; t < COLS; ++t) {
                const int m = w + NW * t;
                yl[t] = (j > 0 && m >= 1) ? car[t] : cx{0.0, 0.0};
                // (the corner is read in the tail: step (s-1, j+2) may be
                // writing it now)
                const bool okr = m < len && lane < nr && !(crow && m == b - 1);
                const bool okd = m < len && lane >= m && lane < len;
                yr[t] = ldx_coh<C>(okr ? cw + t * SNW + rr : bd);
                ad[t] = ldx_coh<C>(okd ? cw + t * SNW + rd : bd);
            }
            // 2. the reflector (wave 0)
            if (w == 0) {
                const double ar = __shfl(x.re, 0, 64);
                const double ai = C ? __shfl(x.im, 0, 64) : 0.0;
                const double xn2 = wave_sum1(lane >= 1 && lane < len ? x.re * x.re + x.im * x.im : 0.0);
                cx tau, v;
                double beta;
                if (xn2 == 0.0 && ai == 0.0) {
                    tau = {0.0, 0.0};
                    beta = ar;
                    v = lane == 0 ? cx{1.0, 0.0} : x;
                } else {
                    const double nrm = sqrt(ar * ar + ai * ai + xn2);
                    const double bt = ar >= 0.0 ? -nrm : nrm;
                    tau = {(bt - ar) / bt, C ? -ai / bt : 0.0};
                    cx scale;
                    if constexpr (C) {
                        const double dr = ar - bt, di = ai, den = dr * dr + di * di;
                        scale = {dr / den, -di / den};
                    } else {
                        scale = {1.0 / (ar - bt), 0.0};
                    }
                    v = lane == 0 ? cx{1.0, 0.0} : cmul<C>(x, scale);
                    beta = bt;
                }
                if (lane >= len) v = cx{0.0, 0.0};
                stx<C>(&vs[lane * E], v);
                if (lane == 0) {
                    tau_s[0] = tau.re;
                    tau_s[1] = tau.im;
                    stx<C>(ht + kref * E, tau);
                }
                if (lane < b) stx<C>(hv + (kref * b + lane) * E, v);
                if (lane < len) stx_coh<C>(bd + (int64_t)c * CS + rd, lane == 0 ? cx{beta, 0.0} : cx{0.0, 0.0});
            }
            // the mirror of the diagonal block (its loads have been in flight
            // while wave 0 built the reflector)
#pragma unroll
            for (int t = 0; t < COLS; ++t) {
                const int m = w + NW * t;
                const bool okr = m < len && lane < nr && !(crow && m == b - 1);
                const bool okd = m < len && lane >= m && lane < len;
                if (!okr) yr[t] = cx{0.0, 0.0};
                if (!okd) ad[t] = cx{0.0, 0.0};
                if (okd) {
                    stx<C>(&As[(m * CH_PITCH + lane) * E], ad[t]);
                    if (lane > m) stx<C>(&As[(lane * CH_PITCH + m) * E], cx{ad[t].re, -ad[t].im});
                }
            }

            __syncthreads();

            // 3. left block; partial products of the right and diagonal blocks
            const cx vi = ldx<C>(&vs[lane * E]);
            const cx tau = {tau_s[0], C ? tau_s[1] : 0.0};
            {
                cx dot[COLS];
#pragma unroll
                for (int t = 0; t < COLS; ++t) dot[t] = cmulc<C>(vi, yl[t]);
                wave_sums<C, COLS>(dot);
#pragma unroll
                for (int t = 0; t < COLS; ++t) {
                    const int m = w + NW * t;
                    if (j > 0 && m >= 1 && m < b) {
                        const cx f = cmulc<C>(tau, dot[t]);           // conj(tau) (v^H y)
                        yl[t] = csub<C>(yl[t], cmul<C>(f, vi));
                        if (lane < len) stx_coh<C>(cl + t * SNW + rd, yl[t]);
                    }
                }
            }
            cx zp = {0.0, 0.0}, pp = {0.0, 0.0};
#pragma unroll
            for (int t = 0; t < COLS; ++t) {
                const int m = w + NW * t;
                if (m < len) {
                    const cx vm = ldx<C>(&vs[m * E]);
                    if (!(crow && m == b - 1)) zp = cadd<C>(zp, cmul<C>(yr[t], vm));
                    if (lane < len) pp = cadd<C>(pp, cmul<C>(ldx<C>(&As[(m * CH_PITCH + lane) * E]), vm));
                }
            }
            stx<C>(&zs[w][lane * E], zp);
            stx<C>(&ps[w][lane * E], pp);
            __syncthreads();

            // 4. right and diagonal blocks
            cx z = ldx<C>(&zs[0][lane * E]), p = ldx<C>(&ps[0][lane * E]);
#pragma unroll
            for (int q = 1; q < NW; ++q) {
                z = cadd<C>(z, ldx<C>(&zs[q][lane * E]));
                p = cadd<C>(p, ldx<C>(&ps[q][lane * E]));
            }
            const double sc = wave_sum1(cmulc<C>(vi, p).re);              // v^H A v (real)
            const double h = 0.5 * (tau.re * tau.re + tau.im * tau.im) * sc;
            const cx tp = cmul<C>(tau, p);
            const cx wv = {tp.re - h * vi.re, C ? tp.im - h * vi.im : 0.0};
            const cx tz = cmul<C>(tau, z);
#pragma unroll
            for (int t = 0; t < COLS; ++t) {
                const int m = w + NW * t;
                if (m < len) {
                    const cx vm = ldx<C>(&vs[m * E]);
                    if (!crow) {
                        yr[t] = csub<C>(yr[t], cmul_cb<C>(tz, vm));
                        if (!has_next && lane < nr) stx_coh<C>(cw + t * SNW + rr, yr[t]);
                    }
                    const cx wm = shfl_x<C>(wv, m);
                    ad[t] = csub<C>(ad[t], cadd<C>(cmul_cb<C>(wv, vm), cmul_cb<C>(vi, wm)));
                    if (lane >= m && lane < len) stx_coh<C>(cw + t * SNW + rd, ad[t]);
                }
            }

            // tail: (s-1, 0 .. j+2) done (all of stage s-1 when it has no
            // step j+2); with the corner, the last row of the right block:
            // z[b-1] completed with the corner's current value, then that
            // row's update.  Every wave waits, so that a finished (s, j)
            // implies a finished (s-1, j+2), and the next step needs no wait
            // of its own.  Wave 0 polls the counter and passes what it saw
            // to the other waves through LDS; on a failed wait it sets the
            // error flag and releases them, and the stage runs on without
            // waiting (its results are discarded: d is filled with NaN).
            if (s > 0) {
                const int need = (int)(j + 3 < Sp ? j + 3 : Sp);
                ++tick;
                if (w == 0) {
                    if (lane == 0) {
                        const bool ok = chase_wait(&prog[s - 1], need, ctl);
                        __hip_atomic_store(&seen_sh, ok ? tick : INT64_MAX, __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                } else if (__hip_atomic_load(&seen_sh, __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_WORKGROUP) < tick) {
                    // bounded like every wait: on time-out, flag the error
                    // and go on
                    const uint64_t t0 = wall_clock64();
                    while (__hip_atomic_load(&seen_sh, __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_WORKGROUP) < tick) {
                        __builtin_amdgcn_s_sleep(1);
                        if (wall_clock64() - t0 > CH_WAIT_TICKS) {
                            __hip_atomic_store(&ctl[1], 1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            break;
                        }
                    }
                }
            }
            if (corner) {
                const cx vb = ldx<C>(&vs[(b - 1) * E]);
                cx zc = z;
                if (crow) {
                    const cx cv = ldx_coh<C>(at(r0 + 2 * (int64_t)b - 1, r0 + b - 1));
                    zc = cadd<C>(z, cmul<C>(cv, vb));
#pragma unroll
                    for (int t = 0; t < COLS; ++t) {
                        const int m = w + NW * t;
                        if (m == b - 1) yr[t] = cv;
                    }
                }
                const cx tzc = cmul<C>(tau, zc);
#pragma unroll
                for (int t = 0; t < COLS; ++t) {
                    const int m = w + NW * t;
                    if (m < len && crow) {
                        yr[t] = csub<C>(yr[t], cmul_cb<C>(tzc, ldx<C>(&vs[m * E])));
                        if (!has_next) stx_coh<C>(cw + t * SNW + rr, yr[t]);
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < COLS; ++t) car[t] = yr[t];

            // publish the step: every wave waits until its (device-coherent)
            // stores have completed, the workgroup meets, and one counter
            // store.  A waiting stage reads the counter, then the band with
            // device-coherent loads, so it sees every store made before the
            // counter.  (Agent-scope release and acquire fences would write
            // back and invalidate the whole L2 of the XCD at every step; one
            // atomic add per wave instead of the barrier was much slower:
            // the adds to one address serialise.)
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_store(&prog[s], (int)(j + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// d = real diagonal, e = first subdiagonal of the reduced band; NaN in d if
// the chase gave up on a wait
template <bool C>
__global__ void k_chase_extract(int64_t n, int b, const double* __restrict__ bd,
                                double* __restrict__ d, double* __restrict__ e,
                                const int* __restrict__ ctl)
{
    constexpr int E = C ? 2 : 1;
    const int64_t LD = 2 * (int64_t)b;
    const bool bad = ctl[1] != 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        d[k] = bad ? __builtin_nan("") : bd[k * LD * E];
        if (k + 1 < n) stx<C>(e + k * E, ldx<C>(bd + (1 + k * LD) * E));
    }
}

inline size_t chase_bytes(int64_t n, int nbw, bool cplx)
{
    if (n <= 0) return 0;
    const size_t prog = ((size_t)n * sizeof(int) + 255) / 256 * 256;
    return CH_HDR + prog + (size_t)n * 2 * nbw * (cplx ? 16 : 8);
}

template <bool C>
int chase(int64_t n, int nbw, const double* ab, int64_t ldab, double* d, double* e, double* hv,
          double* ht, void* work, size_t work_bytes, void* stream_v)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > CH_BMAX) return -2;
    if (n > 0 && !ab) return -3;
    if (ldab < nbw + 1) return -4;
    if (n > 0 && !d) return -5;
    if (n > 1 && !e) return -6;
    const int64_t K = num_reflectors(n, nbw);
    if (K > 0 && !hv) return -7;
    if (K > 0 && !ht) return -8;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -9;
    if (n > (int64_t)1 << 30) return -1;   // stage counters are 32-bit
    if (n == 0) return TRBT_SUCCESS;
    if (!work || work_bytes < chase_bytes(n, nbw, C)) return TRBT_ERR_WORKSPACE;
    int rc = check_device();
    if (rc) return rc;
    hipStream_t stream = (hipStream_t)stream_v;
    char* wb = (char*)work;
    int* ctl = (int*)wb;
    int* prog = (int*)(wb + CH_HDR);
    double* bd = (double*)(wb + CH_HDR + ((size_t)n * sizeof(int) + 255) / 256 * 256);

    const int64_t band = n * 2 * nbw;
    const int ib = (int)((band + 255) / 256 < 4096 ? (band + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_chase_init<C>, dim3(ib > 0 ? ib : 1), dim3(256), 0, stream, n, nbw, ab,
                       ldab, bd, prog, ctl);
    if (K > 0) {
        const int64_t nst = n - 2;
        const int g = (int)(nst < CH_MAX_WG ? nst : CH_MAX_WG);
        hipLaunchKernelGGL((k_chase<C, CH_NW>), dim3(g), dim3(64 * CH_NW), 0, stream, n, nbw, bd, hv,
                           ht, prog, ctl);
    }
    const int eb = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_chase_extract<C>, dim3(eb), dim3(256), 0, stream, n, nbw, bd, d, e, ctl);
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

}  // namespace

extern "C" {

int trbt_band_to_tridi_workspace_bytes(int64_t n, int nbw, int is_complex, size_t* bytes)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > CH_BMAX) return -2;
    if (!bytes) return -4;
    *bytes = chase_bytes(n, nbw, is_complex != 0);
    return TRBT_SUCCESS;
}

int trbt_band_to_tridi_d(int64_t n, int nbw, const double* ab, int64_t ldab, double* d,
                         double* e, double* hh_v, double* hh_tau, void* work,
                         size_t work_bytes, void* stream)
{
    return chase<false>(n, nbw, ab, ldab, d, e, hh_v, hh_tau, work, work_bytes, stream);
}

int trbt_band_to_tridi_z(int64_t n, int nbw, const trbt_z* ab, int64_t ldab, double* d,
                         trbt_z* e, trbt_z* hh_v, trbt_z* hh_tau, void* work,
                         size_t work_bytes, void* stream)
{
    return chase<true>(n, nbw, (const double*)ab, ldab, d, (double*)e, (double*)hh_v,
                       (double*)hh_tau, work, work_bytes, stream);
}

}  // extern "C"
