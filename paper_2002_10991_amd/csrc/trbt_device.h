// trbt_device.h -- device code shared by the single-problem, batched and
// adjoint entry points of libtrbt (gfx950).  Internal header: it defines
// kernels and helpers in an anonymous namespace, so every translation unit
// that includes it gets its own instantiations.
//
//
// Operation (Yu et al., CPC 2020, Sec. 2.2.2, Eq. 2stage_bkwd1 and
// Eq. kernel): apply every Householder reflector H_k = I - tau_k v_k v_k^H
// produced by bulge chasing (Sec. 2.2.1) to every column of Z, in exactly
// the reverse of the generation order.  Columns are independent; reflectors
// of one stage touch disjoint rows; from stage s to s-1 the window of every
// sweep ("slot") moves up by one row (Sec. 3.2, Fig. kernel).
//
// Two device paths:
//
//  * unblocked ("generic"): one lane per column, every reflector applied
//    by a dot product and an axpy on the column in global memory, in a
//    blocked topological order of the reflector DAG.  Any nbw.
//
//  * blocked ("tile ring", nbw a multiple of 16, up to 64 in every form
//    and up to 128 for the single-problem forward): the reflectors
//    of one slot over 16 consecutive stages are merged into one compact-WY
//    factor  H_a ... H_b = I - V T V^H  (Schreiber & Van Loan); a pack
//    kernel precomputes, per (slot, 16-stage block), A1 = T V^H and -V in
//    the register layout of v_mfma_f64_16x16x4_f64.  The main kernel gives
//    each workgroup a strip of columns; each of its 8 waves owns one slot at
//    a time and keeps that slot's (nbw+16) x (16*CT) window of Z in
//    registers while the window slides up 16 rows per block, exchanging one
//    16-row tile per block with the neighbouring slots through Z (same CU,
//    workgroup-scope release/acquire on LDS progress counters).  Per block
//    the update is two small dense products on FP64 MFMA:
//        Y = A1 * Zwin        (16 x 16CT, K = nbw+16)
//        Zwin += (-V) * Y     (nbw+16 x 16CT, K = 16)
//
// Ordering argument for the blocked path (0-based stage s, slot j, block
// t = stages n-3-16t .. n-18-16t): reflector (s, j) depends only on (s+1, j)
// and (s+1, j-1); hence block (t, j) depends on (t-1, j) and (t, j-1).
// A wave walks its slot's blocks in order, and before block t waits until
// slot j-1 has finished block t.  Slot j's window at block t is rows
// [p0, p0+nbw+16) with p0 = s_top-15+j*nbw; its top 16-row tile is exactly
// the tile slot j-1 retires after block t, and its bottom tile is the one
// slot j+1 picks up.

#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include "trbt.h"

namespace {

// --------------------------------------------------------------------------
// Reflector geometry (Sec. 2.2.1), shared by host validation and kernels.
// --------------------------------------------------------------------------
__host__ __device__ inline int64_t sweeps_in_stage(int64_t n, int64_t b, int64_t s)
{
    if (n < 3 || b < 2 || s < 0 || s > n - 3) return 0;
    return (n - s - 2 + b - 1) / b;
}

// F(M) = sum_{m=1..M} ceil(m/b) = b q(q+1)/2 + r(q+1), M = q b + r
__host__ __device__ inline int64_t ceil_sum(int64_t M, int64_t b)
{
    if (M <= 0) return 0;
    int64_t q = M / b, r = M % b;
    return b * q * (q + 1) / 2 + r * (q + 1);
}

// generation index of reflector (s, 0): sum_{s' < s} ceil((n-s'-2)/b)
__host__ __device__ inline int64_t stage_offset(int64_t n, int64_t b, int64_t s)
{
    if (b < 2 || n < 3) return 0;
    return ceil_sum(n - 2, b) - ceil_sum(n - 2 - s, b);
}

__host__ __device__ inline int64_t num_reflectors(int64_t n, int64_t b)
{
    return stage_offset(n, b, n - 2);
}

// --------------------------------------------------------------------------
// Scalar helpers
// --------------------------------------------------------------------------
struct cd {
    double re, im;
};

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline double conj_mul_re(cd a, cd b) { return a.re * b.re + a.im * b.im; }  // Re(conj(a) b)
__device__ inline double conj_mul_im(cd a, cd b) { return a.re * b.im - a.im * b.re; }  // Im(conj(a) b)

// ==========================================================================
// Unblocked kernel: one lane per column.
// Order: 16-stage blocks from the top stage down; inside a block, slot by
// slot (ascending), and inside a slot stage by stage (descending).  This is
// a valid topological order of the reflector DAG for every nbw, and it
// reuses each slot's rows for 16 consecutive reflectors.
// ==========================================================================
__device__ inline void apply_one(double* z, const double* __restrict__ v, double tau, int len)
{
    double d = 0.0;
    for (int i = 0; i < len; ++i) d = fma(v[i], z[i], d);
    const double a = tau * d;
    for (int i = 0; i < len; ++i) z[i] = fma(-a, v[i], z[i]);
}

__device__ inline void apply_one(cd* z, const cd* __restrict__ v, cd tau, int len)
{
    double dr = 0.0, di = 0.0;
    for (int i = 0; i < len; ++i) {
        const cd vi = v[i], zi = z[i];
        dr += conj_mul_re(vi, zi);
        di += conj_mul_im(vi, zi);
    }
    const double ar = tau.re * dr - tau.im * di;
    const double ai = tau.re * di + tau.im * dr;
    for (int i = 0; i < len; ++i) {
        const cd vi = v[i];
        cd zi = z[i];
        zi.re -= ar * vi.re - ai * vi.im;
        zi.im -= ar * vi.im + ai * vi.re;
        z[i] = zi;
    }
}

template <typename T>
__device__ inline void unblocked_column(int64_t n, int nbw, const T* __restrict__ hv,
                                        const T* __restrict__ ht, T* __restrict__ z)
{
    const int64_t nblk = (n - 2 + 15) / 16;
    for (int64_t t = 0; t < nblk; ++t) {
        const int64_t stop = n - 3 - 16 * t;
        const int64_t sbot = stop - 15 > 0 ? stop - 15 : 0;
        const int64_t J = sweeps_in_stage(n, nbw, sbot);
        for (int64_t j = 0; j < J; ++j) {
            for (int64_t s = stop; s >= sbot; --s) {
                if (j >= sweeps_in_stage(n, nbw, s)) continue;
                const int64_t k = stage_offset(n, nbw, s) + j;
                const int64_t r0 = s + 1 + j * nbw;
                const int len = (int)(n - r0 < nbw ? n - r0 : nbw);
                apply_one(z + r0, hv + k * nbw, ht[k], len);
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(64) void k_unblocked(int64_t n, int nbw, int64_t nev,
                                                  const T* __restrict__ hv,
                                                  const T* __restrict__ ht, T* __restrict__ Z,
                                                  int64_t ldz)
{
    const int64_t col = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (col >= nev) return;
    unblocked_column(n, nbw, hv, ht, Z + col * ldz);
}

// ==========================================================================
// Blocked path
// ==========================================================================
constexpr int KB = 16;        // stages per block (one MFMA tile of rows)
constexpr int WAVES = 8;      // slots in flight per workgroup
constexpr int HDR_BYTES = 256;

// Blocks of slot j: t = j*(nbw/16) .. nblk-1.  Slot-major numbering.
__host__ __device__ inline int64_t slot_base(int64_t j, int64_t nblk, int64_t nt1)
{
    return j * nblk - nt1 * j * (j - 1) / 2;
}

__host__ inline int64_t blocked_num_blocks(int64_t n, int nbw)
{
    const int64_t J = sweeps_in_stage(n, nbw, 0);
    const int64_t nblk = (n - 2 + KB - 1) / KB;
    return slot_base(J, nblk, nbw / KB);
}

template <int NB, bool CPLX>
struct Geo {
    static constexpr int NT = NB / 16 + 1;                // tiles in a window
    static constexpr int NC = CPLX ? 2 : 1;               // planes (re, im)
    static constexpr int CHUNK = 64 * NC;                 // doubles per chunk
    static constexpr int A1_DBL = NT * 4 * CHUNK;         // A1 = T V^H, packed
    static constexpr int PB = 2 * A1_DBL;                 // doubles per block
};

// --------------------------------------------------------------------------
// Pack kernel: one workgroup (256 threads) per (slot, block).
//   Vt[r][p]  window row r in [0, 16*NT), reflector p in [0,16) in generation
//             order (p = 15 - m, m = stages below the block's top stage);
//             reflector p occupies window rows [p+1, p+1+len).
//   T         forward compact-WY factor (upper triangular):
//             T[p][p] = tau_p, T[0:p, p] = -tau_p T[0:p,0:p] (Vt[:,0:p]^H v_p)
//   A1[p][r] = sum_{q>=p} T[p][q] conj(Vt[r][q])
// Packed for v_mfma_f64_16x16x4_f64 (A operand: lane i+16k holds A[i][k];
// B operand: lane j+16k holds B[k][j]; accumulator: lane j+16g holds rows
// g, g+4, g+8, g+12 of column j), chunk (q, u) of window tile q:
//   A1 chunk lane l: A1[l%16][16q + 4u + l/16]     stored at position 4h+u
//   -V chunk lane l: -Vt[16q + l%16][4u + l/16]    stored at position
//                    4NT + u*NT + (NT-1-h) (fixed window),
//                    4NT + 4(NT-1-h) + u (rotating window)
// where h is the register tile that holds window tile q during this block:
// h = q for a fixed window (the real kernels with one column tile);
// h = (q + rot) mod NT for a rotating window (complex, and real with two
// column tiles per wave), the main kernel never moving a tile between
// registers (the window's top tile sits in register tile rot = (-o) mod NT
// in the o-th block of a slot).  So the chunks are stored in exactly the
// order the main kernel consumes them.
// --------------------------------------------------------------------------
// Shared-memory image of one block's compact-WY factor (see above).
template <int NB, bool CPLX>
struct WyBlock {
    static constexpr int NT = Geo<NB, CPLX>::NT, NC = Geo<NB, CPLX>::NC, R = 16 * NT;
    double Vt[R][17][NC];       // (one column of padding: the V load writes down columns)
    double Gm[16][16][NC];
    double Tm[16][16][NC];
    double tau[16][NC];
    double Gp[4][16][16][NC];   // per-wave partial Gram matrices
    int64_t j, t;
    int64_t kref[16];           // reflector index of position p (-1: none)
    int lref[16];               // its length
};

// D + A B on v_mfma_f64_16x16x4_f64 (A lane i+16k = A[i][k], B lane j+16k =
// B[k][j]; D lane j+16g, element e = D[g+4e][j]).
__device__ inline d4 pack_mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// wy_factor fills W for block `blk` (slot-major numbering): the reflectors
// in window layout, their Gram matrix and the forward factor T.  All 256
// threads of the workgroup take part; W is complete on return.
template <int NB, bool CPLX>
__device__ inline void wy_factor(int64_t n, const double* __restrict__ hv,
                                 const double* __restrict__ ht, int64_t blk,
                                 WyBlock<NB, CPLX>& W)
{
    constexpr int NC = WyBlock<NB, CPLX>::NC, R = WyBlock<NB, CPLX>::R;
    auto& Vt = W.Vt;
    auto& Gm = W.Gm;
    auto& Tm = W.Tm;
    auto& tau = W.tau;
    const int tid = threadIdx.x;
    const int64_t nblk = (n - 2 + KB - 1) / KB;
    const int64_t J = sweeps_in_stage(n, NB, 0);
    constexpr int64_t nt1 = NB / 16;
    if (tid == 0) {
        int64_t lo = 0, hi = J;  // find j with slot_base(j) <= blk < slot_base(j+1)
        while (hi - lo > 1) {
            int64_t mid = (lo + hi) / 2;
            if (slot_base(mid, nblk, nt1) <= blk) lo = mid; else hi = mid;
        }
        W.j = lo;
        W.t = lo * nt1 + (blk - slot_base(lo, nblk, nt1));
    }
    __syncthreads();
    const int64_t j = W.j, t = W.t;
    const int64_t s_top = n - 3 - KB * t;

    if (tid < 16) {   // the block's reflector in position p, its length and tau
        const int p = tid;
        const int64_t s = s_top - 15 + p;
        int64_t k = -1;
        int len = 0;
        double tr = 0.0, ti = 0.0;
        if (s >= 0 && s <= n - 3 - j * NB) {
            k = stage_offset(n, NB, s) + j;
            const int64_t r0 = s + 1 + j * NB;
            len = (int)(n - r0 < NB ? n - r0 : NB);
            tr = ht[k * NC];
            if (CPLX) ti = ht[k * NC + 1];
        }
        W.kref[p] = k;
        W.lref[p] = len;
        tau[p][0] = tr;
        if (CPLX) tau[p][NC - 1] = ti;
    }
    __syncthreads();
    // reflector by reflector, so that consecutive threads read consecutive
    // elements of one reflector
    for (int idx = tid; idx < R * 16; idx += 256) {
        const int p = idx / R, r = idx % R;
        const int64_t k = W.kref[p];
        const int e = r - (p + 1);
        double re = 0.0, im = 0.0;
        if (k >= 0 && e >= 0 && e < W.lref[p]) {
            re = hv[(k * NB + e) * NC];
            if (CPLX) im = hv[(k * NB + e) * NC + 1];
        }
        Vt[r][p][0] = re;
        if (CPLX) Vt[r][p][NC - 1] = im;
    }
    __syncthreads();
    {   // Gram matrix Gm = V^H V on MFMA: K runs over the window rows, wave w
        // taking the 4-row chunks kc = w (mod 4); the A operand (V^H) and
        // the B operand (V) of a chunk are the same LDS element per lane
        // (conjugated for A)
        const int lane = tid & 63, w = tid >> 6;
        d4 gr = d4{0.0, 0.0, 0.0, 0.0}, gi = gr;
        for (int kc = w; kc < R / 4; kc += 4) {
            const int r = 4 * kc + lane / 16, c = lane % 16;
            const double vr = Vt[r][c][0];
            gr = pack_mfma(vr, vr, gr);
            if (CPLX) {
                const double vi = Vt[r][c][NC - 1];
                gr = pack_mfma(vi, vi, gr);        // Re: vr.vr + vi.vi
                gi = pack_mfma(vr, vi, gi);        // Im: vr.vi - vi.vr
                gi = pack_mfma(-vi, vr, gi);
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            W.Gp[w][lane / 16 + 4 * e][lane % 16][0] = gr[e];
            if (CPLX) W.Gp[w][lane / 16 + 4 * e][lane % 16][NC - 1] = gi[e];
        }
    }
    __syncthreads();
    {   // the waves' partials in a fixed order; T starts as diag(tau)
        const int a = tid / 16, b = tid % 16;
#pragma unroll
        for (int k = 0; k < NC; ++k)
            Gm[a][b][k] = (W.Gp[0][a][b][k] + W.Gp[1][a][b][k]) +
                          (W.Gp[2][a][b][k] + W.Gp[3][a][b][k]);
        Tm[a][b][0] = (a == b) ? tau[a][0] : 0.0;
        if (CPLX) Tm[a][b][NC - 1] = (a == b) ? tau[a][NC - 1] : 0.0;
    }
    __syncthreads();
    // T = (I + D N)^{-1} D with D = diag(tau) and N the strictly upper part
    // of V^H V (the same T as the column recursion T[0:q,q] =
    // -tau_q T[0:q,0:q] V^H v_q, also for tau = 0): column p by back
    // substitution, T[i][p] = -tau_i sum_{k=i+1..p} Gm[i][k] T[k][p], one
    // thread per column and no barrier between the steps.
    if (tid < 16) {
        const int p = tid;
        for (int i = p - 1; i >= 0; --i) {
            double wr = 0.0, wi = 0.0;   // w = sum_{k=i+1}^{p} Gm[i][k] T[k][p]
            for (int k = i + 1; k <= p; ++k) {
                const double gr = Gm[i][k][0], tr = Tm[k][p][0];
                if (CPLX) {
                    const double gi = Gm[i][k][NC - 1], ti = Tm[k][p][NC - 1];
                    wr += gr * tr - gi * ti;
                    wi += gr * ti + gi * tr;
                } else {
                    wr += gr * tr;
                }
            }
            const double ur = tau[i][0], ui = CPLX ? tau[i][NC - 1] : 0.0;
            Tm[i][p][0] = -(ur * wr - ui * wi);
            if (CPLX) Tm[i][p][NC - 1] = -(ur * wi + ui * wr);
        }
    }
    __syncthreads();
}

// Window form of the blocked kernels: complex windows always rotate; real
// ones rotate for nbw = 48 and 64, where each wave's two column tiles on a
// fixed window would spill (the slide needs a second set of tile registers),
// and stay fixed for nbw <= 32 (fewer instructions per block: 5% faster at
// n = 1024, nbw = 32) and for the wide bands (one tile per wave).  Every
// form of the back-transformation (single problem, batched, the adjoint's
// checkpointing forward) takes the same form for the same nbw, so their
// results agree bitwise.
template <int NB, bool CPLX>
constexpr bool rotating_window()
{
    return CPLX || (NB > 32 && NB <= 64);
}

// pack_block packs block `blk` (slot-major numbering) of one problem into
// ws (the problem's packed-block array); all 256 threads of the workgroup
// take part.
template <int NB, bool CPLX, bool ROT = CPLX>
__device__ inline void pack_block(int64_t n, const double* __restrict__ hv,
                                  const double* __restrict__ ht, double* __restrict__ ws,
                                  int64_t blk)
{
    using G = Geo<NB, CPLX>;
    constexpr int NT = G::NT, NC = G::NC;
    __shared__ WyBlock<NB, CPLX> W;
    wy_factor<NB, CPLX>(n, hv, ht, blk, W);
    const auto& Vt = W.Vt;
    const auto& Tm = W.Tm;
    const int tid = threadIdx.x;
    // register tile of window tile 0 in this block (the block's position in
    // its slot's sequence is W.t - W.j * NB/16); real windows do not rotate
    const int rot = ROT ? (int)((NT - (W.t - W.j * (NB / 16)) % NT) % NT) : 0;
    double* out = ws + (size_t)blk * G::PB;
    {   // A1 = T V^H, as A1^T = conj(V) T^T on MFMA, one 16-row window tile
        // q per product (K = the 16 reflectors), wave w taking q = w (mod 4).
        // Element e of the result in lane l is A1^T[16q + 4e + l/16][l%16] =
        // A1[l%16][16q + 4e + l/16]: exactly A1 chunk (q, u = e) as the main
        // kernel reads it.
        const int lane = tid & 63, w = tid >> 6;
        for (int q = w; q < NT; q += 4) {
            const int h = (q + rot) % NT;
            d4 ar = d4{0.0, 0.0, 0.0, 0.0}, ai = ar;
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                const int r = 16 * q + lane % 16, c = 4 * kc + lane / 16;
                const double vr = Vt[r][c][0], tr = Tm[lane % 16][c][0];
                ar = pack_mfma(vr, tr, ar);
                if (CPLX) {   // (vr - i vi)(tr + i ti)
                    const double vi = Vt[r][c][NC - 1], ti = Tm[lane % 16][c][NC - 1];
                    ar = pack_mfma(vi, ti, ar);
                    ai = pack_mfma(vr, ti, ai);
                    ai = pack_mfma(-vi, tr, ai);
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                out[(4 * h + e) * G::CHUNK + lane] = ar[e];
                if (CPLX) out[(4 * h + e) * G::CHUNK + 64 + lane] = ai[e];
            }
        }
    }
    for (int idx = tid; idx < NT * 4 * 64; idx += 256) {
        const int lane = idx % 64, qu = idx / 64, q = qu / 4, u = qu % 4;
        const int h = (q + rot) % NT;
        {   // -V chunks in the order the main kernel reads them.  Real: u
            // ascending, and within each u the tiles from the bottom of the
            // window up.  Complex: tile by tile from the bottom up, u
            // ascending inside a tile.
            const int r = 16 * q + lane % 16, p = 4 * u + lane / 16;
            const int pos = ROT ? (NT - 1 - h) * 4 + u : u * NT + (NT - 1 - h);
            out[G::A1_DBL + pos * G::CHUNK + lane] = -Vt[r][p][0];
            if (CPLX) out[G::A1_DBL + pos * G::CHUNK + 64 + lane] = -Vt[r][p][NC - 1];
        }
    }
}

template <int NB, bool CPLX, bool ROT = CPLX>
__global__ __launch_bounds__(256) void k_pack(int64_t n, const double* __restrict__ hv,
                                              const double* __restrict__ ht,
                                              double* __restrict__ ws)
{
    pack_block<NB, CPLX, ROT>(n, hv, ht, ws, blockIdx.x);
}

// --------------------------------------------------------------------------
// Main blocked kernel.
// Register tile (accumulator layout of v_mfma_f64_16x16x4_f64, checked on
// gfx950): lane l holds rows l/16 + 4e (e = 0..3) of column l%16.  A K-chunk
// (q, u) of the window is the 4 consecutive rows 16q + 4u + {0..3}: its B
// operand in lane l is element u of tile q, so the Z window is an MFMA
// operand without any data movement.  Likewise element u of the Y tile is
// the B operand for the reflectors 4u + {0..3}.
// --------------------------------------------------------------------------
template <bool CPLX>
struct Tile;
template <>
struct Tile<false> {
    d4 re;
};
template <>
struct Tile<true> {
    d4 re, im;
};

__device__ inline d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

typedef double d2 __attribute__((ext_vector_type(2)));

// MFMA with the FP64 negate modifiers of gfx950 (bit 0 negates A, bit 1 B).
template <int NEG>
__device__ inline d4 mfma_n(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, NEG);
}

// Device-coherent (agent-scope relaxed atomic) loads and stores of single
// elements: for tiles handed from one workgroup to another, which may run on
// another CU and another XCD's L2.
__device__ inline double ld_coh(const double* p)
{
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void st_coh(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile load.  Interior tiles (all rows inside the matrix, whole strip inside
// nev: a wave-uniform test) load directly; edge tiles read a clamped, valid
// address and zero what lies outside, so all loads issue back to back.
// coh (wave-uniform): device-coherent loads of a tile another workgroup
// stored with store_tile(..., coh = true).
template <bool CPLX>
__device__ inline void load_tile(Tile<CPLX>& t, const double* __restrict__ Z, int64_t ldz,
                                 int64_t n, int64_t nev, int64_t row0, int64_t col,
                                 bool interior, bool coh = false)
{
    if (coh) {
        const bool colok = col < nev;
        const int64_t cc = colok ? col : nev - 1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r = row0 + 4 * e;
            const bool ok = colok && r >= 0 && r < n;
            const int64_t rr = r < 0 ? 0 : (r >= n ? n - 1 : r);
            if constexpr (CPLX) {
                const double xr = ld_coh(Z + 2 * (cc * ldz + rr));
                const double xi = ld_coh(Z + 2 * (cc * ldz + rr) + 1);
                t.re[e] = ok ? xr : 0.0;
                t.im[e] = ok ? xi : 0.0;
            } else {
                const double x = ld_coh(Z + cc * ldz + rr);
                t.re[e] = ok ? x : 0.0;
            }
        }
        return;
    }
    if (interior) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r = row0 + 4 * e;
            if constexpr (CPLX) {
                const d2 x = *(const d2*)(Z + 2 * (col * ldz + r));
                t.re[e] = x[0];
                t.im[e] = x[1];
            } else {
                t.re[e] = Z[col * ldz + r];
            }
        }
        return;
    }
    const bool colok = col < nev;
    const int64_t cc = colok ? col : nev - 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t r = row0 + 4 * e;
        const bool ok = colok && r >= 0 && r < n;
        const int64_t rr = r < 0 ? 0 : (r >= n ? n - 1 : r);
        if constexpr (CPLX) {
            const d2 x = *(const d2*)(Z + 2 * (cc * ldz + rr));
            t.re[e] = ok ? x[0] : 0.0;
            t.im[e] = ok ? x[1] : 0.0;
        } else {
            const double x = Z[cc * ldz + rr];
            t.re[e] = ok ? x : 0.0;
        }
    }
}

// Tile store; `interior` (wave-uniform: all 16 rows inside the matrix and
// the whole strip inside nev) skips the per-row checks.
template <bool CPLX>
__device__ inline void store_tile(const Tile<CPLX>& t, double* __restrict__ Z, int64_t ldz,
                                  int64_t n, int64_t nev, int64_t row0, int64_t col,
                                  bool interior = false, bool coh = false)
{
    if (coh) {   // device-coherent stores (read by another workgroup)
        if (col >= nev) return;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r = row0 + 4 * e;
            if (r >= 0 && r < n) {
                if constexpr (CPLX) {
                    st_coh(Z + 2 * (col * ldz + r), t.re[e]);
                    st_coh(Z + 2 * (col * ldz + r) + 1, t.im[e]);
                } else {
                    st_coh(Z + col * ldz + r, t.re[e]);
                }
            }
        }
        return;
    }
    if (interior) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r = row0 + 4 * e;
            if constexpr (CPLX) {
                *(d2*)(Z + 2 * (col * ldz + r)) = d2{t.re[e], t.im[e]};
            } else {
                Z[col * ldz + r] = t.re[e];
            }
        }
        return;
    }
    if (col >= nev) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t r = row0 + 4 * e;
        if (r >= 0 && r < n) {
            if constexpr (CPLX) {
                *(d2*)(Z + 2 * (col * ldz + r)) = d2{t.re[e], t.im[e]};
            } else {
                Z[col * ldz + r] = t.re[e];
            }
        }
    }
}

// Spin (with s_sleep) until prog[idx] >= need.  A bounded wait: on the
// never-expected timeout the wave flags the error word and gives up.
__device__ inline bool wait_progress(int* prog, int idx, int need, unsigned* err, int lane)
{
    unsigned spins = 0;
    while (__hip_atomic_load(&prog[idx], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < need) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1u << 26)) {
            if (lane == 0) atomicOr(err, 1u);
            return false;
        }
    }
    return true;
}

// The same wait for a counter that only grows, with `seen` the last value
// this wave read from it: when that already satisfies the wait, the LDS
// round trip is skipped (the acquire that read `seen` also made visible
// everything released before any smaller value).
// Debug builds with TRBT_WAIT_JITTER (libtrbt_jitter.so, see build.py) delay
// every wave by a pseudo-random 0..15 sleep quanta (64 clocks each) in front
// of every wait, so that the hand-offs between waves run in many orders;
// results must stay bitwise the same.  Release builds compile it away.
__device__ inline void wait_jitter(int idx, int need)
{
#ifdef TRBT_WAIT_JITTER
    uint32_t h = (uint32_t)wall_clock64() * 2654435761u ^ (uint32_t)(idx * 40503 + need * 977);
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    const int r = __builtin_amdgcn_readfirstlane((int)(h & 15u));
    for (int k = 0; k < r; ++k) __builtin_amdgcn_s_sleep(1);
#else
    (void)idx;
    (void)need;
#endif
}

__device__ inline bool wait_counter(int* ctr, int idx, int need, unsigned* err, int lane,
                                    int& seen)
{
    wait_jitter(idx, need);
    if (seen >= need) return true;
    unsigned spins = 0;
    int v;
    while ((v = __hip_atomic_load(&ctr[idx], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) <
           need) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1u << 26)) {
            if (lane == 0) atomicOr(err, 1u);
            return false;
        }
    }
    seen = v;
    return true;
}

// The same wait on a progress counter in global memory, published by a wave
// of another workgroup (publish_global).  The data that workgroup handed
// over was stored device-coherently before the counter and is read
// device-coherently after it: the counter load has returned (and been
// waited for) before any of those loads issues, and the compiler may not
// move them above the wait.  (An agent-scope acquire fence would instead
// invalidate the whole L2 of this XCD each time.)
__device__ inline bool wait_global(const int* ctr, int need, unsigned* err, int lane, int& seen)
{
    wait_jitter(need, need);
    if (seen >= need) return true;
    unsigned spins = 0;
    int v;
    while ((v = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < need) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1u << 26)) {
            if (lane == 0) atomicOr(err, 1u);
            return false;
        }
    }
    asm volatile("" ::: "memory");
    seen = v;
    return true;
}

// Publish a progress value for another workgroup: every earlier memory
// operation of this wave (among them the device-coherent tile stores it
// hands over) completes first, then the counter is stored device-coherently.
// (An agent-scope release would write back the whole L2 of this XCD.)
__device__ inline void publish_global(int* ctr, int val)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_store(ctr, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Operand ring depth (chunks loaded ahead of use).  The ring position of a
// chunk is its index in the block's stream modulo D, and the ring runs on
// into the next block, so D must divide the chunk count per block.  Real
// blocks with one column tile (one MFMA per chunk) read a whole block ahead,
// with two tiles half a block; complex blocks (three MFMAs per chunk, two
// registers per slot) 8 chunks.
template <int NB, bool CPLX, int CT = 1>
__host__ __device__ constexpr int ring_depth()
{
    return CPLX ? 8 : (CT == 1 ? 8 : 4) * Geo<NB, CPLX>::NT;
}

// Operand chunks are read through a buffer resource holding the slot's
// operand stream (all of its blocks, contiguous): the per-lane offset is a
// constant register and the chunk offset a scalar, so the loads need no
// vector address arithmetic.
__device__ inline __amdgpu_buffer_rsrc_t stream_rsrc(const double* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), 0, (int)bytes,
                                             0x00020000);
}

__device__ inline double buffer_load_f64(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <bool CPLX, int D>
__device__ inline void load_chunk(__amdgpu_buffer_rsrc_t r, uint32_t boff, int c, int lane,
                                  double (&re)[D], double (&im)[D], int slot)
{
    constexpr uint32_t CH = CPLX ? 128 : 64;
    const uint32_t soff = boff + (uint32_t)c * CH * 8;
    re[slot] = buffer_load_f64(r, lane * 8, soff);
    if constexpr (CPLX) im[slot] = buffer_load_f64(r, lane * 8 + 512, soff);
}

// Per-workgroup LDS state of the strip pipeline.
//   prog[w]      blocks finished by wave w (slot-sequence encoding)
//   written[w]   hand-off tiles wave w has put into its exchange ring
//   consumed[w]  hand-off tiles of wave w's ring that wave w+1 has taken
//   ring[w][R]   wave w -> wave w+1 exchange ring of retired bottom tiles
// Consecutive waves of a workgroup hold consecutive slots of one round, so
// most hand-off tiles travel through LDS; only each slot's first NT retired
// tiles (the next slot's initial window), the slot's last block and the
// last wave's tiles (read by wave 0 in the next round) go through Z.
// LDS traffic counts in lgkmcnt, so it never holds up the waits for the
// operand stream the way a global store does (stores count in vmcnt).
template <int NB, int CT, bool CPLX, int NW>
struct StripLds {
    static constexpr int R = 3;                              // tiles per ring
    static constexpr int TD = 256 * (CPLX ? 2 : 1) * CT;     // doubles per tile set
    int prog[NW];
    int written[NW];
    int consumed[NW];
    double ring[NW > 1 ? NW - 1 : 1][R][TD];
    __device__ void reset()
    {
        if (threadIdx.x < NW) {
            prog[threadIdx.x] = 0;
            written[threadIdx.x] = 0;
            consumed[threadIdx.x] = 0;
        }
    }
};

template <bool CPLX, int CT>
__device__ inline void lds_put(double* __restrict__ dst, const Tile<CPLX> (&t)[CT], int lane)
{
    constexpr int NC = CPLX ? 2 : 1;
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            dst[((c * NC) * 4 + e) * 64 + lane] = t[c].re[e];
            if constexpr (CPLX) dst[((c * NC + 1) * 4 + e) * 64 + lane] = t[c].im[e];
        }
}

template <bool CPLX, int CT>
__device__ inline void lds_get(Tile<CPLX> (&t)[CT], const double* __restrict__ src, int lane)
{
    constexpr int NC = CPLX ? 2 : 1;
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            t[c].re[e] = src[((c * NC) * 4 + e) * 64 + lane];
            if constexpr (CPLX) t[c].im[e] = src[((c * NC + 1) * 4 + e) * 64 + lane];
        }
}

// Main blocked kernel.  Per block the operand stream is consumed in order:
//   chunks 0 .. 4NT-1       A1 chunk (h, u) = (c/4, c%4):   Y += A1 * Zwin
//   chunks 4NT .. 8NT-1     -V chunks:                       Zwin += (-V) * Y
//                           real: (u, h), u ascending, h descending;
//                           complex: (h, u), h descending, u ascending
// where h is a register tile.  Complex windows never move between registers
// (a loop-carried rotation would cost a register copy of the whole window per
// block): in the o-th block of a slot, window tile q (q = 0 at the top) lives
// in register tile (q + rot) mod NT with rot = (-o) mod NT, and the pack
// kernel stores every block's chunks in that order.  When the window slides,
// the bottom tile (register tile rot - 1) retires after GEMM2 and its
// registers take the next block's top tile.  Real windows (a third of the
// registers, and many short slots in batched use, where the hand-off latency
// counts) keep register tile = window tile: the last MFMA of each tile writes
// it one tile lower (zsh), and the bottom tile is handed off as soon as its
// last MFMA is done.
//
// blocked_strip runs the whole back-transformation of column strip `strip`
// (columns 16*CT*strip ..) with the NW waves of the calling workgroup; wsb
// is the problem's packed-block array, S the workgroup's LDS state, all zero
// on entry.  On the (never expected) time-out of a progress wait a wave sets
// *err and leaves.
//
// Slot groups: with ngroups = G > 1 the strip's slots are shared by G
// workgroups (group grp = 0 .. G-1) that run as one pipeline of NW*G waves:
// slot j goes to group (j / NW) mod G, wave j mod NW.  Wave 0's predecessor slot then
// sits in wave NW-1 of the previous group, another workgroup: that wave
// publishes its progress in gprog[its group] (global memory, agent-scope
// publish_global, after its tiles have gone to Z with device-coherent
// stores) and wave 0 waits on it (wait_global) and reads those tiles with
// device-coherent loads.  The G workgroups of a strip must run concurrently
// (a cooperative launch).
//
// With CKPT (the first pass of the adjoint), every block's input window is
// also written to ckpt (non-temporal stores: read once, much later, so they
// should not displace the operand stream in the caches), one 16x16 tile at a
// time in register order:
//   ckpt[((((b * NT + q) * nstrips + strip) * NC + plane) * 4 + e) * 64 + lane]
// b = the block's slot-major index, q = tile of the window, plane = real or
// imaginary part (NC = 2 complex, 1 real), e = element.
template <int NB, int CT, bool CPLX, int D, int NW, bool CKPT = false, bool ROT = CPLX,
          bool SG = false>
__device__ __attribute__((always_inline)) inline void blocked_strip(int64_t n, int64_t nev, const double* __restrict__ wsb,
                                     double* __restrict__ Z, int64_t ldz,
                                     unsigned* __restrict__ err, int64_t strip,
                                     StripLds<NB, CT, CPLX, NW>& S,
                                     double* __restrict__ ckpt = nullptr, int64_t nstrips = 0,
                                     int ngroups = 1, int grp = 0,
                                     int* __restrict__ gprog = nullptr)
{
    constexpr int XR = StripLds<NB, CT, CPLX, NW>::R;
    int* prog = S.prog;
    int xput = 0, xget = 0;   // exchange tiles this wave has put / taken so far
    // last values read from the counters this wave waits on (all only grow)
    int seen_prog = 0, seen_written = 0, seen_consumed = 0;
    static_assert(!CKPT || CT == 1, "checkpoints: one 16-column tile");
    static_assert(ROT || !CPLX, "complex windows rotate");
    using G = Geo<NB, CPLX>;
    constexpr int NT = G::NT;
    constexpr int NCH = 8 * NT;            // operand chunks per block
    static_assert(NCH % D == 0, "ring depth must divide the chunks per block");
    constexpr int64_t nt1 = NB / 16;

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const int64_t nblk = (n - 2 + KB - 1) / KB;
    const int64_t J = sweeps_in_stage(n, NB, 0);
    const int64_t col_base = strip * 16 * CT + (lane & 15);
    const bool cols_inside = (strip + 1) * 16 * CT <= nev;
    const int rsub = lane >> 4;
    const int wprev = (w + NW - 1) % NW;

    Tile<CPLX> zt[NT][CT];
    double ring_re[D], ring_im[D];
    // the predecessor of this wave's slots: wave w-1 of this workgroup, or
    // (wave 0 with slot groups) wave NW-1 of the previous group
    // (SG: compiled for slot groups; without it the cross-workgroup paths
    // are not generated at all)
    const bool pred_global = SG && ngroups > 1 && w == 0;
    const bool coh_out = SG && ngroups > 1 && w == NW - 1;   // tiles go to another group
    const int* gpred = pred_global ? gprog + (grp + ngroups - 1) % ngroups : nullptr;
    auto wait_pred = [&](int need) -> bool {
        return pred_global ? wait_global(gpred, need, err, lane, seen_prog)
                           : wait_counter(prog, wprev, need, err, lane, seen_prog);
    };

    for (int64_t j = (int64_t)grp * NW + w; j < J; j += (int64_t)NW * ngroups) {
        const int64_t t0 = j * nt1;
        // the slot's operand stream; blocks are PB doubles apart
        const __amdgpu_buffer_rsrc_t ops =
            stream_rsrc(wsb + (size_t)slot_base(j, nblk, nt1) * G::PB,
                        (uint32_t)((nblk - t0) * G::PB * sizeof(double)));
        uint32_t boff = 0;
        const int need0 = (int)((j - 1) * (nblk + 1));   // + t + 1: slot j-1 done block t
        if (j > 0 && !wait_pred(need0 + (int)t0 + 1)) return;
        int64_t p0 = n - 3 - KB * t0 - 15 + j * NB;
        // first block of the slot: window tile q in register tile q
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const bool inside = cols_inside && p0 + 16 * q >= 0 && p0 + 16 * q + 16 <= n;
#pragma unroll
            for (int c = 0; c < CT; ++c)
                load_tile<CPLX>(zt[q][c], Z, ldz, n, nev, p0 + 16 * q + rsub,
                                col_base + 16 * c, inside, pred_global);
        }
#pragma unroll
        for (int c = 0; c < D; ++c) load_chunk<CPLX, D>(ops, 0, c, lane, ring_re, ring_im, c);

        int rot = 0;   // register tile of the window's top tile (wave-uniform)
        for (int64_t t = t0; t < nblk; ++t, boff += G::PB * sizeof(double), p0 -= KB) {
            const bool has_next = t + 1 < nblk;
            const int ret = rot == 0 ? NT - 1 : rot - 1;   // register tile of the bottom tile
            // the top tile of the next block: slot j-1 must have retired it.
            // From wave w-1's exchange ring when it put it there (slot j-1 is
            // in the same round and this is not the tile of its last block),
            // else from Z.
            Tile<CPLX> znext[CT];
            const bool xin = has_next && w > 0 && t + 2 < nblk;
            if (xin) {
                if (!wait_counter(S.written, w - 1, xget + 1, err, lane, seen_written)) return;
                lds_get<CPLX, CT>(znext, &S.ring[w - 1][xget % XR][0], lane);
                ++xget;
            } else if (has_next) {
                if (j > 0 && !wait_pred(need0 + (int)t + 2)) return;
                const bool inside = cols_inside && p0 - 16 >= 0 && p0 <= n;
#pragma unroll
                for (int c = 0; c < CT; ++c)
                    load_tile<CPLX>(znext[c], Z, ldz, n, nev, p0 - 16 + rsub, col_base + 16 * c,
                                    inside, pred_global);
            }

            // operand chunk c of this block sits in ring slot c % D; as soon
            // as it has been read the slot is refilled with chunk c + D
            // (running into the next block).  (Refilling only after the
            // chunk's MFMAs saves register copies but makes the load wait for
            // the MFMA to read its operand: slower.)
            auto refill = [&](int c) {
                const int slot = c % D;
                if (c + D < NCH)
                    load_chunk<CPLX, D>(ops, boff, c + D, lane, ring_re, ring_im, slot);
                else if (has_next)
                    load_chunk<CPLX, D>(ops, boff + G::PB * sizeof(double), c + D - NCH, lane,
                                        ring_re, ring_im, slot);
            };
            bool xfail = false;
            Tile<CPLX> zsh[ROT ? 1 : NT + 1][CT];   // fixed window: the window after the slide
            auto store_bottom = [&](const Tile<CPLX> (&zb)[CT]) {   // the final bottom tile
                if (!has_next) return;
                // to wave w+1 through LDS: slot j+1 exists, is in this round, and
                // this is not one of the first NT tiles (its initial window)
                const bool xout = w < NW - 1 && j + 1 < J && t >= t0 + NT;
                if (xout) {
                    if (!wait_counter(S.consumed, w, xput - XR + 1, err, lane, seen_consumed)) {
                        xfail = true;
                        return;
                    }
                    lds_put<CPLX, CT>(&S.ring[w][xput % XR][0], zb, lane);
                    ++xput;
                    __hip_atomic_store(&S.written[w], xput, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    // complex: opaque to the optimizer, so that the
                    // addressing of this rare path is not hoisted out of the
                    // per-register-tile hand-off sites into every block
                    int64_t rb = p0 + 16 * (NT - 1);
                    if constexpr (CPLX) asm volatile("" : "+s"(rb));
                    const bool inside = cols_inside && rb >= 0 && rb + 16 <= n;
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc)
                        store_tile<CPLX>(zb[cc], Z, ldz, n, nev, rb + rsub, col_base + 16 * cc,
                                         inside, coh_out);
                }
            };

            if constexpr (ROT && !CPLX) {
                // Real, rotating window (two column tiles): GEMM1 by
                // register tile, then GEMM2 register tiles from NT-1 down,
                // u ascending; each operand chunk feeds CT MFMAs.
                Tile<CPLX> y[2][CT];
#pragma unroll
                for (int hp = 0; hp < 2; ++hp)
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc) y[hp][cc].re = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 4 * NT; ++c) {
                    const double ar = ring_re[c % D];
                    refill(c);
                    const int h = c / 4, u = c % 4;
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc)
                        y[h & 1][cc].re = mfma_n<0>(ar, zt[h][cc].re[u], y[h & 1][cc].re);
                }
#pragma unroll
                for (int cc = 0; cc < CT; ++cc) y[0][cc].re += y[1][cc].re;
                if constexpr (CKPT) {
                    // the block's input window (GEMM1 has only read it);
                    // window tile q sits in register tile (q + rot) mod NT
                    double* cp = ckpt + ((size_t)(slot_base(j, nblk, nt1) + t - t0) * NT *
                                             nstrips + strip) * 256 + lane;
#pragma unroll
                    for (int h = 0; h < NT; ++h) {
                        const int q = h >= rot ? h - rot : h + NT - rot;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            __builtin_nontemporal_store(
                                zt[h][0].re[e], &cp[(size_t)q * nstrips * 256 + e * 64]);
                    }
                }
#pragma unroll
                for (int c2 = 0; c2 < 4 * NT; ++c2) {
                    const int c = 4 * NT + c2;
                    const double ar = ring_re[c % D];
                    refill(c);
                    const int h = NT - 1 - c2 / 4, u = c2 % 4;
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc)
                        zt[h][cc].re = mfma_n<0>(ar, y[0][cc].re[u], zt[h][cc].re);
                }
            } else if constexpr (CPLX) {
                // Complex products with three real MFMAs each.
                // GEMM1 (Gauss): Y = A1 * Zwin from P1 = sum ax, P2 = sum by and
                // P3 = sum (a+b)(x+y), (a + ib)(x + iy) = (P1 - P2) + i(P3 - P1 - P2).
                d4 ya[CT], yb[CT], yc[CT];
#pragma unroll
                for (int cc = 0; cc < CT; ++cc) ya[cc] = yb[cc] = yc[cc] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 4 * NT; ++c) {
                    const double ar = ring_re[c % D], ai = ring_im[c % D];
                    refill(c);
                    const double as = ar + ai;
                    const int h = c / 4, u = c % 4;
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc) {
                        const double zr = zt[h][cc].re[u], zi = zt[h][cc].im[u];
                        ya[cc] = mfma_n<0>(ar, zr, ya[cc]);
                        yb[cc] = mfma_n<0>(ai, zi, yb[cc]);
                        yc[cc] = mfma_n<0>(as, zr + zi, yc[cc]);
                    }
                }
                if constexpr (CKPT) {
                    // the block's input window: GEMM1 has only read it and
                    // GEMM2 is about to overwrite it; window tile q sits in
                    // register tile (q + rot) mod NT
                    double* cp = ckpt + ((size_t)(slot_base(j, nblk, nt1) + t - t0) * NT *
                                             nstrips + strip) * 512 + lane;
#pragma unroll
                    for (int h = 0; h < NT; ++h) {
                        const int q = h >= rot ? h - rot : h + NT - rot;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            __builtin_nontemporal_store(
                                zt[h][0].re[e], &cp[(size_t)q * nstrips * 512 + e * 64]);
                            __builtin_nontemporal_store(
                                zt[h][0].im[e], &cp[(size_t)q * nstrips * 512 + 256 + e * 64]);
                        }
                    }
                }
                // GEMM2 in the other three-product form, which accumulates in
                // place: with -V = a + ib and Y = c + id,
                //   Re += (a+b)c - b(c+d),   Im += (a+b)c + a(d-c),
                // the B operands c = P1 - P2, -(c+d) = 2 P2 - P3, d-c = P3 - 2 P1.
                d4 yr[CT], ym[CT], yk[CT], kk[CT];
#pragma unroll
                for (int cc = 0; cc < CT; ++cc)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        yr[cc][e] = ya[cc][e] - yb[cc][e];
                        ym[cc][e] = __builtin_fma(2.0, yb[cc][e], -yc[cc][e]);
                        yk[cc][e] = __builtin_fma(-2.0, ya[cc][e], yc[cc][e]);
                    }
                // tile by tile (register tiles from NT-1 down), u ascending
#pragma unroll
                for (int c2 = 0; c2 < 4 * NT; ++c2) {
                    const int c = 4 * NT + c2;
                    const double ar = ring_re[c % D], ai = ring_im[c % D];
                    refill(c);
                    const double as = ar + ai;
                    const int h = NT - 1 - c2 / 4, u = c2 % 4;
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc) {
                        zt[h][cc].re = mfma_n<0>(ai, ym[cc][u], zt[h][cc].re);
                        zt[h][cc].im = mfma_n<0>(ar, yk[cc][u], zt[h][cc].im);
                        kk[cc] = mfma_n<0>(as, yr[cc][u], u == 0 ? d4{0.0, 0.0, 0.0, 0.0} : kk[cc]);
                        if (u == 3) {
                            zt[h][cc].re += kk[cc];
                            zt[h][cc].im += kk[cc];
                        }
                    }
                }
            } else {
                Tile<CPLX> y[2][CT];   // two partial sums: more independent MFMA chains
#pragma unroll
                for (int hp = 0; hp < 2; ++hp)
#pragma unroll
                    for (int c = 0; c < CT; ++c) y[hp][c].re = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const double ar = ring_re[c % D];
                    refill(c);
                    if constexpr (CKPT) {
                        // the block's input window: GEMM1 has only read it and
                        // GEMM2 is about to overwrite it (storing here rather
                        // than at the top of the block keeps the stores out of
                        // the way of the next tile's wait and load)
                        if (c == 4 * NT) {
                            double* cp = ckpt + ((size_t)(slot_base(j, nblk, nt1) + t - t0) * NT *
                                                 nstrips + strip) * 256 + lane;
#pragma unroll
                            for (int q = 0; q < NT; ++q)
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    __builtin_nontemporal_store(
                                        zt[q][0].re[e], &cp[(size_t)q * nstrips * 256 + e * 64]);
                        }
                    }
                    if (c < 4 * NT) {
                        // Y += A1(:, chunk) * Zwin(chunk, :)
                        const int h = c / 4, u = c % 4, hp = h & 1;
#pragma unroll
                        for (int cc = 0; cc < CT; ++cc)
                            y[hp][cc].re = mfma_n<0>(ar, zt[h][cc].re[u], y[hp][cc].re);
                        if (c == 4 * NT - 1) {
#pragma unroll
                            for (int cc = 0; cc < CT; ++cc) y[0][cc].re += y[1][cc].re;
                        }
                    } else {
                        // Zwin(tile q, :) += (-V)(tile q, chunk u) * Y(chunk u, :);
                        // the last pass (u = 3) writes tile q into zsh[q+1]
                        const int c2 = c - 4 * NT, u = c2 / NT, q = NT - 1 - c2 % NT;
#pragma unroll
                        for (int cc = 0; cc < CT; ++cc) {
                            const Tile<CPLX>& src = zt[q][cc];
                            Tile<CPLX>& dst = (u == 3) ? zsh[q + 1][cc] : zt[q][cc];
                            dst.re = mfma_n<0>(ar, y[0][cc].re[u], src.re);
                        }
                        if (u == 3 && q == NT - 1) store_bottom(zsh[NT]);
                    }
                }
            }

            if constexpr (ROT) {
                // the bottom tile is final: hand it off; its registers take
                // the next block's top tile
#pragma unroll
                for (int h = 0; h < NT; ++h)
                    if (h == ret) {
                        store_bottom(zt[h]);
                        if (has_next) {
#pragma unroll
                            for (int c = 0; c < CT; ++c) zt[h][c] = znext[c];
                        }
                    }
            }
            if (xfail) return;
            if (!has_next) {
                // the slot's last block: the whole window is final
#pragma unroll
                for (int h = 0; h < NT; ++h) {
                    const int q = h >= rot ? h - rot : h + NT - rot;
#pragma unroll
                    for (int c = 0; c < CT; ++c) {
                        if constexpr (ROT)
                            store_tile<CPLX>(zt[h][c], Z, ldz, n, nev, p0 + 16 * q + rsub,
                                             col_base + 16 * c, false, coh_out);
                        else
                            store_tile<CPLX>(zsh[h + 1][c], Z, ldz, n, nev, p0 + 16 * h + rsub,
                                             col_base + 16 * c, false, coh_out);
                    }
                }
            }
            if (xin)   // the exchange tile read at the start of this block is in registers
                __hip_atomic_store(&S.consumed[w - 1], xget, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_store(&prog[w], (int)(j * (nblk + 1) + t + 1), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
            if (coh_out)   // the next group's wave 0 waits on this
                publish_global(&gprog[grp], (int)(j * (nblk + 1) + t + 1));
            if constexpr (ROT) {
                rot = ret;
            } else if (has_next) {
#pragma unroll
                for (int q = 1; q < NT; ++q)
#pragma unroll
                    for (int c = 0; c < CT; ++c) zt[q][c] = zsh[q][c];
#pragma unroll
                for (int c = 0; c < CT; ++c) zt[0][c] = znext[c];
            }
        }
    }
}

// One workgroup per (strip, slot group).  With G > 1 the G workgroups of a
// strip are numbered so that they land on one XCD (workgroups are handed to
// the 8 XCDs in turn): workgroup b is XCD b % 8's (b / 8)-th, strip
// ((b / 8) / G) * 8 + b % 8, group (b / 8) % G; the grid is padded to a
// multiple of 8 strips and the workgroups of padding strips leave at once.
// gprog: G progress counters per strip (zero on entry).
template <int NB, int CT, bool CPLX, int D, int NW, bool ROT = CPLX, bool SG = false>
__global__ __launch_bounds__(64 * NW) void k_blocked(int64_t n, int64_t nev,
                                                     const double* __restrict__ ws,
                                                     double* __restrict__ Z, int64_t ldz,
                                                     unsigned* __restrict__ err, int G,
                                                     int* __restrict__ gprog)
{
    __shared__ StripLds<NB, CT, CPLX, NW> S;
    int64_t strip = blockIdx.x;
    int g = 0;
    if (SG && G > 1) {
        const int64_t i = blockIdx.x / 8;
        strip = (i / G) * 8 + blockIdx.x % 8;
        g = (int)(i % G);
        if (strip * 16 * CT >= nev) return;
    }
    S.reset();
    __syncthreads();
    blocked_strip<NB, CT, CPLX, D, NW, false, ROT, SG>(n, nev, ws + HDR_BYTES / sizeof(double),
                                                       Z, ldz, err, strip, S, nullptr, 0, G, g,
                                                       SG && G > 1 ? gprog + strip * G : nullptr);
}

__global__ void k_zero_words(unsigned* p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// --------------------------------------------------------------------------
// Host-side helpers shared by the entry points
// --------------------------------------------------------------------------
inline int check_device()
{
    // The device capability is looked up once per device id and cached.
    static int cached[64];   // 0 unknown, 1 gfx950, 2 other
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TRBT_ERR_HIP;
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev] == 1 ? TRBT_SUCCESS : TRBT_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return TRBT_ERR_HIP;
    const int ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (dev >= 0 && dev < 64) cached[dev] = ok ? 1 : 2;
    return ok ? TRBT_SUCCESS : TRBT_ERR_DEVICE;
}

// Band widths with blocked kernels in every form (single problem, batched,
// adjoint).
inline bool blocked_eligible(int nbw) { return nbw == 16 || nbw == 32 || nbw == 48 || nbw == 64; }

// Band widths with a blocked single-problem forward kernel: every multiple
// of 16 up to 128.
inline bool apply_eligible(int nbw) { return nbw % 16 == 0 && nbw >= 16 && nbw <= 128; }

// Doubles per packed block: the pack kernel's layout, Geo<NB, CPLX>::PB, is
// the only definition (workspace sizes and stream limits derive from it).
inline int64_t packed_block_doubles(int nbw, bool cplx)
{
    switch (nbw) {
        case 16: return cplx ? Geo<16, true>::PB : Geo<16, false>::PB;
        case 32: return cplx ? Geo<32, true>::PB : Geo<32, false>::PB;
        case 48: return cplx ? Geo<48, true>::PB : Geo<48, false>::PB;
        case 64: return cplx ? Geo<64, true>::PB : Geo<64, false>::PB;
        case 80: return cplx ? Geo<80, true>::PB : Geo<80, false>::PB;
        case 96: return cplx ? Geo<96, true>::PB : Geo<96, false>::PB;
        case 112: return cplx ? Geo<112, true>::PB : Geo<112, false>::PB;
        case 128: return cplx ? Geo<128, true>::PB : Geo<128, false>::PB;
        default: return 0;
    }
}

// The blocked kernels address one slot's operand stream (at most
// ceil((n-2)/16) blocks) through a 32-bit buffer range.
inline bool blocked_fits(int64_t n, int nbw, bool cplx)
{
    const int64_t nblk = (n - 2 + KB - 1) / KB;
    return nblk * packed_block_doubles(nbw, cplx) * (int64_t)sizeof(double) < ((int64_t)1 << 31);
}

// Problems the blocked (compact-WY, MFMA) kernels take; the rest run the
// unblocked ones.
inline bool use_blocked(int64_t n, int nbw, bool cplx)
{
    return blocked_eligible(nbw) && blocked_fits(n, nbw, cplx);
}

// The same for the single-problem forward transformation.
inline bool use_blocked_apply(int64_t n, int nbw, bool cplx)
{
    return apply_eligible(nbw) && blocked_fits(n, nbw, cplx);
}

inline size_t blocked_bytes(int64_t n, int nbw, bool cplx)
{
    return HDR_BYTES +
           (size_t)blocked_num_blocks(n, nbw) * (size_t)packed_block_doubles(nbw, cplx) *
               sizeof(double);
}

inline int validate(int64_t n, int nbw, int64_t nev, const void* hv, const void* ht,
                    const void* Z, int64_t ldz, const void* work, size_t work_bytes)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (nev < 0 || nev > n) return -3;
    const int64_t K = num_reflectors(n, nbw);
    const bool active = K > 0 && nev > 0;
    if (active && !hv) return -4;
    if (active && !ht) return -5;
    if (nev > 0 && n > 0 && !Z) return -6;
    if (ldz < (n > 1 ? n : 1)) return -7;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -8;
    if (work_bytes && !work) return -8;
    (void)work_bytes;
    return TRBT_SUCCESS;
}

}  // namespace
