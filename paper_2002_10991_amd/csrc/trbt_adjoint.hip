// trbt_adjoint.hip -- adjoint (reverse-mode derivative) of the real
// tridiagonal-to-banded eigenvector back-transformation on MI355X (gfx950).
//
// Forward map (Yu et al., CPC 2020, Eq. 2stage_bkwd1, real reflectors):
//     Z_out = H_0 H_1 ... H_{K-1} Z_in,   H_k = I - tau_k v_k v_k^T.
// Given G = dL/dZ_out the adjoint returns dL/dZ_in = H_{K-1}^T ... H_0^T G
// (in place in G), dL/dv (K x nbw) and dL/dtau (K).  Per reflector, with z
// the rows of the state entering H_k in the forward pass and g the current
// gradient rows:  gk = v.g, wk = v.z, dtau = -sum_c gk wk,
// dv = -tau sum_c (wk g + gk z), and g <- g - tau gk v.
//
// Blocked path (nbw in {16, 32, 48, 64}): the reflectors of one slot over
// 16 consecutive stages form one compact-WY block Q = H_0..H_15 = I - V T V^T
// (generation order p = 0..15 inside the block).  With X the block's input
// window (80 rows for nbw 64) and Go the gradient on its output window:
//   w_p  = v_p^T Z^(p+1) = (R^T V^T X)_p      R[:,p] = e_p - [0; T_{>p}^T M_{>p,p}]
//   g_p  = v_p^T G^(p)   = (S^T V^T Go)_p     S[:,p] = e_p - [T_{<p} M_{<p,p}; 0]
//   Gi   = Q^T Go        = Go - V (T^T V^T Go)
//   dv_p = -tau_p [ (I - V_{<p} T_{<p}^T V_{<p}^T) P1_p
//                 + (I - V_{>p} T_{>p}   V_{>p}^T) P2_p ]   on v_p's rows,
//   P1 = Go W, P2 = X g  (sums over columns),  dtau_p = -sum_c g_p w_p,
// M = V^T V.  The intermediate states inside a block are never formed: the
// block's input window is the checkpoint (one per slot every 16 stages),
// written by a first forward pass.  The backward sweep walks every slot's
// blocks from the lowest stages up (the window slides down one tile per
// block) in a wave pipeline that mirrors the forward one, propagating only
// the gradient (Gi) and saving each block's Go like a checkpoint.  A
// reduction pass then takes one block per workgroup: it forms w, g and the
// column sums P1, P2, dtau over all column strips in registers (fixed order,
// so results are deterministic) and applies the corrections.  No per-strip
// partial sums cross memory.
//
// Streaming path (any nbw): one lane per column; the column's state is
// checkpointed at the start of every 16-stage block, each block is
// recomputed into a tape of per-reflector input rows, and the reverse sweep
// reduces dv and dtau over the 64 columns of a wave through LDS.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include "trbt.h"
#include "trbt_device.h"

namespace {

// ==========================================================================
// Blocked adjoint
// ==========================================================================
template <int NB>
struct AdjGeo {
    static constexpr int NT = NB / 16 + 1;               // tiles per window
    static constexpr int VT_OFF = 0;                     // V^T chunks (q,u) at 4q+u
    static constexpr int NV_OFF = 4 * NT * 64;           // -V chunks  (q,u) at 4q+u
    static constexpr int RT_OFF = 8 * NT * 64;           // R^T chunks u = 0..3
    static constexpr int ST_OFF = RT_OFF + 256;          // S^T chunks
    static constexpr int TT_OFF = ST_OFF + 256;          // T^T chunks
    static constexpr int T_OFF = TT_OFF + 256;           // T, row major 16 x 16
    static constexpr int TAU_OFF = T_OFF + 256;          // tau_p
    static constexpr int APB = (TAU_OFF + 16 + 31) / 32 * 32;   // doubles per block
};

// Operand pack for the backward pass: one workgroup (256 threads) per block.
// MFMA A-operand chunks (lane i + 16k holds A[i][k]):
//   V^T chunk (q, u):   V^T[i][16q + 4u + k]     (K runs over window rows)
//   -V chunk (q, u):    -V[16q + i][4u + k]      (K runs over reflectors)
//   R^T, S^T, T^T chunk u: X^T[i][4u + k] = X[4u + k][i]
template <int NB>
__global__ __launch_bounds__(256) void k_pack_adj(int64_t n, const double* __restrict__ hv,
                                                  const double* __restrict__ ht,
                                                  double* __restrict__ apk)
{
    using A = AdjGeo<NB>;
    constexpr int NT = A::NT;
    __shared__ WyBlock<NB, false> W;
    __shared__ double Rm[16][17], Sm[16][17];
    wy_factor<NB, false>(n, hv, ht, blockIdx.x, W);
    const int tid = threadIdx.x;
    {
        const int a = tid / 16, p = tid % 16;
        double r = (a == p) ? 1.0 : 0.0, s = r;
        for (int a2 = p + 1; a2 <= a; ++a2) r -= W.Tm[a2][a][0] * W.Gm[a2][p][0];
        for (int a2 = a; a2 < p; ++a2) s -= W.Tm[a][a2][0] * W.Gm[a2][p][0];
        Rm[a][p] = r;
        Sm[a][p] = s;
    }
    __syncthreads();
    double* out = apk + (size_t)blockIdx.x * A::APB;
    for (int idx = tid; idx < 4 * NT * 64; idx += 256) {
        const int lane = idx % 64, c = idx / 64, q = c / 4, u = c % 4;
        out[A::VT_OFF + idx] = W.Vt[16 * q + 4 * u + lane / 16][lane % 16][0];
        out[A::NV_OFF + idx] = -W.Vt[16 * q + lane % 16][4 * u + lane / 16][0];
    }
    {
        const int lane = tid % 64, u = tid / 64, i = lane % 16, k = lane / 16;
        out[A::RT_OFF + tid] = Rm[4 * u + k][i];
        out[A::ST_OFF + tid] = Sm[4 * u + k][i];
        out[A::TT_OFF + tid] = W.Tm[4 * u + k][i][0];
        out[A::T_OFF + tid] = W.Tm[tid / 16][tid % 16][0];
    }
    if (tid < 16) out[A::TAU_OFF + tid] = W.tau[tid][0];
}

// First pass: the forward transformation of a scratch copy of Z_in that
// also checkpoints every block's input window.
template <int NB, int NW>
__global__ __launch_bounds__(64 * NW) void k_blocked_ckpt(int64_t n, int64_t nev,
                                                          const double* __restrict__ blocks,
                                                          double* __restrict__ Z, int64_t ldz,
                                                          double* __restrict__ ckpt,
                                                          unsigned* __restrict__ err)
{
    __shared__ StripLds<NB, 1, false, NW> S;
    S.reset();
    __syncthreads();
    blocked_strip<NB, 1, false, ring_depth<NB, false>(), NW, true>(
        n, nev, blocks, Z, ldz, err, blockIdx.x, S, ckpt, gridDim.x);
}

// Lane-to-lane exchange through LDS inside one wave: the wave's LDS
// operations complete in order, so only the compiler must keep the writes
// before the reads (wavefront-scope fences emit no wait instruction).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Backward sweep.  Workgroup = one 16-column strip, NW waves = NW slots in
// flight.  Slot j runs its blocks t = nblk-1 down to j*nbw/16; block (t, j)
// needs (t+1, j) (same wave, earlier) and (t, j+1), whose retired top tile
// is this block's new bottom tile.  Slot j is handled by wave
// (J-1-j) mod NW, so slot j+1 is on the previous wave.  Per block the
// gradient window Go becomes Gi = Q^T Go = Go - V (T^T (V^T Go)), and Go is
// saved to gck in the checkpoint layout for the reduction pass.
// Hand-off: a retired top tile goes to the next wave through an LDS ring
// (counters written/consumed, back-pressure of XR tiles) when that wave holds
// slot j-1 in the same round; through G (with the prog counters) for the
// slot's first block (the next slot loads its first window from G), its last
// block (the whole window is final) and across rounds.
// Per-workgroup LDS state of the sweep: progress counters and the
// wave-to-wave exchange ring (zero counters on entry).
template <int NW>
struct SweepLds {
    static constexpr int XR = 3;
    int prog[NW], written[NW], consumed[NW];
    double ring[NW - 1][XR][256];
    __device__ void reset()
    {
        if (threadIdx.x < NW) prog[threadIdx.x] = written[threadIdx.x] = consumed[threadIdx.x] = 0;
    }
};

template <int NB, int NW>
__device__ __attribute__((always_inline)) inline void adj_sweep_strip(int64_t n, int64_t nev, const double* __restrict__ apk,
                                       double* __restrict__ G, int64_t ldg,
                                       double* __restrict__ gck, unsigned* __restrict__ err,
                                       int64_t strip, int64_t nstrips, SweepLds<NW>& S)
{
    using A = AdjGeo<NB>;
    constexpr int NT = A::NT;
    constexpr int64_t nt1 = NB / 16;
    constexpr int XR = SweepLds<NW>::XR;
    int* prog = S.prog;
    int* written = S.written;
    int* consumed = S.consumed;
    auto& ring = S.ring;

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nblk = (n - 2 + KB - 1) / KB;
    const int64_t J = sweeps_in_stage(n, NB, 0);
    const int64_t col = strip * 16 + (lane & 15);
    const bool cols_inside = (strip + 1) * 16 <= nev;
    const int rsub = lane >> 4;
    const int wprev = (w + NW - 1) % NW;
    // last values read from the counters this wave waits on (all only grow)
    int seen = 0, seen_written = 0, seen_consumed = 0;
    int xput = 0, xget = 0;   // ring tiles put / taken so far

    Tile<false> g[NT];

    for (int64_t j = J - 1 - w; j >= 0; j -= NW) {
        const int64_t t0 = j * nt1;
        const bool has_succ = j + 1 < J;
        const int64_t t0s = (j + 1) * nt1;
        const int base = (int)((J - 1 - j) * (nblk + 1));    // + nblk - t after block t
        const int base_s = base - (int)(nblk + 1);           // the same for slot j+1
        if (has_succ && !wait_counter(prog, wprev, base_s + 1, err, lane, seen)) return;
        int64_t p0 = n - 3 - KB * (nblk - 1) - 15 + j * NB;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const bool inside = cols_inside && p0 + 16 * q >= 0 && p0 + 16 * q + 16 <= n;
            load_tile<false>(g[q], G, ldg, n, nev, p0 + 16 * q + rsub, col, inside);
        }

        for (int64_t t = nblk - 1; t >= t0; --t, p0 += KB) {
            const int64_t b = slot_base(j, nblk, nt1) + (t - t0);
            const double* __restrict__ pk = apk + (size_t)b * A::APB;
            // the block's operands are read ahead of its stores: loads issued
            // after stores wait for them (one in-order vector-memory counter)
            double vt[4 * NT], nv[4 * NT], tt[4];
#pragma unroll
            for (int c = 0; c < 4 * NT; ++c) {
                vt[c] = pk[A::VT_OFF + c * 64 + lane];
                nv[c] = pk[A::NV_OFF + c * 64 + lane];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) tt[u] = pk[A::TT_OFF + u * 64 + lane];
            // Go of this block, read once by the reduction pass: non-temporal
            double* __restrict__ gp = gck + ((size_t)b * NT * nstrips + strip) * 256 + lane;
#pragma unroll
            for (int q = 0; q < NT; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    __builtin_nontemporal_store(g[q].re[e], &gp[(size_t)q * nstrips * 256 + e * 64]);
            // Bt = V^T Go, Y = T^T Bt, Gi = Go - V Y
            d4 bt[2];
            bt[0] = bt[1] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4 * NT; ++c) {
                const int q = c >> 2, u = c & 3;
                bt[q & 1] = mfma(vt[c], g[q].re[u], bt[q & 1]);
            }
            const d4 Bt = bt[0] + bt[1];
            d4 Y = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int u = 0; u < 4; ++u) Y = mfma(tt[u], Bt[u], Y);
#pragma unroll
            for (int c = 0; c < 4 * NT; ++c) {
                const int q = c >> 2, u = c & 3;
                g[q].re = mfma(nv[c], Y[u], g[q].re);
            }
            // slide down: the top tile leaves for slot j-1, a new bottom tile
            // arrives from slot j+1 (or from G when slot j+1 has no block)
            if (t > t0) {
                if (w < NW - 1 && j >= 1 && t < nblk - 1) {   // to wave w+1 through LDS
                    if (!wait_counter(consumed, w, xput - XR + 1, err, lane, seen_consumed))
                        return;
                    double* dst = &ring[w][xput % XR][0];
#pragma unroll
                    for (int e = 0; e < 4; ++e) dst[e * 64 + lane] = g[0].re[e];
                    ++xput;
                    __hip_atomic_store(&written[w], xput, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    store_tile<false>(g[0], G, ldg, n, nev, p0 + rsub, col,
                                      cols_inside && p0 >= 0 && p0 + 16 <= n);
                }
                __hip_atomic_store(&prog[w], base + (int)(nblk - t), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
                for (int q = 0; q + 1 < NT; ++q) g[q] = g[q + 1];
                if (w > 0 && has_succ && t - 1 > t0s) {   // from wave w-1's ring
                    if (!wait_counter(written, w - 1, xget + 1, err, lane, seen_written)) return;
                    const double* src = &ring[w - 1][xget % XR][0];
#pragma unroll
                    for (int e = 0; e < 4; ++e) g[NT - 1].re[e] = src[e * 64 + lane];
                    ++xget;
                    __hip_atomic_store(&consumed[w - 1], xget, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    if (has_succ && t - 1 >= t0s &&
                        !wait_counter(prog, wprev, base_s + (int)(nblk - (t - 1)), err, lane,
                                      seen))
                        return;
                    const int64_t r = p0 + KB + 16 * (NT - 1);
                    const bool inside = cols_inside && r >= 0 && r + 16 <= n;
                    load_tile<false>(g[NT - 1], G, ldg, n, nev, r + rsub, col, inside);
                }
            } else {
#pragma unroll
                for (int q = 0; q < NT; ++q)
                    store_tile<false>(g[q], G, ldg, n, nev, p0 + 16 * q + rsub, col);
                __hip_atomic_store(&prog[w], base + (int)(nblk - t), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
}

template <int NB, int NW>
__global__ __launch_bounds__(64 * NW) void k_adj_sweep(int64_t n, int64_t nev,
                                                       const double* __restrict__ apk,
                                                       double* __restrict__ G, int64_t ldg,
                                                       double* __restrict__ gck,
                                                       unsigned* __restrict__ err)
{
    __shared__ SweepLds<NW> S;
    S.reset();
    __syncthreads();
    adj_sweep_strip<NB, NW>(n, nev, apk, G, ldg, gck, err, blockIdx.x, gridDim.x, S);
}

// The one-call adjoint runs the checkpointing forward and the sweep in one
// launch: they are independent (the sweep needs only G and the adjoint
// packs), and each has only one workgroup per column strip, so together
// they fill twice as many CUs.  Workgroups [0, ns) run the forward,
// [ns, 2 ns) the sweep.
template <int NB, int NW>
__global__ __launch_bounds__(64 * NW) void k_adj_fwd_sweep(int64_t n, int64_t nev,
                                                           const double* __restrict__ blocks,
                                                           double* __restrict__ Z, int64_t ldz,
                                                           double* __restrict__ ckpt,
                                                           const double* __restrict__ apk,
                                                           double* __restrict__ G, int64_t ldg,
                                                           double* __restrict__ gck,
                                                           unsigned* __restrict__ err)
{
    __shared__ union {
        StripLds<NB, 1, false, NW> f;
        SweepLds<NW> b;
    } U;
    const int64_t ns = gridDim.x / 2;
    if ((int64_t)blockIdx.x < ns) {
        U.f.reset();
        __syncthreads();
        blocked_strip<NB, 1, false, ring_depth<NB, false>(), NW, true>(
            n, nev, blocks, Z, ldz, err, blockIdx.x, U.f, ckpt, ns);
    } else {
        U.b.reset();
        __syncthreads();
        adj_sweep_strip<NB, NW>(n, nev, apk, G, ldg, gck, err, blockIdx.x - ns, ns, U.b);
    }
}

// Reduction pass: one workgroup per block, RW waves.  From the block's input
// window X (checkpoint) and output gradient Go of every column strip:
//   w = R^T (V^T X), g = S^T (V^T Go), dtau_p = -sum_c g_p w_p,
//   P1 = Go W, P2 = X g   (sums over all columns),
// each wave summing its strips (s = w, w + RW, ...) in registers and the waves
// then combined in wave order (the same result on every run); finally the
// column-independent corrections give dv and dtau of the block's reflectors.
template <int NB, int RW>
__global__ __launch_bounds__(64 * RW, 2) void k_adj_reduce(int64_t n, int64_t nstrips,
                                                        const double* __restrict__ apk,
                                                        const double* __restrict__ ckpt,
                                                        const double* __restrict__ gck,
                                                        double* __restrict__ dv,
                                                        double* __restrict__ dtau)
{
    static_assert(RW * 64 == 256, "the finishing steps use 256 threads");
    using A = AdjGeo<NB>;
    constexpr int NT = A::NT, R = 16 * NT;
    constexpr int64_t nt1 = NB / 16;
    __shared__ double tr[RW][2][16][17];   // per-wave transposes
    __shared__ double P1[R][17], P2[R][17], Vs[R][17];
    __shared__ double Ts[16][17], U1[16][17], U2[16][17], Cm[16][17];
    __shared__ double dts[16], taus[16];
    __shared__ int64_t s_j, s_t;

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rsub = lane >> 4, cl = lane & 15;
    const int64_t b = blockIdx.x;
    const int64_t nblk = (n - 2 + KB - 1) / KB;
    const int64_t J = sweeps_in_stage(n, NB, 0);
    if (tid == 0) {
        int64_t lo = 0, hi = J;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (slot_base(mid, nblk, nt1) <= b) lo = mid; else hi = mid;
        }
        s_j = lo;
        s_t = lo * nt1 + (b - slot_base(lo, nblk, nt1));
    }
    const double* pk = apk + (size_t)b * A::APB;
    double rt[4], st[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        rt[u] = pk[A::RT_OFF + u * 64 + lane];
        st[u] = pk[A::ST_OFF + u * 64 + lane];
    }
    double (*Ma)[17] = tr[w][0];
    double (*Mb)[17] = tr[w][1];
    d4 p1[NT], p2[NT], dg = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NT; ++q) p1[q] = p2[q] = d4{0.0, 0.0, 0.0, 0.0};

    for (int64_t s = w; s < nstrips; s += RW) {
        const size_t off = ((size_t)b * NT * nstrips + s) * 256 + lane;
        Tile<false> x[NT], go[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                x[q].re[e] = __builtin_nontemporal_load(&ckpt[off + (size_t)q * nstrips * 256 + e * 64]);
                go[q].re[e] = __builtin_nontemporal_load(&gck[off + (size_t)q * nstrips * 256 + e * 64]);
            }
        // Ax = V^T X, Bt = V^T Go (V^T chunks from L1/L2: shared by the waves)
        d4 ax[2], bt[2];
        ax[0] = ax[1] = bt[0] = bt[1] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 4 * NT; ++c) {
            const int q = c >> 2, u = c & 3;
            const double a = pk[A::VT_OFF + c * 64 + lane];
            ax[q & 1] = mfma(a, x[q].re[u], ax[q & 1]);
            bt[q & 1] = mfma(a, go[q].re[u], bt[q & 1]);
        }
        const d4 Ax = ax[0] + ax[1], Bt = bt[0] + bt[1];
        // W^T = R^T Ax, g^T = S^T Bt
        d4 Wt = d4{0.0, 0.0, 0.0, 0.0}, Gt = Wt;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            Wt = mfma(rt[u], Ax[u], Wt);
            Gt = mfma(st[u], Bt[u], Gt);
        }
        // chunk u of W^T and g^T (B operands) through an LDS transpose
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            Ma[rsub + 4 * e][cl] = Wt[e];
            Mb[rsub + 4 * e][cl] = Gt[e];
        }
        wave_lds_sync();
        double bw[4], bg[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            bw[u] = Ma[cl][4 * u + rsub];
            bg[u] = Mb[cl][4 * u + rsub];
        }
        wave_lds_sync();
        // g W^T: its diagonal is sum_c g_p w_p (bg read as the A operand is
        // chunk u of g, reflectors x columns)
#pragma unroll
        for (int u = 0; u < 4; ++u) dg = mfma(bg[u], bw[u], dg);
        // P1 += Go W, P2 += X g, tile by tile (Go and X transposed to A operands)
#pragma unroll
        for (int q = 0; q < NT; ++q) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                Ma[rsub + 4 * e][cl] = go[q].re[e];
                Mb[rsub + 4 * e][cl] = x[q].re[e];
            }
            wave_lds_sync();
            double ag[4], axx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ag[u] = Ma[cl][4 * u + rsub];
                axx[u] = Mb[cl][4 * u + rsub];
            }
            wave_lds_sync();
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                p1[q] = mfma(ag[u], bw[u], p1[q]);
                p2[q] = mfma(axx[u], bg[u], p2[q]);
            }
        }
    }
    // combine the waves in order: P1[16q + rsub + 4e][cl] is element e of
    // p1[q]; element (p, p) of g W^T sits in lane p + 16 (p % 4), element p / 4
    const int de = (cl - rsub) >> 2;
    const bool dlane = ((cl - rsub) & 3) == 0 && cl >= rsub;
    for (int ww = 0; ww < RW; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int q = 0; q < NT; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 16 * q + rsub + 4 * e;
                    P1[r][cl] = (ww ? P1[r][cl] : 0.0) + p1[q][e];
                    P2[r][cl] = (ww ? P2[r][cl] : 0.0) + p2[q][e];
                }
            if (dlane) {
                const double d = de == 0 ? dg[0] : de == 1 ? dg[1] : de == 2 ? dg[2] : dg[3];
                dts[cl] = (ww ? dts[cl] : 0.0) - d;
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < R * 16; idx += 256) {   // V[r][p] from the V^T chunks
        const int r = idx / 16, p = idx % 16;
        const int c = 4 * (r / 16) + (r % 16) / 4, l = p + 16 * (r % 4);
        Vs[r][p] = pk[A::VT_OFF + c * 64 + l];
    }
    Ts[tid / 16][tid % 16] = pk[A::T_OFF + tid];
    if (tid < 16) taus[tid] = pk[A::TAU_OFF + tid];
    __syncthreads();
    {
        const int a = tid / 16, p = tid % 16;
        double u1 = 0.0, u2 = 0.0;
        for (int r = 0; r < R; ++r) {
            u1 += Vs[r][a] * P1[r][p];
            u2 += Vs[r][a] * P2[r][p];
        }
        U1[a][p] = u1;
        U2[a][p] = u2;
    }
    __syncthreads();
    {
        const int a = tid / 16, p = tid % 16;
        double c = 0.0;
        if (a < p)
            for (int a2 = 0; a2 <= a; ++a2) c += Ts[a2][a] * U1[a2][p];
        if (a > p)
            for (int a2 = a; a2 < 16; ++a2) c += Ts[a][a2] * U2[a2][p];
        Cm[a][p] = c;
    }
    __syncthreads();
    const int64_t j = s_j, t = s_t;
    const int64_t s_top = n - 3 - KB * t;
    for (int idx = tid; idx < 16 * NB; idx += 256) {
        const int p = idx / NB, i = idx % NB;
        const int64_t s = s_top - 15 + p;
        if (s < 0 || s > n - 3 - j * NB) continue;   // no reflector in this position
        const int64_t k = stage_offset(n, NB, s) + j;
        const int64_t r0 = s + 1 + j * NB;
        const int len = (int)(n - r0 < NB ? n - r0 : NB);
        double val = 0.0;
        if (i < len) {
            const int r = p + 1 + i;
            double term = P1[r][p] + P2[r][p];
            for (int a = 0; a < 16; ++a) term -= Vs[r][a] * Cm[a][p];
            val = -taus[p] * term;
        }
        dv[k * NB + i] = val;
        if (i == 0) dtau[k] = dts[p];
    }
}

// ==========================================================================
// Streaming adjoint (any nbw): one lane per column
// ==========================================================================
__host__ __device__ inline int64_t blk_sbot(int64_t n, int64_t t)
{
    const int64_t stop = n - 3 - KB * t;
    return stop - 15 > 0 ? stop - 15 : 0;
}

// Reflectors of 16-stage block t in the forward order of the unblocked
// kernel (slot ascending, stage descending); f(k, r0, len) per reflector.
template <typename F>
__device__ inline void for_block_forward(int64_t n, int nbw, int64_t t, F&& f)
{
    const int64_t stop = n - 3 - KB * t, sbot = blk_sbot(n, t);
    const int64_t J = sweeps_in_stage(n, nbw, sbot);
    for (int64_t j = 0; j < J; ++j)
        for (int64_t s = stop; s >= sbot; --s) {
            if (j >= sweeps_in_stage(n, nbw, s)) continue;
            const int64_t r0 = s + 1 + j * nbw;
            f(stage_offset(n, nbw, s) + j, r0, (int)(n - r0 < nbw ? n - r0 : nbw));
        }
}

template <typename F>
__device__ inline void for_block_reverse(int64_t n, int nbw, int64_t t, F&& f)
{
    const int64_t stop = n - 3 - KB * t, sbot = blk_sbot(n, t);
    const int64_t J = sweeps_in_stage(n, nbw, sbot);
    for (int64_t j = J - 1; j >= 0; --j)
        for (int64_t s = sbot; s <= stop; ++s) {
            if (j >= sweeps_in_stage(n, nbw, s)) continue;
            const int64_t r0 = s + 1 + j * nbw;
            f(stage_offset(n, nbw, s) + j, r0, (int)(n - r0 < nbw ? n - r0 : nbw));
        }
}

__device__ inline void apply_real(double* z, const double* __restrict__ v, double tau, int len)
{
    double d = 0.0;
    for (int i = 0; i < len; ++i) d = fma(v[i], z[i], d);
    const double a = tau * d;
    for (int i = 0; i < len; ++i) z[i] = fma(-a, v[i], z[i]);
}

// Forward pass with a checkpoint of rows [sbot+1, n) at the start of every
// block, stored row-major (row-contiguous across columns):
//   ck[(cb_t + r - sbot_t - 1) * nev + c],  cb_t = sum_{t' < t} (n - sbot_t' - 1).
__global__ __launch_bounds__(64) void k_adj_stream_fwd(int64_t n, int nbw, int64_t nev,
                                                       const double* __restrict__ hv,
                                                       const double* __restrict__ ht,
                                                       double* __restrict__ Z, int64_t ldz,
                                                       double* __restrict__ ck)
{
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (c >= nev) return;
    double* z = Z + c * ldz;
    const int64_t nblk = (n - 2 + KB - 1) / KB;
    int64_t cb = 0;
    for (int64_t t = 0; t < nblk; ++t) {
        const int64_t rlo = blk_sbot(n, t) + 1;
        for (int64_t r = rlo; r < n; ++r) ck[(cb + r - rlo) * nev + c] = z[r];
        cb += n - rlo;
        for_block_forward(n, nbw, t, [&](int64_t k, int64_t r0, int len) {
            apply_real(z + r0, hv + k * nbw, ht[k], len);
        });
    }
}

constexpr int RCH = 32;   // dv entries reduced per LDS round

// Reverse pass: per block (lowest stages first) restore the checkpoint,
// recompute the block into the tape, then walk it backwards.  Per reflector
// the wave's 64 column contributions to dv (entries 0..len-1) and dtau
// (entry len) are summed through LDS and written as this wave's partial:
//   part[(wave * K + k) * (nbw + 1) + e]   (dtau at e = nbw).
__global__ __launch_bounds__(64) void k_adj_stream_bwd(int64_t n, int nbw, int64_t nev,
                                                       const double* __restrict__ hv,
                                                       const double* __restrict__ ht,
                                                       double* __restrict__ Zs,
                                                       const double* __restrict__ ck,
                                                       double* __restrict__ tape,
                                                       double* __restrict__ G, int64_t ldg,
                                                       double* __restrict__ part, int64_t K)
{
    __shared__ double red[64][RCH + 1];
    const int tid = threadIdx.x;
    const int64_t c = (int64_t)blockIdx.x * 64 + tid;
    const bool valid = c < nev;
    const int64_t cc = valid ? c : 0;
    double* z = Zs + cc * n;
    double* g = G + cc * ldg;
    const int64_t nblk = (n - 2 + KB - 1) / KB;
    int64_t cb = 0;
    for (int64_t t = 0; t < nblk; ++t) cb += n - blk_sbot(n, t) - 1;
    for (int64_t t = nblk - 1; t >= 0; --t) {
        const int64_t rlo = blk_sbot(n, t) + 1;
        cb -= n - rlo;
        int64_t pos = 0;
        if (valid) {
            for (int64_t r = rlo; r < n; ++r) z[r] = ck[(cb + r - rlo) * nev + c];
            for_block_forward(n, nbw, t, [&](int64_t k, int64_t r0, int len) {
                for (int i = 0; i < len; ++i) tape[(pos + i) * nev + c] = z[r0 + i];
                pos += len;
                apply_real(z + r0, hv + k * nbw, ht[k], len);
            });
        } else {
            for_block_forward(n, nbw, t, [&](int64_t, int64_t, int len) { pos += len; });
        }
        for_block_reverse(n, nbw, t, [&](int64_t k, int64_t r0, int len) {
            pos -= len;
            const double* v = hv + k * nbw;
            const double tau = ht[k];
            double gk = 0.0, wk = 0.0;
            if (valid)
                for (int i = 0; i < len; ++i) {
                    gk = fma(v[i], g[r0 + i], gk);
                    wk = fma(v[i], tape[(pos + i) * nev + c], wk);
                }
            for (int e0 = 0; e0 <= len; e0 += RCH) {
                for (int i = 0; i < RCH; ++i) {
                    const int e = e0 + i;
                    double val = 0.0;
                    if (valid && e < len)
                        val = -tau * (wk * g[r0 + e] + gk * tape[(pos + e) * nev + c]);
                    else if (valid && e == len)
                        val = -gk * wk;
                    red[tid][i] = val;
                }
                __syncthreads();
                if (tid < RCH && e0 + tid <= len) {
                    double s = 0.0;
                    for (int l = 0; l < 64; ++l) s += red[l][tid];
                    const int e = e0 + tid;
                    part[((int64_t)blockIdx.x * K + k) * (nbw + 1) + (e < len ? e : nbw)] = s;
                }
                __syncthreads();
            }
            if (valid)
                for (int i = 0; i < len; ++i) g[r0 + i] = fma(-tau * gk, v[i], g[r0 + i]);
        });
    }
}

// dv, dtau = sums of the waves' partials in wave order.
__global__ __launch_bounds__(256) void k_adj_stream_finish(int64_t n, int nbw, int64_t K,
                                                           int64_t nwaves,
                                                           const double* __restrict__ part,
                                                           double* __restrict__ dv,
                                                           double* __restrict__ dtau)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= K * (nbw + 1)) return;
    const int64_t k = idx / (nbw + 1);
    const int e = (int)(idx % (nbw + 1));
    // the reflector's stage: largest s with stage_offset(s) <= k
    int64_t lo = 0, hi = n - 2;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (stage_offset(n, nbw, mid) <= k) lo = mid; else hi = mid;
    }
    const int64_t j = k - stage_offset(n, nbw, lo);
    const int64_t r0 = lo + 1 + j * nbw;
    const int len = (int)(n - r0 < nbw ? n - r0 : nbw);
    if (e < nbw && e >= len) {
        dv[k * nbw + e] = 0.0;
        return;
    }
    double s = 0.0;
    for (int64_t w = 0; w < nwaves; ++w) s += part[(w * K + k) * (nbw + 1) + e];
    if (e == nbw) dtau[k] = s;
    else dv[k * nbw + e] = s;
}

__global__ void k_fill_zero(double* p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------
constexpr int ADJ_WAVES = 8;

struct AdjLayout {
    size_t zs = 0, fwd = 0, apk = 0, ckpt = 0, gck = 0, part = 0, tape = 0, total = 0;
    int64_t nblocks = 0, nstrips = 0, nwaves = 0;
};

size_t al(size_t x) { return (x + 255) / 256 * 256; }

int adj_tiles(int nbw) { return nbw / 16 + 1; }

int adj_apb(int nbw)
{
    switch (nbw) {
        case 16: return AdjGeo<16>::APB;
        case 32: return AdjGeo<32>::APB;
        case 48: return AdjGeo<48>::APB;
        default: return AdjGeo<64>::APB;
    }
}

AdjLayout adj_layout(int64_t n, int nbw, int64_t nev)
{
    AdjLayout L;
    size_t off = HDR_BYTES;
    L.zs = off;
    off = al(off + (size_t)n * nev * sizeof(double));
    if (use_blocked(n, nbw, false)) {
        const int nt = adj_tiles(nbw);
        L.nblocks = blocked_num_blocks(n, nbw);
        L.nstrips = (nev + 15) / 16;
        const size_t pb = (size_t)packed_block_doubles(nbw, false);
        L.fwd = off;
        off = al(off + (size_t)L.nblocks * pb * sizeof(double));
        L.apk = off;
        off = al(off + (size_t)L.nblocks * adj_apb(nbw) * sizeof(double));
        L.ckpt = off;
        off = al(off + (size_t)L.nblocks * nt * L.nstrips * 256 * sizeof(double));
        L.gck = off;   // every block's output-gradient window, checkpoint layout
        off = al(off + (size_t)L.nblocks * nt * L.nstrips * 256 * sizeof(double));
    } else {
        const int64_t nblk = (n - 2 + KB - 1) / KB;
        int64_t ckrows = 0, taperows = 0;
        for (int64_t t = 0; t < nblk; ++t) {
            const int64_t sbot = blk_sbot(n, t), stop = n - 3 - KB * t;
            ckrows += n - sbot - 1;
            int64_t rows = 0;   // sum of the block's reflector lengths
            for (int64_t s = sbot; s <= stop; ++s)
                rows += (n - s - 1) - (((n - s - 1) % nbw) == 1 ? 1 : 0);
            taperows = rows > taperows ? rows : taperows;
        }
        L.nwaves = (nev + 63) / 64;
        L.ckpt = off;
        off = al(off + (size_t)ckrows * nev * sizeof(double));
        L.tape = off;
        off = al(off + (size_t)taperows * nev * sizeof(double));
        L.part = off;
        off = al(off + (size_t)L.nwaves * num_reflectors(n, nbw) * (nbw + 1) * sizeof(double));
    }
    L.total = off;
    return L;
}

int adj_validate(int64_t n, int nbw, int64_t nev, const double* hv, const double* ht,
                 const double* Zin, int64_t ldz, const double* G, int64_t ldg, const double* dv,
                 const double* dtau, int ckpt_every, const void* work, size_t work_bytes)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (nev < 0 || nev > n) return -3;
    const int64_t K = num_reflectors(n, nbw);
    const bool cols = nev > 0 && n > 0;
    if (K > 0 && !hv) return -4;
    if (K > 0 && !ht) return -5;
    if (cols && K > 0 && !Zin) return -6;
    if (ldz < (n > 1 ? n : 1)) return -7;
    if (cols && K > 0 && !G) return -8;
    if (ldg < (n > 1 ? n : 1)) return -9;
    if (K > 0 && !dv) return -10;
    if (K > 0 && !dtau) return -11;
    if (ckpt_every != 0 && ckpt_every != 16) return -12;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -13;
    if (work_bytes && !work) return -13;
    return TRBT_SUCCESS;
}

// The adjoint in two halves.  adj_forward: the forward transformation of Z
// (in place) that also writes the checkpoints into the workspace;
// adj_backward: the reverse sweep from those checkpoints.
template <int NB>
void blocked_forward(int64_t n, int64_t nev, const double* hv, const double* ht, double* Z,
                     int64_t ldz, char* ws, const AdjLayout& L, hipStream_t st)
{
    double* fwd = (double*)(ws + L.fwd);
    const unsigned nb = (unsigned)L.nblocks, ns = (unsigned)L.nstrips;
    hipLaunchKernelGGL((k_pack<NB, false>), dim3(nb), dim3(256), 0, st, n, hv, ht, fwd);
    hipLaunchKernelGGL((k_blocked_ckpt<NB, ADJ_WAVES>), dim3(ns), dim3(64 * ADJ_WAVES), 0, st, n,
                       nev, (const double*)fwd, Z, ldz, (double*)(ws + L.ckpt), (unsigned*)ws);
}

template <int NB>
void blocked_backward(int64_t n, int64_t nev, const double* hv, const double* ht, double* G,
                      int64_t ldg, double* dv, double* dtau, char* ws, const AdjLayout& L,
                      hipStream_t st)
{
    double* apk = (double*)(ws + L.apk);
    double* gck = (double*)(ws + L.gck);
    const unsigned nb = (unsigned)L.nblocks, ns = (unsigned)L.nstrips;
    hipLaunchKernelGGL((k_pack_adj<NB>), dim3(nb), dim3(256), 0, st, n, hv, ht, apk);
    hipLaunchKernelGGL((k_adj_sweep<NB, ADJ_WAVES>), dim3(ns), dim3(64 * ADJ_WAVES), 0, st, n,
                       nev, (const double*)apk, G, ldg, gck, (unsigned*)ws);
    hipLaunchKernelGGL((k_adj_reduce<NB, 4>), dim3(nb), dim3(256), 0, st, n, (int64_t)ns,
                       (const double*)apk, (const double*)(ws + L.ckpt), (const double*)gck, dv,
                       dtau);
}

// Both halves in one go (the one-call adjoint): the checkpointing forward and
// the backward sweep share one launch, then the reduction.
template <int NB>
void blocked_both(int64_t n, int64_t nev, const double* hv, const double* ht, double* Z,
                  int64_t ldz, double* G, int64_t ldg, double* dv, double* dtau, char* ws,
                  const AdjLayout& L, hipStream_t st)
{
    double* fwd = (double*)(ws + L.fwd);
    double* apk = (double*)(ws + L.apk);
    double* gck = (double*)(ws + L.gck);
    const unsigned nb = (unsigned)L.nblocks, ns = (unsigned)L.nstrips;
    hipLaunchKernelGGL((k_pack<NB, false>), dim3(nb), dim3(256), 0, st, n, hv, ht, fwd);
    hipLaunchKernelGGL((k_pack_adj<NB>), dim3(nb), dim3(256), 0, st, n, hv, ht, apk);
    hipLaunchKernelGGL((k_adj_fwd_sweep<NB, ADJ_WAVES>), dim3(2 * ns), dim3(64 * ADJ_WAVES), 0,
                       st, n, nev, (const double*)fwd, Z, ldz, (double*)(ws + L.ckpt),
                       (const double*)apk, G, ldg, gck, (unsigned*)ws);
    hipLaunchKernelGGL((k_adj_reduce<NB, 4>), dim3(nb), dim3(256), 0, st, n, (int64_t)ns,
                       (const double*)apk, (const double*)(ws + L.ckpt), (const double*)gck, dv,
                       dtau);
}

int adj_forward(int64_t n, int nbw, int64_t nev, const double* hv, const double* ht, double* Z,
                int64_t ldz, char* ws, const AdjLayout& L, hipStream_t st)
{
    if (use_blocked(n, nbw, false)) {
        switch (nbw) {
            case 16: blocked_forward<16>(n, nev, hv, ht, Z, ldz, ws, L, st); break;
            case 32: blocked_forward<32>(n, nev, hv, ht, Z, ldz, ws, L, st); break;
            case 48: blocked_forward<48>(n, nev, hv, ht, Z, ldz, ws, L, st); break;
            case 64: blocked_forward<64>(n, nev, hv, ht, Z, ldz, ws, L, st); break;
            default: return TRBT_ERR_INTERNAL;
        }
    } else {
        hipLaunchKernelGGL(k_adj_stream_fwd, dim3((unsigned)L.nwaves), dim3(64), 0, st, n, nbw,
                           nev, hv, ht, Z, ldz, (double*)(ws + L.ckpt));
    }
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

int adj_backward(int64_t n, int nbw, int64_t nev, const double* hv, const double* ht,
                 double* G, int64_t ldg, double* dv, double* dtau, char* ws, const AdjLayout& L,
                 hipStream_t st)
{
    if (use_blocked(n, nbw, false)) {
        switch (nbw) {
            case 16: blocked_backward<16>(n, nev, hv, ht, G, ldg, dv, dtau, ws, L, st); break;
            case 32: blocked_backward<32>(n, nev, hv, ht, G, ldg, dv, dtau, ws, L, st); break;
            case 48: blocked_backward<48>(n, nev, hv, ht, G, ldg, dv, dtau, ws, L, st); break;
            case 64: blocked_backward<64>(n, nev, hv, ht, G, ldg, dv, dtau, ws, L, st); break;
            default: return TRBT_ERR_INTERNAL;
        }
    } else {
        const int64_t K = num_reflectors(n, nbw);
        const unsigned nw = (unsigned)L.nwaves;
        hipLaunchKernelGGL(k_adj_stream_bwd, dim3(nw), dim3(64), 0, st, n, nbw, nev, hv, ht,
                           (double*)(ws + L.zs), (const double*)(ws + L.ckpt),
                           (double*)(ws + L.tape), G, ldg, (double*)(ws + L.part), K);
        const int64_t cnt = K * (nbw + 1);
        hipLaunchKernelGGL(k_adj_stream_finish, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                           st, n, nbw, K, L.nwaves, (const double*)(ws + L.part), dv, dtau);
    }
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

int zero_grads(int64_t K, int nbw, double* dv, double* dtau, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((K * nbw + 255) / 256)), dim3(256), 0, st, dv,
                       K * nbw);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, dtau, K);
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

}  // namespace

extern "C" {

int trbt_adjoint_workspace_bytes_d(int64_t n, int nbw, int64_t nev, int ckpt_every,
                                   size_t* bytes)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (nev < 0 || nev > n) return -3;
    if (ckpt_every != 0 && ckpt_every != 16) return -4;
    if (!bytes) return -5;
    *bytes = (num_reflectors(n, nbw) > 0 && nev > 0) ? adj_layout(n, nbw, nev).total : 0;
    return TRBT_SUCCESS;
}

int trans_ev_tridi_to_band_adjoint_d(int64_t n, int nbw, int64_t nev, const double* hh_v,
                                     const double* hh_tau, const double* Z_in, int64_t ldz,
                                     double* G, int64_t ldg, double* dv, double* dtau,
                                     int ckpt_every, void* work, size_t work_bytes,
                                     void* stream)
{
    int rc = adj_validate(n, nbw, nev, hh_v, hh_tau, Z_in, ldz, G, ldg, dv, dtau, ckpt_every,
                          work, work_bytes);
    if (rc) return rc;
    const int64_t K = num_reflectors(n, nbw);
    if (K == 0) return TRBT_SUCCESS;   // dL/dZ_in = G, nothing else to write
    rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (nev == 0) return zero_grads(K, nbw, dv, dtau, st);
    const AdjLayout L = adj_layout(n, nbw, nev);
    if (!work || work_bytes < L.total) return TRBT_ERR_WORKSPACE;
    char* ws = (char*)work;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (unsigned*)work, 64);
    double* Zs = (double*)(ws + L.zs);
    if (hipMemcpy2DAsync(Zs, (size_t)n * sizeof(double), Z_in, (size_t)ldz * sizeof(double),
                         (size_t)n * sizeof(double), (size_t)nev, hipMemcpyDeviceToDevice,
                         st) != hipSuccess)
        return TRBT_ERR_HIP;
    if (use_blocked(n, nbw, false)) {
        switch (nbw) {
            case 16: blocked_both<16>(n, nev, hh_v, hh_tau, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
            case 32: blocked_both<32>(n, nev, hh_v, hh_tau, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
            case 48: blocked_both<48>(n, nev, hh_v, hh_tau, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
            case 64: blocked_both<64>(n, nev, hh_v, hh_tau, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
            default: return TRBT_ERR_INTERNAL;
        }
        return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
    }
    rc = adj_forward(n, nbw, nev, hh_v, hh_tau, Zs, n, ws, L, st);
    if (rc) return rc;
    return adj_backward(n, nbw, nev, hh_v, hh_tau, G, ldg, dv, dtau, ws, L, st);
}

int trans_ev_tridi_to_band_fwd_ckpt_d(int64_t n, int nbw, int64_t nev, const double* hh_v,
                                      const double* hh_tau, double* Z, int64_t ldz,
                                      int ckpt_every, void* work, size_t work_bytes, void* stream)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (nev < 0 || nev > n) return -3;
    const int64_t K = num_reflectors(n, nbw);
    const bool active = K > 0 && nev > 0;
    if (active && !hh_v) return -4;
    if (active && !hh_tau) return -5;
    if (active && !Z) return -6;
    if (ldz < (n > 1 ? n : 1)) return -7;
    if (ckpt_every != 0 && ckpt_every != 16) return -8;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -9;
    if (work_bytes && !work) return -9;
    if (!active) return TRBT_SUCCESS;
    int rc = check_device();
    if (rc) return rc;
    const AdjLayout L = adj_layout(n, nbw, nev);
    if (!work || work_bytes < L.total) return TRBT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (unsigned*)work, 64);
    return adj_forward(n, nbw, nev, hh_v, hh_tau, Z, ldz, (char*)work, L, st);
}

int trans_ev_tridi_to_band_bwd_ckpt_d(int64_t n, int nbw, int64_t nev, const double* hh_v,
                                      const double* hh_tau, double* G, int64_t ldg, double* dv,
                                      double* dtau, int ckpt_every, void* work,
                                      size_t work_bytes, void* stream)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (nev < 0 || nev > n) return -3;
    const int64_t K = num_reflectors(n, nbw);
    if (K > 0 && !hh_v) return -4;
    if (K > 0 && !hh_tau) return -5;
    if (K > 0 && nev > 0 && !G) return -6;
    if (ldg < (n > 1 ? n : 1)) return -7;
    if (K > 0 && !dv) return -8;
    if (K > 0 && !dtau) return -9;
    if (ckpt_every != 0 && ckpt_every != 16) return -10;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -11;
    if (work_bytes && !work) return -11;
    if (K == 0) return TRBT_SUCCESS;
    int rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (nev == 0) return zero_grads(K, nbw, dv, dtau, st);
    const AdjLayout L = adj_layout(n, nbw, nev);
    if (!work || work_bytes < L.total) return TRBT_ERR_WORKSPACE;
    return adj_backward(n, nbw, nev, hh_v, hh_tau, G, ldg, dv, dtau, (char*)work, L, st);
}

}  // extern "C"
