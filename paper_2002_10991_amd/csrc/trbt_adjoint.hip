// trbt_adjoint.hip -- adjoint (reverse-mode derivative) of the
// tridiagonal-to-banded eigenvector back-transformation on MI355X (gfx950):
// the real adjoint (blocked and streaming forms) and the blocked form of the
// complex one (conjugate-Wirtinger gradients, see trbt_adjoint_z.hip; every
// formula below holds with conj the identity for real data).
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
// 16 consecutive stages form one compact-WY block Q = H_0..H_15 = I - V T V^H
// (generation order p = 0..15 inside the block).  With X the block's input
// window (80 rows for nbw 64), Go the gradient on its output window,
// Z^(p+1) the state entering H_p and G^(p) the gradient leaving it:
//   w_p  = v_p^H Z^(p+1) = (R V^H X)_p    R[p][a] = delta - sum_{p<b<=a} M[p][b] T[b][a]
//   g_p  = v_p^H G^(p)   = (S V^H Go)_p   S[p][b] = delta - sum_{b<=a<p} M[p][a] conj(T[b][a])
//   Gi   = Q^H Go        = Go - V (T^H V^H Go)
//   dv_p = -conj(tau_p) (I - V_{<p} T_{<p}^H V_{<p}^H) P1_p
//          - tau_p (I - V_{>p} T_{>p} V_{>p}^H) P2_p      on v_p's rows,
//   P1 = Go W^H, P2 = X g^H  (sums over columns),  dtau_p = -sum_c conj(w_p) g_p,
// M = V^H V (Z^(p+1) = (I - V_{>p} T_{>p} V_{>p}^H) X and G^(p) =
// (I - V_{<p} T_{<p}^H V_{<p}^H) Go, the trailing and leading blocks of T
// being the factors of the trailing and leading reflectors).  The intermediate states inside a block are never formed: the
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
// Blocked adjoint (real and complex)
// ==========================================================================
template <int NB, bool CPLX = false>
struct AdjGeo {
    static constexpr int NT = NB / 16 + 1;               // tiles per window
    static constexpr int NC = CPLX ? 2 : 1;              // planes (re, im)
    static constexpr int CH = 64 * NC;                   // doubles per operand chunk
    static constexpr int VT_OFF = 0;                     // V^H chunks (q,u) at 4q+u
    static constexpr int NV_OFF = 4 * NT * CH;           // -V chunks  (q,u) at 4q+u
    static constexpr int RT_OFF = 8 * NT * CH;           // R chunks u = 0..3
    static constexpr int ST_OFF = RT_OFF + 4 * CH;       // S chunks
    static constexpr int TT_OFF = ST_OFF + 4 * CH;       // T^H chunks
    static constexpr int T_OFF = TT_OFF + 4 * CH;        // T, row major 16 x 16 (x NC)
    static constexpr int TAU_OFF = T_OFF + 256 * NC;     // tau_p (x NC)
    static constexpr int APB = (TAU_OFF + 16 * NC + 31) / 32 * 32;   // doubles per block
};

// D += A B on FP64 MFMA for real or complex operands (complex: four real
// products, the negate modifier giving -Im(A) Im(B)).
template <bool CPLX>
__device__ inline void cmma(double ar, double ai, double br, double bi, Tile<CPLX>& d)
{
    d.re = mfma(ar, br, d.re);
    if constexpr (CPLX) {
        d.re = mfma_n<1>(ai, bi, d.re);
        d.im = mfma(ar, bi, d.im);
        d.im = mfma(ai, br, d.im);
    } else {
        (void)ai;
        (void)bi;
    }
}

template <bool CPLX>
__device__ inline Tile<CPLX> tile_zero()
{
    Tile<CPLX> t;
    t.re = d4{0.0, 0.0, 0.0, 0.0};
    if constexpr (CPLX) t.im = t.re;
    return t;
}

template <bool CPLX>
__device__ inline Tile<CPLX> tile_add(const Tile<CPLX>& a, const Tile<CPLX>& b)
{
    Tile<CPLX> t;
    t.re = a.re + b.re;
    if constexpr (CPLX) t.im = a.im + b.im;
    return t;
}

template <bool CPLX>
__device__ inline double tim(const Tile<CPLX>& t, int e)
{
    if constexpr (CPLX) return t.im[e];
    (void)t;
    (void)e;
    return 0.0;
}

// Operand pack for the backward pass: one workgroup (256 threads) per block.
// MFMA A-operand chunks (lane i + 16k holds A[i][k]; complex chunks hold the
// real parts in lanes 0..63 and the imaginary parts after them):
//   V^H chunk (q, u):   conj(V[16q + 4u + k][i])   (K runs over window rows)
//   -V chunk (q, u):    -V[16q + i][4u + k]        (K runs over reflectors)
//   R, S, T^H chunk u:  X[i][4u + k]
// With M = V^H V and the block's factor T (Q = H_0 .. H_15 = I - V T V^H):
//   R[p][a] = delta_pa - sum_{p < b <= a} M[p][b] T[b][a]      (0 for a < p)
//   S[p][b] = delta_pb - sum_{b <= a < p} M[p][a] conj(T[b][a]) (0 for b > p)
// so that, per column, w = R (V^H X) holds v_p^H (state entering H_p) and
// g = S (V^H Go) holds v_p^H (gradient leaving H_p).
template <int NB, bool CPLX>
__global__ __launch_bounds__(256) void k_pack_adj(int64_t n, const double* __restrict__ hv,
                                                  const double* __restrict__ ht,
                                                  double* __restrict__ apk)
{
    using A = AdjGeo<NB, CPLX>;
    constexpr int NT = A::NT, NC = A::NC, CH = A::CH;
    __shared__ WyBlock<NB, CPLX> W;
    __shared__ double Rm[16][17][NC], Sm[16][17][NC];
    wy_factor<NB, CPLX>(n, hv, ht, blockIdx.x, W);
    const int tid = threadIdx.x;
    {
        const int p = tid / 16, a = tid % 16;
        double rr = (a == p) ? 1.0 : 0.0, ri = 0.0, sr = rr, si = 0.0;
        for (int b = p + 1; b <= a; ++b) {
            const double mr = W.Gm[p][b][0], tr = W.Tm[b][a][0];
            if constexpr (CPLX) {
                const double mi = W.Gm[p][b][NC - 1], ti = W.Tm[b][a][NC - 1];
                rr -= mr * tr - mi * ti;
                ri -= mr * ti + mi * tr;
            } else {
                rr -= mr * tr;
            }
        }
        for (int c = a; c < p; ++c) {   // S[p][a]: sum over a <= c < p
            const double mr = W.Gm[p][c][0], tr = W.Tm[a][c][0];
            if constexpr (CPLX) {
                const double mi = W.Gm[p][c][NC - 1], ti = -W.Tm[a][c][NC - 1];
                sr -= mr * tr - mi * ti;
                si -= mr * ti + mi * tr;
            } else {
                sr -= mr * tr;
            }
        }
        Rm[p][a][0] = rr;
        Sm[p][a][0] = sr;
        if constexpr (CPLX) {
            Rm[p][a][NC - 1] = ri;
            Sm[p][a][NC - 1] = si;
        }
    }
    __syncthreads();
    double* out = apk + (size_t)blockIdx.x * A::APB;
    for (int idx = tid; idx < 4 * NT * 64; idx += 256) {
        const int lane = idx % 64, c = idx / 64, q = c / 4, u = c % 4;
        const int r1 = 16 * q + 4 * u + lane / 16, p1 = lane % 16;
        const int r2 = 16 * q + lane % 16, p2 = 4 * u + lane / 16;
        out[A::VT_OFF + c * CH + lane] = W.Vt[r1][p1][0];
        out[A::NV_OFF + c * CH + lane] = -W.Vt[r2][p2][0];
        if constexpr (CPLX) {
            out[A::VT_OFF + c * CH + 64 + lane] = -W.Vt[r1][p1][NC - 1];
            out[A::NV_OFF + c * CH + 64 + lane] = -W.Vt[r2][p2][NC - 1];
        }
    }
    {
        const int lane = tid % 64, u = tid / 64, i = lane % 16, k = lane / 16;
        out[A::RT_OFF + u * CH + lane] = Rm[i][4 * u + k][0];
        out[A::ST_OFF + u * CH + lane] = Sm[i][4 * u + k][0];
        out[A::TT_OFF + u * CH + lane] = W.Tm[4 * u + k][i][0];
        if constexpr (CPLX) {
            out[A::RT_OFF + u * CH + 64 + lane] = Rm[i][4 * u + k][NC - 1];
            out[A::ST_OFF + u * CH + 64 + lane] = Sm[i][4 * u + k][NC - 1];
            out[A::TT_OFF + u * CH + 64 + lane] = -W.Tm[4 * u + k][i][NC - 1];
        }
#pragma unroll
        for (int pl = 0; pl < NC; ++pl)
            out[A::T_OFF + tid * NC + pl] = W.Tm[tid / 16][tid % 16][pl];
    }
    if (tid < 16) {
#pragma unroll
        for (int pl = 0; pl < NC; ++pl) out[A::TAU_OFF + tid * NC + pl] = W.tau[tid][pl];
    }
}

// First pass: the forward transformation of a scratch copy of Z_in that
// also checkpoints every block's input window.
// SG: slot groups (G workgroups per strip, numbered like k_blocked's, a
// cooperative launch; G progress counters per strip in gprog, zero on entry).
template <int NB, int NW, bool CPLX, bool SG = false>
__global__ __launch_bounds__(64 * NW) void k_blocked_ckpt(int64_t n, int64_t nev,
                                                          const double* __restrict__ blocks,
                                                          double* __restrict__ Z, int64_t ldz,
                                                          double* __restrict__ ckpt,
                                                          unsigned* __restrict__ err, int G = 1,
                                                          int* __restrict__ gprog = nullptr)
{
    __shared__ StripLds<NB, 1, CPLX, NW> S;
    const int64_t nstrips = (nev + 15) / 16;
    int64_t strip = blockIdx.x;
    int g = 0;
    if (SG && G > 1) {
        const int64_t i = blockIdx.x / 8;
        strip = (i / G) * 8 + blockIdx.x % 8;
        g = (int)(i % G);
        if (strip >= nstrips) return;
    }
    S.reset();
    __syncthreads();
    blocked_strip<NB, 1, CPLX, ring_depth<NB, CPLX>(), NW, true, rotating_window<NB, CPLX>(),
                  SG>(
        n, nev, blocks, Z, ldz, err, strip, S, ckpt, nstrips, G, g,
        SG && G > 1 ? gprog + strip * G : nullptr);
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
// gradient window Go becomes Gi = Q^H Go = Go - V (T^H (V^H Go)), and Go is
// saved to gck in the checkpoint layout for the reduction pass.
// Hand-off: a retired top tile goes to the next wave through an LDS ring
// (counters written/consumed, back-pressure of XR tiles) when that wave holds
// slot j-1 in the same round; through G (with the prog counters) for the
// slot's first block (the next slot loads its first window from G), its last
// block (the whole window is final) and across rounds.
// Per-workgroup LDS state of the sweep: progress counters and the
// wave-to-wave exchange ring (zero counters on entry).
template <int NW, bool CPLX>
struct SweepLds {
    static constexpr int XR = 3;
    static constexpr int TD = 256 * (CPLX ? 2 : 1);   // doubles per tile
    int prog[NW], written[NW], consumed[NW];
    double ring[NW - 1][XR][TD];
    __device__ void reset()
    {
        if (threadIdx.x < NW) prog[threadIdx.x] = written[threadIdx.x] = consumed[threadIdx.x] = 0;
    }
};

template <int NB, int NW, bool CPLX, bool SG = false>
__device__ __attribute__((always_inline)) inline void adj_sweep_strip(
    int64_t n, int64_t nev, const double* __restrict__ apk, double* __restrict__ G, int64_t ldg,
    double* __restrict__ gck, unsigned* __restrict__ err, int64_t strip, int64_t nstrips,
    SweepLds<NW, CPLX>& S, int ngroups = 1, int grp = 0, int* __restrict__ gprog = nullptr)
{
    using A = AdjGeo<NB, CPLX>;
    constexpr int NT = A::NT, NC = A::NC, CH = A::CH;
    constexpr int64_t nt1 = NB / 16;
    constexpr int XR = SweepLds<NW, CPLX>::XR;
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
    // Slot groups, as in blocked_strip: slot j goes to group ((J-1-j)/NW) mod
    // G, wave (J-1-j) mod NW; wave 0's predecessor (slot j+1) is wave NW-1
    // of the previous group, which hands its tiles over through G with
    // device-coherent stores and publishes its progress in gprog.
    const bool pred_global = SG && ngroups > 1 && w == 0;
    const bool coh_out = SG && ngroups > 1 && w == NW - 1;
    const int* gpred = pred_global ? gprog + (grp + ngroups - 1) % ngroups : nullptr;
    auto wait_pred = [&](int need) -> bool {
        return pred_global ? wait_global(gpred, need, err, lane, seen)
                           : wait_counter(prog, wprev, need, err, lane, seen);
    };

    Tile<CPLX> g[NT];

    for (int64_t j = J - 1 - ((int64_t)grp * NW + w); j >= 0; j -= (int64_t)NW * ngroups) {
        const int64_t t0 = j * nt1;
        const bool has_succ = j + 1 < J;
        const int64_t t0s = (j + 1) * nt1;
        const int base = (int)((J - 1 - j) * (nblk + 1));    // + nblk - t after block t
        const int base_s = base - (int)(nblk + 1);           // the same for slot j+1
        if (has_succ && !wait_pred(base_s + 1)) return;
        int64_t p0 = n - 3 - KB * (nblk - 1) - 15 + j * NB;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const bool inside = cols_inside && p0 + 16 * q >= 0 && p0 + 16 * q + 16 <= n;
            load_tile<CPLX>(g[q], G, ldg, n, nev, p0 + 16 * q + rsub, col, inside, pred_global);
        }

        for (int64_t t = nblk - 1; t >= t0; --t, p0 += KB) {
            const int64_t b = slot_base(j, nblk, nt1) + (t - t0);
            const double* __restrict__ pk = apk + (size_t)b * A::APB;
            // the block's operands are read ahead of its stores: loads issued
            // after stores wait for them (one in-order vector-memory counter)
            double vt[4 * NT][NC], nv[4 * NT][NC], tt[4][NC];
#pragma unroll
            for (int c = 0; c < 4 * NT; ++c)
#pragma unroll
                for (int pl = 0; pl < NC; ++pl) {
                    vt[c][pl] = pk[A::VT_OFF + c * CH + pl * 64 + lane];
                    nv[c][pl] = pk[A::NV_OFF + c * CH + pl * 64 + lane];
                }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int pl = 0; pl < NC; ++pl) tt[u][pl] = pk[A::TT_OFF + u * CH + pl * 64 + lane];
            // Go of this block, read once by the reduction pass: non-temporal
            double* __restrict__ gp = gck + ((size_t)b * NT * nstrips + strip) * 256 * NC + lane;
#pragma unroll
            for (int q = 0; q < NT; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    __builtin_nontemporal_store(g[q].re[e],
                                                &gp[(size_t)q * nstrips * 256 * NC + e * 64]);
                    if constexpr (CPLX)
                        __builtin_nontemporal_store(
                            g[q].im[e], &gp[(size_t)q * nstrips * 512 + 256 + e * 64]);
                }
            // Bt = V^H Go, Y = T^H Bt, Gi = Go - V Y
            Tile<CPLX> bt[2];
            bt[0] = bt[1] = tile_zero<CPLX>();
#pragma unroll
            for (int c = 0; c < 4 * NT; ++c) {
                const int q = c >> 2, u = c & 3;
                cmma<CPLX>(vt[c][0], vt[c][NC - 1], g[q].re[u], tim(g[q], u), bt[q & 1]);
            }
            const Tile<CPLX> Bt = tile_add(bt[0], bt[1]);
            Tile<CPLX> Y = tile_zero<CPLX>();
#pragma unroll
            for (int u = 0; u < 4; ++u) cmma<CPLX>(tt[u][0], tt[u][NC - 1], Bt.re[u], tim(Bt, u), Y);
#pragma unroll
            for (int c = 0; c < 4 * NT; ++c) {
                const int q = c >> 2, u = c & 3;
                cmma<CPLX>(nv[c][0], nv[c][NC - 1], Y.re[u], tim(Y, u), g[q]);
            }
            // slide down: the top tile leaves for slot j-1, a new bottom tile
            // arrives from slot j+1 (or from G when slot j+1 has no block)
            if (t > t0) {
                if (w < NW - 1 && j >= 1 && t < nblk - 1) {   // to wave w+1 through LDS
                    if (!wait_counter(consumed, w, xput - XR + 1, err, lane, seen_consumed))
                        return;
                    double* dst = &ring[w][xput % XR][0];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        dst[e * 64 + lane] = g[0].re[e];
                        if constexpr (CPLX) dst[256 + e * 64 + lane] = g[0].im[e];
                    }
                    ++xput;
                    __hip_atomic_store(&written[w], xput, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    store_tile<CPLX>(g[0], G, ldg, n, nev, p0 + rsub, col,
                                     cols_inside && p0 >= 0 && p0 + 16 <= n, coh_out);
                }
                __hip_atomic_store(&prog[w], base + (int)(nblk - t), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                if (coh_out) publish_global(&gprog[grp], base + (int)(nblk - t));
#pragma unroll
                for (int q = 0; q + 1 < NT; ++q) g[q] = g[q + 1];
                if (w > 0 && has_succ && t - 1 > t0s) {   // from wave w-1's ring
                    if (!wait_counter(written, w - 1, xget + 1, err, lane, seen_written)) return;
                    const double* src = &ring[w - 1][xget % XR][0];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        g[NT - 1].re[e] = src[e * 64 + lane];
                        if constexpr (CPLX) g[NT - 1].im[e] = src[256 + e * 64 + lane];
                    }
                    ++xget;
                    __hip_atomic_store(&consumed[w - 1], xget, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    if (has_succ && t - 1 >= t0s && !wait_pred(base_s + (int)(nblk - (t - 1))))
                        return;
                    const int64_t r = p0 + KB + 16 * (NT - 1);
                    const bool inside = cols_inside && r >= 0 && r + 16 <= n;
                    load_tile<CPLX>(g[NT - 1], G, ldg, n, nev, r + rsub, col, inside, pred_global);
                }
            } else {
#pragma unroll
                for (int q = 0; q < NT; ++q)
                    store_tile<CPLX>(g[q], G, ldg, n, nev, p0 + 16 * q + rsub, col, false,
                                     coh_out);
                __hip_atomic_store(&prog[w], base + (int)(nblk - t), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                if (coh_out) publish_global(&gprog[grp], base + (int)(nblk - t));
            }
        }
    }
}

template <int NB, int NW, bool CPLX, bool SG = false>
__global__ __launch_bounds__(64 * NW) void k_adj_sweep(int64_t n, int64_t nev,
                                                       const double* __restrict__ apk,
                                                       double* __restrict__ G, int64_t ldg,
                                                       double* __restrict__ gck,
                                                       unsigned* __restrict__ err, int NG = 1,
                                                       int* __restrict__ gprog = nullptr)
{
    __shared__ SweepLds<NW, CPLX> S;
    const int64_t nstrips = (nev + 15) / 16;
    int64_t strip = blockIdx.x;
    int g = 0;
    if (SG && NG > 1) {
        const int64_t i = blockIdx.x / 8;
        strip = (i / NG) * 8 + blockIdx.x % 8;
        g = (int)(i % NG);
        if (strip >= nstrips) return;
    }
    S.reset();
    __syncthreads();
    adj_sweep_strip<NB, NW, CPLX, SG>(n, nev, apk, G, ldg, gck, err, strip, nstrips, S, NG, g,
                                      SG && NG > 1 ? gprog + strip * NG : nullptr);
}

// The one-call adjoint runs the checkpointing forward and the sweep in one
// launch: they are independent (the sweep needs only G and the adjoint
// packs), and each has only one workgroup per column strip, so together
// they fill twice as many CUs.  Workgroups [0, ns) run the forward,
// [ns, 2 ns) the sweep.
template <int NB, int NW, bool CPLX>
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
        StripLds<NB, 1, CPLX, NW> f;
        SweepLds<NW, CPLX> b;
    } U;
    const int64_t ns = gridDim.x / 2;
    if ((int64_t)blockIdx.x < ns) {
        U.f.reset();
        __syncthreads();
        blocked_strip<NB, 1, CPLX, ring_depth<NB, CPLX>(), NW, true,
                      rotating_window<NB, CPLX>()>(
            n, nev, blocks, Z, ldz, err, blockIdx.x, U.f, ckpt, ns);
    } else {
        U.b.reset();
        __syncthreads();
        adj_sweep_strip<NB, NW, CPLX>(n, nev, apk, G, ldg, gck, err, blockIdx.x - ns, ns, U.b);
    }
}

// Reduction pass: one workgroup per block, RW waves.  From the block's input
// window X (checkpoint) and output gradient Go of every column strip:
//   w = R (V^H X), g = S (V^H Go), dtau_p = -sum_c conj(w_p) g_p,
//   P1 = Go W^H, P2 = X g^H   (sums over all columns),
// each wave summing its strips (s = w, w + RW, ...) in registers and the waves
// then combined in wave order (the same result on every run); finally the
// column-independent corrections
//   dv_p = -conj(tau_p) (I - V_<p T_<p^H V_<p^H) P1_p - tau_p (I - V_>p T_>p V_>p^H) P2_p
// on v_p's rows give dv and dtau of the block's reflectors (real: conj is
// the identity).
template <int NB, int RW, bool CPLX>
__global__ __launch_bounds__(64 * RW, CPLX ? 1 : 2) void k_adj_reduce(
    int64_t n, int64_t nstrips, const double* __restrict__ apk, const double* __restrict__ ckpt,
    const double* __restrict__ gck, double* __restrict__ dv, double* __restrict__ dtau)
{
    static_assert(RW * 64 == 256, "the finishing steps use 256 threads");
    using A = AdjGeo<NB, CPLX>;
    constexpr int NT = A::NT, NC = A::NC, CH = A::CH, R = 16 * NT;
    constexpr int64_t nt1 = NB / 16;
    // the per-wave transposes of the column loop and the combined sums after
    // it share one area
    __shared__ union {
        double tr[RW][2][NC][16][17];
        struct {
            double P1[R][16][NC], P2[R][16][NC];
        } f;
    } U;
    __shared__ double Vs[R][16][NC];
    __shared__ double Ts[16][17][NC], U1[16][17][NC], U2[16][17][NC], Cm[16][17][NC];
    __shared__ double dts[16][NC], taus[16][NC];
    __shared__ int64_t s_j, s_t;
    auto& P1 = U.f.P1;
    auto& P2 = U.f.P2;

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
    double rt[4][NC], st[4][NC];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int pl = 0; pl < NC; ++pl) {
            rt[u][pl] = CPLX ? 0.0 : pk[A::RT_OFF + u * CH + pl * 64 + lane];
            st[u][pl] = CPLX ? 0.0 : pk[A::ST_OFF + u * CH + pl * 64 + lane];
        }
    auto& Ma = U.tr[w][0];
    auto& Mb = U.tr[w][1];
    Tile<CPLX> p1[NT], p2[NT], dg = tile_zero<CPLX>();
#pragma unroll
    for (int q = 0; q < NT; ++q) p1[q] = p2[q] = tile_zero<CPLX>();

    // Complex: X and Go are not kept in registers between their two uses
    // (V^H X, V^H Go, then P1 and P2) but read again (from the caches: the
    // wave has just read them), which leaves the accumulators room without
    // spilling.
    constexpr bool KEEPX = !CPLX;
    // real: each tile is read once, non-temporally; complex: read twice, so
    // ordinary loads, which leave the tile in the caches for the second read
    // (non-temporal first reads made the second miss: 42.8 -> 41.2 ms for the
    // n = 4096, nev = 2048 forward + adjoint)
    auto load_t = [&](const double* __restrict__ src, size_t o, Tile<CPLX>& t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if constexpr (KEEPX) {
                t.re[e] = __builtin_nontemporal_load(&src[o + e * 64]);
            } else {
                t.re[e] = src[o + e * 64];
                t.im[e] = src[o + 256 + e * 64];
            }
        }
    };
    for (int64_t s = w; s < nstrips; s += RW) {
        const size_t off = ((size_t)b * NT * nstrips + s) * 256 * NC + lane;
        const size_t qstride = (size_t)nstrips * 256 * NC;
        // complex: the V^H chunks are read again for every strip (from L1/L2)
        // rather than held in registers across the loop
        const double* pkv = pk;
        if constexpr (!KEEPX) asm volatile("" : "+s"(pkv));
        Tile<CPLX> x[KEEPX ? NT : 1], go[KEEPX ? NT : 1];
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            if constexpr (KEEPX) {
                load_t(ckpt, off + q * qstride, x[q]);
                load_t(gck, off + q * qstride, go[q]);
            }
        }
        // Ax = V^H X, Bt = V^H Go (V^H chunks from L1/L2: shared by the waves)
        Tile<CPLX> ax[2], bt[2];
        ax[0] = ax[1] = bt[0] = bt[1] = tile_zero<CPLX>();
#pragma unroll
        for (int c = 0; c < 4 * NT; ++c) {
            const int q = c >> 2, u = c & 3;
            if (!KEEPX && u == 0) {
                load_t(ckpt, off + q * qstride, x[0]);
                load_t(gck, off + q * qstride, go[0]);
            }
            const Tile<CPLX>& xq = x[KEEPX ? q : 0];
            const Tile<CPLX>& gq = go[KEEPX ? q : 0];
            const double ar = pkv[A::VT_OFF + c * CH + lane];
            const double ai = CPLX ? pkv[A::VT_OFF + c * CH + 64 + lane] : 0.0;
            cmma<CPLX>(ar, ai, xq.re[u], tim(xq, u), ax[q & 1]);
            cmma<CPLX>(ar, ai, gq.re[u], tim(gq, u), bt[q & 1]);
        }
        const Tile<CPLX> Ax = tile_add(ax[0], ax[1]), Bt = tile_add(bt[0], bt[1]);
        // W = R Ax, g = S Bt (reflectors x columns)
        Tile<CPLX> Wt = tile_zero<CPLX>(), Gt = tile_zero<CPLX>();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if constexpr (!KEEPX) {
#pragma unroll
                for (int pl = 0; pl < NC; ++pl) {
                    rt[u][pl] = pkv[A::RT_OFF + u * CH + pl * 64 + lane];
                    st[u][pl] = pkv[A::ST_OFF + u * CH + pl * 64 + lane];
                }
            }
            cmma<CPLX>(rt[u][0], rt[u][NC - 1], Ax.re[u], tim(Ax, u), Wt);
            cmma<CPLX>(st[u][0], st[u][NC - 1], Bt.re[u], tim(Bt, u), Gt);
        }
        // chunk u of W and g through an LDS transpose: lane (j + 16k) holds
        // W[j][4u + k], the A operand of chunk u of W and the B operand of
        // chunk u of W^T (likewise g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            Ma[0][rsub + 4 * e][cl] = Wt.re[e];
            Mb[0][rsub + 4 * e][cl] = Gt.re[e];
            if constexpr (CPLX) {
                Ma[NC - 1][rsub + 4 * e][cl] = Wt.im[e];
                Mb[NC - 1][rsub + 4 * e][cl] = Gt.im[e];
            }
        }
        wave_lds_sync();
        double bw[4][NC], bg[4][NC];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int pl = 0; pl < NC; ++pl) {
                bw[u][pl] = Ma[pl][cl][4 * u + rsub];
                bg[u][pl] = Mb[pl][cl][4 * u + rsub];
            }
        wave_lds_sync();
        // g conj(W)^T: its diagonal is sum_c g_p conj(w_p)
#pragma unroll
        for (int u = 0; u < 4; ++u) cmma<CPLX>(bg[u][0], bg[u][NC - 1], bw[u][0], -bw[u][NC - 1], dg);
        // P1 += Go conj(W)^T, P2 += X conj(g)^T, tile by tile (Go and X
        // transposed to A operands)
        if constexpr (!KEEPX) asm volatile("" ::: "memory");   // read again, do not keep
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            if (!KEEPX) {
                load_t(ckpt, off + q * qstride, x[0]);
                load_t(gck, off + q * qstride, go[0]);
            }
            const Tile<CPLX>& xq = x[KEEPX ? q : 0];
            const Tile<CPLX>& gq = go[KEEPX ? q : 0];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                Ma[0][rsub + 4 * e][cl] = gq.re[e];
                Mb[0][rsub + 4 * e][cl] = xq.re[e];
                if constexpr (CPLX) {
                    Ma[NC - 1][rsub + 4 * e][cl] = gq.im[e];
                    Mb[NC - 1][rsub + 4 * e][cl] = xq.im[e];
                }
            }
            wave_lds_sync();
            double ag[4][NC], axx[4][NC];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int pl = 0; pl < NC; ++pl) {
                    ag[u][pl] = Ma[pl][cl][4 * u + rsub];
                    axx[u][pl] = Mb[pl][cl][4 * u + rsub];
                }
            wave_lds_sync();
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                cmma<CPLX>(ag[u][0], ag[u][NC - 1], bw[u][0], -bw[u][NC - 1], p1[q]);
                cmma<CPLX>(axx[u][0], axx[u][NC - 1], bg[u][0], -bg[u][NC - 1], p2[q]);
            }
        }
    }
    __syncthreads();   // every wave is done with its transposes (the sums reuse them)
    // combine the waves in order: P1[16q + rsub + 4e][cl] is element e of
    // p1[q]; element (p, p) of g conj(W)^T sits in lane p + 16 (p % 4),
    // element p / 4
    const int de = (cl - rsub) >> 2;
    const bool dlane = ((cl - rsub) & 3) == 0 && cl >= rsub;
    for (int ww = 0; ww < RW; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int q = 0; q < NT; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 16 * q + rsub + 4 * e;
                    P1[r][cl][0] = (ww ? P1[r][cl][0] : 0.0) + p1[q].re[e];
                    P2[r][cl][0] = (ww ? P2[r][cl][0] : 0.0) + p2[q].re[e];
                    if constexpr (CPLX) {
                        P1[r][cl][NC - 1] = (ww ? P1[r][cl][NC - 1] : 0.0) + p1[q].im[e];
                        P2[r][cl][NC - 1] = (ww ? P2[r][cl][NC - 1] : 0.0) + p2[q].im[e];
                    }
                }
            if (dlane) {
                const double dr = de == 0 ? dg.re[0] : de == 1 ? dg.re[1] : de == 2 ? dg.re[2] : dg.re[3];
                dts[cl][0] = (ww ? dts[cl][0] : 0.0) - dr;
                if constexpr (CPLX) {
                    const double di = de == 0 ? dg.im[0] : de == 1 ? dg.im[1] : de == 2 ? dg.im[2] : dg.im[3];
                    dts[cl][NC - 1] = (ww ? dts[cl][NC - 1] : 0.0) - di;
                }
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < R * 16; idx += 256) {   // V[r][p] from the V^H chunks
        const int r = idx / 16, p = idx % 16;
        const int c = 4 * (r / 16) + (r % 16) / 4, l = p + 16 * (r % 4);
        Vs[r][p][0] = pk[A::VT_OFF + c * CH + l];
        if constexpr (CPLX) Vs[r][p][NC - 1] = -pk[A::VT_OFF + c * CH + 64 + l];
    }
#pragma unroll
    for (int pl = 0; pl < NC; ++pl) Ts[tid / 16][tid % 16][pl] = pk[A::T_OFF + tid * NC + pl];
    if (tid < 16) {
#pragma unroll
        for (int pl = 0; pl < NC; ++pl) taus[tid][pl] = pk[A::TAU_OFF + tid * NC + pl];
    }
    __syncthreads();
    {   // U1 = V^H P1, U2 = V^H P2
        const int a = tid / 16, p = tid % 16;
        double u1r = 0.0, u1i = 0.0, u2r = 0.0, u2i = 0.0;
        for (int r = 0; r < R; ++r) {
            const double vr = Vs[r][a][0];
            if constexpr (CPLX) {
                const double vi = -Vs[r][a][NC - 1];   // conj
                u1r += vr * P1[r][p][0] - vi * P1[r][p][NC - 1];
                u1i += vr * P1[r][p][NC - 1] + vi * P1[r][p][0];
                u2r += vr * P2[r][p][0] - vi * P2[r][p][NC - 1];
                u2i += vr * P2[r][p][NC - 1] + vi * P2[r][p][0];
            } else {
                u1r += vr * P1[r][p][0];
                u2r += vr * P2[r][p][0];
            }
        }
        U1[a][p][0] = u1r;
        U2[a][p][0] = u2r;
        if constexpr (CPLX) {
            U1[a][p][NC - 1] = u1i;
            U2[a][p][NC - 1] = u2i;
        }
    }
    __syncthreads();
    {   // Cm[a][p] = sum_{a2 <= a} conj(T[a2][a]) U1[a2][p]   (a < p)
        //          = sum_{a2 >= a} T[a][a2] U2[a2][p]          (a > p)
        const int a = tid / 16, p = tid % 16;
        double cr = 0.0, ci = 0.0;
        if (a < p)
            for (int a2 = 0; a2 <= a; ++a2) {
                const double tr = Ts[a2][a][0];
                if constexpr (CPLX) {
                    const double ti = -Ts[a2][a][NC - 1];
                    cr += tr * U1[a2][p][0] - ti * U1[a2][p][NC - 1];
                    ci += tr * U1[a2][p][NC - 1] + ti * U1[a2][p][0];
                } else {
                    cr += tr * U1[a2][p][0];
                }
            }
        if (a > p)
            for (int a2 = a; a2 < 16; ++a2) {
                const double tr = Ts[a][a2][0];
                if constexpr (CPLX) {
                    const double ti = Ts[a][a2][NC - 1];
                    cr += tr * U2[a2][p][0] - ti * U2[a2][p][NC - 1];
                    ci += tr * U2[a2][p][NC - 1] + ti * U2[a2][p][0];
                } else {
                    cr += tr * U2[a2][p][0];
                }
            }
        Cm[a][p][0] = cr;
        if constexpr (CPLX) Cm[a][p][NC - 1] = ci;
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
        double vr = 0.0, vi = 0.0;
        if (i < len) {
            const int r = p + 1 + i;
            // t1 = P1 - V_<p Cm_<p, t2 = P2 - V_>p Cm_>p on row r
            double t1r = P1[r][p][0], t1i = CPLX ? P1[r][p][NC - 1] : 0.0;
            double t2r = P2[r][p][0], t2i = CPLX ? P2[r][p][NC - 1] : 0.0;
            for (int a = 0; a < 16; ++a) {
                if (a == p) continue;
                const double xr = Vs[r][a][0], cr = Cm[a][p][0];
                double pr, pi = 0.0;
                if constexpr (CPLX) {
                    const double xi = Vs[r][a][NC - 1], ci = Cm[a][p][NC - 1];
                    pr = xr * cr - xi * ci;
                    pi = xr * ci + xi * cr;
                } else {
                    pr = xr * cr;
                }
                if (a < p) {
                    t1r -= pr;
                    t1i -= pi;
                } else {
                    t2r -= pr;
                    t2i -= pi;
                }
            }
            const double ur = taus[p][0], ui = CPLX ? taus[p][NC - 1] : 0.0;
            // -(conj(tau) t1 + tau t2)
            vr = -((ur * t1r + ui * t1i) + (ur * t2r - ui * t2i));
            vi = -((ur * t1i - ui * t1r) + (ur * t2i + ui * t2r));
        }
        dv[(k * NB + i) * NC] = vr;
        if constexpr (CPLX) dv[(k * NB + i) * NC + 1] = vi;
        if (i == 0) {
#pragma unroll
            for (int pl = 0; pl < NC; ++pl) dtau[k * NC + pl] = dts[p][pl];
        }
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
constexpr int ADJ_WAVES = 8;     // waves (slots in flight) per strip, real
// the same, complex: two waves per SIMD, with the complex checkpointing
// forward's registers spilling a little (140 bytes per lane at nbw = 64),
// beats one wave per SIMD without spills (n = 4096, nev = 2048: 48.7 ->
// 43.3 ms for forward + adjoint)
constexpr int ADJ_WAVES_Z = 8;

constexpr int ADJ_GMAX = 4;   // slot groups per strip in the split form, at most

// CUs of the current device (looked up once per device id).
inline int adj_device_cus()
{
    static int cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (dev >= 0 && dev < 64) cached[dev] = cus;
    return cus;
}

// Slot groups for a strip kernel of `strips` workgroups with nw waves over
// J slots: G = min(CUs / strips, rounds of slots, ADJ_GMAX) when the strips
// alone leave CUs idle, else 1.
inline int adj_slot_groups(int64_t strips, int64_t J, int nw)
{
    const int cus = adj_device_cus();
    if (cus <= 0 || strips >= cus) return 1;
    int64_t G = cus / strips;
    const int64_t rounds = (J + nw - 1) / nw;
    if (G > rounds) G = rounds;
    if (G > ADJ_GMAX) G = ADJ_GMAX;
    return G < 1 ? 1 : (int)G;
}

struct AdjLayout {
    size_t zs = 0, fwd = 0, apk = 0, ckpt = 0, gck = 0, gprog = 0, part = 0, tape = 0, total = 0;
    int64_t nblocks = 0, nstrips = 0, nwaves = 0;
};

size_t al(size_t x) { return (x + 255) / 256 * 256; }

int adj_tiles(int nbw) { return nbw / 16 + 1; }

int adj_apb(int nbw, bool cplx)
{
    switch (nbw) {
        case 16: return cplx ? AdjGeo<16, true>::APB : AdjGeo<16>::APB;
        case 32: return cplx ? AdjGeo<32, true>::APB : AdjGeo<32>::APB;
        case 48: return cplx ? AdjGeo<48, true>::APB : AdjGeo<48>::APB;
        default: return cplx ? AdjGeo<64, true>::APB : AdjGeo<64>::APB;
    }
}

// Workspace of the adjoint: the blocked layout when use_blocked(n, nbw,
// cplx) (complex: only that one; the complex streaming form has its own),
// else the real streaming layout.
AdjLayout adj_layout(int64_t n, int nbw, int64_t nev, bool cplx = false)
{
    AdjLayout L;
    const size_t elt = cplx ? 2 * sizeof(double) : sizeof(double);
    size_t off = HDR_BYTES;
    L.zs = off;
    off = al(off + (size_t)n * nev * elt);
    if (use_blocked(n, nbw, cplx)) {
        const int nt = adj_tiles(nbw);
        L.nblocks = blocked_num_blocks(n, nbw);
        L.nstrips = (nev + 15) / 16;
        const size_t pb = (size_t)packed_block_doubles(nbw, cplx);
        L.fwd = off;
        off = al(off + (size_t)L.nblocks * pb * sizeof(double));
        L.apk = off;
        off = al(off + (size_t)L.nblocks * adj_apb(nbw, cplx) * sizeof(double));
        L.ckpt = off;
        off = al(off + (size_t)L.nblocks * nt * L.nstrips * 256 * elt);
        L.gck = off;   // every block's output-gradient window, checkpoint layout
        off = al(off + (size_t)L.nblocks * nt * L.nstrips * 256 * elt);
        L.gprog = off;   // slot-group progress counters (split form)
        off = al(off + (size_t)(L.nstrips + 8) * ADJ_GMAX * sizeof(int));
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

// Launch a strip kernel of the split form with slot groups when its strips
// leave CUs idle and the grid fits at once (cooperative launch, zeroed
// counters), else one workgroup per strip.  kern1 / kernG: the kernel
// without / with slot groups; args: the kernel's arguments before (G, gprog).
template <typename K1, typename KG, typename... Args>
int launch_strips(K1 kern1, KG kernG, int64_t ns, int64_t J, int nw, int* gprog, hipStream_t st,
                  Args... args)
{
    const int G = adj_slot_groups(ns, J, nw);
    if (G > 1) {
        const int64_t grid = (ns + 7) / 8 * 8 * G;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernG, 64 * nw, 0) ==
                hipSuccess &&
            (int64_t)per_cu * adj_device_cus() >= grid) {
            const int cnt = (int)(ns * G);
            hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
                               (unsigned*)gprog, cnt);
            int g32 = G;
            void* argv[] = {(void*)&args..., (void*)&g32, (void*)&gprog};
            if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kernG),
                                           dim3((unsigned)grid), dim3(64 * nw), argv, 0,
                                           st) == hipSuccess)
                return TRBT_SUCCESS;
        }
        (void)hipGetLastError();
    }
    hipLaunchKernelGGL(kern1, dim3((unsigned)ns), dim3(64 * nw), 0, st, args..., 1, (int*)nullptr);
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

// The adjoint in two halves.  adj_forward: the forward transformation of Z
// (in place) that also writes the checkpoints into the workspace;
// adj_backward: the reverse sweep from those checkpoints.  Real or complex
// (interleaved re, im; ldz, ldg in elements).
template <int NB, bool CPLX = false>
void blocked_forward(int64_t n, int64_t nev, const double* hv, const double* ht, double* Z,
                     int64_t ldz, char* ws, const AdjLayout& L, hipStream_t st)
{
    constexpr int NW = CPLX ? ADJ_WAVES_Z : ADJ_WAVES;
    double* fwd = (double*)(ws + L.fwd);
    const unsigned nb = (unsigned)L.nblocks;
    hipLaunchKernelGGL((k_pack<NB, CPLX, rotating_window<NB, CPLX>()>), dim3(nb), dim3(256), 0,
                       st, n, hv, ht, fwd);
    launch_strips(k_blocked_ckpt<NB, NW, CPLX, false>, k_blocked_ckpt<NB, NW, CPLX, true>,
                  L.nstrips, sweeps_in_stage(n, NB, 0), NW, (int*)(ws + L.gprog), st, n, nev,
                  (const double*)fwd, Z, ldz, (double*)(ws + L.ckpt), (unsigned*)ws);
}

template <int NB, bool CPLX = false>
void blocked_backward(int64_t n, int64_t nev, const double* hv, const double* ht, double* G,
                      int64_t ldg, double* dv, double* dtau, char* ws, const AdjLayout& L,
                      hipStream_t st)
{
    constexpr int NW = CPLX ? ADJ_WAVES_Z : ADJ_WAVES;
    double* apk = (double*)(ws + L.apk);
    double* gck = (double*)(ws + L.gck);
    const unsigned nb = (unsigned)L.nblocks, ns = (unsigned)L.nstrips;
    hipLaunchKernelGGL((k_pack_adj<NB, CPLX>), dim3(nb), dim3(256), 0, st, n, hv, ht, apk);
    launch_strips(k_adj_sweep<NB, NW, CPLX, false>, k_adj_sweep<NB, NW, CPLX, true>, L.nstrips,
                  sweeps_in_stage(n, NB, 0), NW, (int*)(ws + L.gprog), st, n, nev,
                  (const double*)apk, G, ldg, gck, (unsigned*)ws);
    hipLaunchKernelGGL((k_adj_reduce<NB, 4, CPLX>), dim3(nb), dim3(256), 0, st, n, (int64_t)ns,
                       (const double*)apk, (const double*)(ws + L.ckpt), (const double*)gck, dv,
                       dtau);
}

// Both halves in one go (the one-call adjoint): the checkpointing forward and
// the backward sweep share one launch, then the reduction.  Real or complex
// (interleaved re, im) data.
template <int NB, bool CPLX>
void blocked_both(int64_t n, int64_t nev, const double* hv, const double* ht, double* Z,
                  int64_t ldz, double* G, int64_t ldg, double* dv, double* dtau, char* ws,
                  const AdjLayout& L, hipStream_t st)
{
    constexpr int NW = CPLX ? ADJ_WAVES_Z : ADJ_WAVES;
    double* fwd = (double*)(ws + L.fwd);
    double* apk = (double*)(ws + L.apk);
    double* gck = (double*)(ws + L.gck);
    const unsigned nb = (unsigned)L.nblocks, ns = (unsigned)L.nstrips;
    hipLaunchKernelGGL((k_pack<NB, CPLX, rotating_window<NB, CPLX>()>), dim3(nb), dim3(256), 0,
                       st, n, hv, ht, fwd);
    hipLaunchKernelGGL((k_pack_adj<NB, CPLX>), dim3(nb), dim3(256), 0, st, n, hv, ht, apk);
    hipLaunchKernelGGL((k_adj_fwd_sweep<NB, NW, CPLX>), dim3(2 * ns), dim3(64 * NW), 0, st, n,
                       nev, (const double*)fwd, Z, ldz, (double*)(ws + L.ckpt),
                       (const double*)apk, G, ldg, gck, (unsigned*)ws);
    hipLaunchKernelGGL((k_adj_reduce<NB, 4, CPLX>), dim3(nb), dim3(256), 0, st, n, (int64_t)ns,
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

// Blocked complex adjoint, called by trans_ev_tridi_to_band_adjoint_z (in
// trbt_adjoint_z.hip) after its argument checks when use_blocked(n, nbw,
// true); K > 0 and nev > 0.  Not exported.
__attribute__((visibility("hidden"))) size_t trbt_adjoint_blocked_bytes_z(int64_t n, int nbw,
                                                                          int64_t nev)
{
    return adj_layout(n, nbw, nev, true).total;
}

__attribute__((visibility("hidden"))) int trbt_adjoint_blocked_z(
    int64_t n, int nbw, int64_t nev, const double* hv, const double* ht, const double* Z_in,
    int64_t ldz, double* G, int64_t ldg, double* dv, double* dtau, void* work,
    size_t work_bytes, hipStream_t st)
{
    const AdjLayout L = adj_layout(n, nbw, nev, true);
    if (!work || work_bytes < L.total) return TRBT_ERR_WORKSPACE;
    char* ws = (char*)work;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (unsigned*)work, 64);
    double* Zs = (double*)(ws + L.zs);
    if (hipMemcpy2DAsync(Zs, (size_t)n * 16, Z_in, (size_t)ldz * 16, (size_t)n * 16,
                         (size_t)nev, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return TRBT_ERR_HIP;
    switch (nbw) {
        case 16: blocked_both<16, true>(n, nev, hv, ht, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
        case 32: blocked_both<32, true>(n, nev, hv, ht, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
        case 48: blocked_both<48, true>(n, nev, hv, ht, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
        case 64: blocked_both<64, true>(n, nev, hv, ht, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
        default: return TRBT_ERR_INTERNAL;
    }
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

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
            case 16: blocked_both<16, false>(n, nev, hh_v, hh_tau, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
            case 32: blocked_both<32, false>(n, nev, hh_v, hh_tau, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
            case 48: blocked_both<48, false>(n, nev, hh_v, hh_tau, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
            case 64: blocked_both<64, false>(n, nev, hh_v, hh_tau, Zs, n, G, ldg, dv, dtau, ws, L, st); break;
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

int trans_ev_tridi_to_band_fwd_ckpt_z(int64_t n, int nbw, int64_t nev, const trbt_z* hh_v,
                                      const trbt_z* hh_tau, trbt_z* Z, int64_t ldz,
                                      int ckpt_every, void* work, size_t work_bytes, void* stream)
{
    if (n < 0) return -1;
    if (!blocked_eligible(nbw)) return -2;
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
    if (active && !use_blocked(n, nbw, true)) return -1;   // beyond the blocked kernels' range
    if (!active) return TRBT_SUCCESS;
    int rc = check_device();
    if (rc) return rc;
    const AdjLayout L = adj_layout(n, nbw, nev, true);
    if (!work || work_bytes < L.total) return TRBT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (unsigned*)work, 64);
    const double *hv = (const double*)hh_v, *ht = (const double*)hh_tau;
    double* Zd = (double*)Z;
    char* ws = (char*)work;
    switch (nbw) {
        case 16: blocked_forward<16, true>(n, nev, hv, ht, Zd, ldz, ws, L, st); break;
        case 32: blocked_forward<32, true>(n, nev, hv, ht, Zd, ldz, ws, L, st); break;
        case 48: blocked_forward<48, true>(n, nev, hv, ht, Zd, ldz, ws, L, st); break;
        case 64: blocked_forward<64, true>(n, nev, hv, ht, Zd, ldz, ws, L, st); break;
        default: return TRBT_ERR_INTERNAL;
    }
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

int trans_ev_tridi_to_band_bwd_ckpt_z(int64_t n, int nbw, int64_t nev, const trbt_z* hh_v,
                                      const trbt_z* hh_tau, trbt_z* G, int64_t ldg, trbt_z* dv,
                                      trbt_z* dtau, int ckpt_every, void* work,
                                      size_t work_bytes, void* stream)
{
    if (n < 0) return -1;
    if (!blocked_eligible(nbw)) return -2;
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
    if (K > 0 && nev > 0 && !use_blocked(n, nbw, true)) return -1;
    if (K == 0) return TRBT_SUCCESS;
    int rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    // complex dv (K x nbw) and dtau (K): twice the doubles of the real ones
    if (nev == 0) return zero_grads(2 * K, nbw, (double*)dv, (double*)dtau, st);
    const AdjLayout L = adj_layout(n, nbw, nev, true);
    if (!work || work_bytes < L.total) return TRBT_ERR_WORKSPACE;
    const double *hv = (const double*)hh_v, *ht = (const double*)hh_tau;
    double *Gd = (double*)G, *dvd = (double*)dv, *dtd = (double*)dtau;
    char* ws = (char*)work;
    switch (nbw) {
        case 16: blocked_backward<16, true>(n, nev, hv, ht, Gd, ldg, dvd, dtd, ws, L, st); break;
        case 32: blocked_backward<32, true>(n, nev, hv, ht, Gd, ldg, dvd, dtd, ws, L, st); break;
        case 48: blocked_backward<48, true>(n, nev, hv, ht, Gd, ldg, dvd, dtd, ws, L, st); break;
        case 64: blocked_backward<64, true>(n, nev, hv, ht, Gd, ldg, dvd, dtd, ws, L, st); break;
        default: return TRBT_ERR_INTERNAL;
    }
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

}  // extern "C"
