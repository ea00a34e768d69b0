// trbt_b2f.hip -- band-to-full eigenvector back-transformation on gfx950:
// C = P^* Y (Sec. 2.1, Eq. 2stage_bkwd2), the step after the
// tridiagonal-to-banded one, with P^* = H_0 H_1 ... H_{J-1} the Householder
// reflectors of the full-to-band reduction B = P A P^* (Eq. 2stage_fwd1):
// one reflector per column j = 0 .. n-nbw-2, acting on rows [j+nbw, n).
//
// Unlike the stage-2 reflectors (length <= nbw, a few per column of Z),
// these are long, so the update is GEMM-rich: PW consecutive reflectors
// form a panel, H_{j0} ... H_{j0+PW-1} = I - V T V^H (forward compact WY,
// T upper triangular), and the panels are applied last to first:
//     W = V^H Z,  W' = T W,  Z <- Z - V W'     (rows [j0+nbw, n) of Z).
//
// Kernels:
//  * k_b2f_tfac (one workgroup per panel): the Gram matrix V^H V on FP64
//    MFMA, then T column by column, T[0:q, q] = -tau_q T[0:q, 0:q] G[0:q, q],
//    stored column-major (PW x PW) in the workspace.
//  * k_b2f_apply (one workgroup per strip of 16 CT columns of Z, NW waves):
//    for every panel p from the last to the first, the waves walk the
//    panel's rows in 16-row blocks (block b to wave b mod NW).  A block is
//    loaded once into MFMA accumulators, updated with panel p
//    (Z -= V_p W'_p, W'_p in LDS), stored, and -- while still in registers --
//    contracted with the next panel's reflectors, W_{p-1} += V_{p-1}^H Z.
//    So each panel reads and writes its rows of Z once.  The waves' partial
//    W_{p-1} are summed in wave order through LDS (bitwise reproducible),
//    multiplied by T_{p-1} on MFMA into W'_{p-1}, and the next panel starts.
//
// Register layout of v_mfma_f64_16x16x4_f64 (A lane i+16k = A[i][k], B lane
// j+16k = B[k][j], D lane j+16g element e = D[g+4e][j]): a 16-row block of Z
// in accumulator layout holds rows g+4e of column j, so element e is exactly
// the B operand of the contraction over its rows 4e..4e+3; likewise element
// e of a W tile is the B operand for reflectors 4e..4e+3 of that tile.

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>

#include "trbt.h"
#include "trbt_device.h"

namespace {

constexpr int B2F_PW = 64;         // reflectors per panel
constexpr int B2F_PT = B2F_PW / 16;
constexpr int B2F_NW = 8;          // waves per workgroup of the apply kernel
constexpr int B2F_HDR = 256;       // workspace header (fault word, unused here)

__host__ __device__ inline int64_t b2f_reflectors(int64_t n, int nbw)
{
    return (nbw >= 1 && n - nbw - 1 > 0) ? n - nbw - 1 : 0;
}

__host__ __device__ inline int64_t b2f_panels(int64_t J) { return (J + B2F_PW - 1) / B2F_PW; }

// one stored element: real or complex (interleaved re, im)
template <bool CPLX>
struct Elt;
template <>
struct Elt<false> {
    double re;
    static constexpr double im = 0.0;
};
template <>
struct Elt<true> {
    double re, im;
};

template <bool CPLX>
__device__ inline Elt<CPLX> ld_elt(const double* __restrict__ p, int64_t idx)
{
    Elt<CPLX> e;
    if constexpr (CPLX) {
        const d2 v = *reinterpret_cast<const d2*>(p + 2 * idx);
        e.re = v.x;
        e.im = v.y;
    } else {
        e.re = p[idx];
    }
    return e;
}

template <bool CPLX>
__device__ inline void st_elt(double* __restrict__ p, int64_t idx, double re, double im)
{
    if constexpr (CPLX) {
        d2 v;
        v.x = re;
        v.y = im;
        *reinterpret_cast<d2*>(p + 2 * idx) = v;
    } else {
        (void)im;
        p[idx] = re;
    }
}

// element (row r, reflector j) of the stored reflectors, or 0 where the
// reflector has no entry (rows above its start j+nbw, rows >= n, j >= J)
template <bool CPLX>
__device__ inline Elt<CPLX> v_at(const double* __restrict__ V, int64_t ldv, int64_t n,
                                 int nbw, int64_t J, int64_t r, int64_t j)
{
    Elt<CPLX> e{};
    if (j < J && r >= j + nbw && r < n) e = ld_elt<CPLX>(V, r + j * ldv);
    return e;
}

// The same without a branch: the load reads a clamped address inside the
// n x J array (row min(r, n-1), column min(j, J-1)) and the value is
// replaced by 0 where the reflector has no entry, so a block's loads can all
// be issued before the first is needed.
template <bool CPLX>
__device__ inline Elt<CPLX> v_sel(const double* __restrict__ V, int64_t ldv, int64_t n,
                                  int nbw, int64_t J, int64_t r, int64_t j)
{
    const bool ok = j < J && r >= j + nbw && r < n;
    const int64_t rr = r < n ? r : n - 1, jj = j < J ? j : J - 1;
    Elt<CPLX> e = ld_elt<CPLX>(V, rr + jj * ldv);
    e.re = ok ? e.re : 0.0;
    if constexpr (CPLX) e.im = ok ? e.im : 0.0;
    return e;
}

// --------------------------------------------------------------------------
// k_b2f_tfac: T of panel p (reflectors j0 .. j0+PW-1), 256 threads.
// G = V^H V over the panel's rows (upper 16x16 tiles only, on MFMA, written
// to the panel's T area in global memory), then T column by column in LDS
// (thread i owns row i), then T over G.
// --------------------------------------------------------------------------
template <bool CPLX>
__global__ __launch_bounds__(256) void k_b2f_tfac(int64_t n, int nbw, const double* __restrict__ V,
                                                  int64_t ldv, const double* __restrict__ tau,
                                                  double* __restrict__ Tw)
{
    constexpr int PW = B2F_PW, PT = B2F_PT, NC = CPLX ? 2 : 1;
    const int64_t J = b2f_reflectors(n, nbw);
    const int64_t p = blockIdx.x;
    const int64_t j0 = p * PW;
    const int64_t rlo = j0 + nbw;          // first row any reflector of the panel touches
    double* __restrict__ Tp = Tw + p * (int64_t)PW * PW * NC;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i16 = lane & 15, k4 = lane >> 4;

    // upper tiles (a <= b), numbered row by row, tile w + 4t to wave w
    constexpr int NTILE = PT * (PT + 1) / 2;
    constexpr int MY = (NTILE + 3) / 4;
    int ta[MY], tb[MY];
#pragma unroll
    for (int t = 0; t < MY; ++t) {
        int tg = w + 4 * t, a = 0;
        while (a < PT && tg >= PT - a) {
            tg -= PT - a;
            ++a;
        }
        ta[t] = a;           // a == PT: no tile
        tb[t] = a + tg;
    }
    const int cnt = (NTILE - w + 3) / 4;
    d4 gr[MY], gi[MY];
#pragma unroll
    for (int t = 0; t < MY; ++t) {
        gr[t] = d4{0.0, 0.0, 0.0, 0.0};
        gi[t] = gr[t];
    }
    for (int64_t r0 = rlo; r0 < n; r0 += 4) {
        const int64_t r = r0 + k4;
#pragma unroll
        for (int t = 0; t < MY; ++t) {
            if (t >= cnt) break;
            // A[i][k] = conj(V[r0+k][j0+16a+i]), B[k][j] = V[r0+k][j0+16b+j]
            const Elt<CPLX> x = v_at<CPLX>(V, ldv, n, nbw, J, r, j0 + 16 * ta[t] + i16);
            const Elt<CPLX> y = v_at<CPLX>(V, ldv, n, nbw, J, r, j0 + 16 * tb[t] + i16);
            gr[t] = mfma(x.re, y.re, gr[t]);
            if constexpr (CPLX) {
                gr[t] = mfma(x.im, y.im, gr[t]);          // Re conj(x) y
                gi[t] = mfma(x.re, y.im, gi[t]);          // Im conj(x) y
                gi[t] = mfma_n<1>(x.im, y.re, gi[t]);
            }
        }
    }
    // G tile (a, b) element e of lane l: G[16a + l/16 + 4e][16b + l%16]
#pragma unroll
    for (int t = 0; t < MY; ++t) {
        if (t >= cnt) break;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gi_ = 16 * ta[t] + k4 + 4 * e, gj = 16 * tb[t] + i16;
            st_elt<CPLX>(Tp, gi_ + (int64_t)gj * PW, gr[t][e], CPLX ? gi[t][e] : 0.0);
        }
    }
    __syncthreads();

    // T = forward compact-WY factor: T[q][q] = tau_q, and for i < q
    // T[i][q] = -tau_q sum_{k=i}^{q-1} T[i][k] G[k][q]  (row i by thread i)
    __shared__ double Ts[PW][PW + 1][NC];
    const int i = threadIdx.x;
    for (int q = 0; q < PW; ++q) {
        if (i < PW) {
            const int64_t jq = j0 + q;
            Elt<CPLX> tq{};
            if (jq < J) tq = ld_elt<CPLX>(tau, jq);
            double sr = 0.0, si = 0.0;
            if (i < q) {
                for (int k = i; k < q; ++k) {
                    const Elt<CPLX> g = ld_elt<CPLX>(Tp, k + (int64_t)q * PW);
                    const double ar = Ts[i][k][0], ai = CPLX ? Ts[i][k][NC - 1] : 0.0;
                    sr += ar * g.re - ai * g.im;
                    si += ar * g.im + ai * g.re;
                }
            }
            double outr, outi;
            if (i == q) {
                outr = tq.re;
                outi = tq.im;
            } else if (i < q) {   // -tau_q * s
                outr = -(tq.re * sr - tq.im * si);
                outi = -(tq.re * si + tq.im * sr);
            } else {
                outr = 0.0;
                outi = 0.0;
            }
            Ts[i][q][0] = outr;
            if (CPLX) Ts[i][q][NC - 1] = outi;
        }
        __syncthreads();
    }
    // T over G, column-major
    for (int idx = threadIdx.x; idx < PW * PW; idx += 256) {
        const int r = idx % PW, c = idx / PW;
        st_elt<CPLX>(Tp, r + (int64_t)c * PW, Ts[r][c][0], CPLX ? Ts[r][c][NC - 1] : 0.0);
    }
}

// --------------------------------------------------------------------------
// k_b2f_apply
// --------------------------------------------------------------------------
template <bool CPLX, int CT>
struct B2FLds {
    // W (summed partials) and W' = T W, in accumulator layout:
    // [reflector tile][column tile][element e][plane][lane]
    double W[B2F_PT][CT][4][CPLX ? 2 : 1][64];
    double Wp[B2F_PT][CT][4][CPLX ? 2 : 1][64];
};

template <bool CPLX, int CT, int NW>
__global__ __launch_bounds__(64 * NW) void k_b2f_apply(
    int64_t n, int nbw, int64_t nev, const double* __restrict__ V, int64_t ldv,
    const double* __restrict__ Tw, double* __restrict__ Z, int64_t ldz)
{
    constexpr int PW = B2F_PW, PT = B2F_PT, NP = CPLX ? 2 : 1;
    __shared__ B2FLds<CPLX, CT> S;
    const int64_t J = b2f_reflectors(n, nbw);
    const int64_t P = b2f_panels(J);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i16 = lane & 15, g4 = lane >> 4;
    const int64_t col0 = (int64_t)blockIdx.x * 16 * CT;

    Tile<CPLX> w[PT][CT];   // this wave's partial W of the next panel

    for (int64_t p = P; p >= 0; --p) {
        if (p < P) {
            // ---- sum the waves' partials of W_p in wave order, then W'_p = T_p W_p
            __syncthreads();   // every wave is done with the previous W'
            for (int q = 0; q < NW; ++q) {
                if (wv == q) {
#pragma unroll
                    for (int a = 0; a < PT; ++a)
#pragma unroll
                        for (int c = 0; c < CT; ++c)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                double* sr = &S.W[a][c][e][0][lane];
                                *sr = (q == 0) ? w[a][c].re[e] : *sr + w[a][c].re[e];
                                if constexpr (CPLX) {
                                    double* si = &S.W[a][c][e][NP - 1][lane];
                                    *si = (q == 0) ? w[a][c].im[e] : *si + w[a][c].im[e];
                                }
                            }
                }
                __syncthreads();
            }
            const double* __restrict__ Tp = Tw + p * (int64_t)PW * PW * NP;
            for (int t = wv; t < PT * CT; t += NW) {
                const int a = t / CT, c = t % CT;
                d4 accr = d4{0.0, 0.0, 0.0, 0.0}, acci = accr;
                for (int k0 = 16 * a; k0 < PW; k0 += 4) {
                    // A[i][k] = T[16a+i][k0+k], B[k][j] = W[k0+k][16c+j]
                    const Elt<CPLX> tv = ld_elt<CPLX>(Tp, (16 * a + i16) + (int64_t)(k0 + g4) * PW);
                    const int bt = k0 / 16, be = (k0 % 16) / 4;
                    const double br = S.W[bt][c][be][0][lane];
                    accr = mfma(tv.re, br, accr);
                    if constexpr (CPLX) {
                        const double bi = S.W[bt][c][be][NP - 1][lane];
                        accr = mfma_n<1>(tv.im, bi, accr);
                        acci = mfma(tv.re, bi, acci);
                        acci = mfma(tv.im, br, acci);
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    S.Wp[a][c][e][0][lane] = accr[e];
                    if constexpr (CPLX) S.Wp[a][c][e][NP - 1][lane] = acci[e];
                }
            }
            __syncthreads();
        }
        // ---- one pass over the rows: update with panel p (if p < P), then
        // accumulate the next panel's W (if p > 0)
#pragma unroll
        for (int a = 0; a < PT; ++a)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                w[a][c].re = d4{0.0, 0.0, 0.0, 0.0};
                if constexpr (CPLX) w[a][c].im = w[a][c].re;
            }
        const int64_t jp = p * PW;            // first reflector of panel p
        const int64_t jn = (p - 1) * PW;      // first reflector of panel p-1
        const int64_t lo = (p > 0) ? jn + nbw : jp + nbw;
        const bool upd = p < P, acc = p > 0;
        for (int64_t r0 = lo + 16 * (int64_t)wv; r0 < n; r0 += 16 * NW) {
            // W'_p is read from LDS block by block, not held in registers
            // across the loop (room for the block's operands)
            asm volatile("" ::: "memory");
            // every load of the block first (clamped addresses, masked
            // values), then the products
            Tile<CPLX> z[CT];
            // the 16-row block: lane (j, g) element e = Z[r0+g+4e][col0+16c+j]
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int64_t col = col0 + 16 * c + i16;
                const int64_t cc = col < nev ? col : nev - 1;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t r = r0 + g4 + 4 * e;
                    const bool ok = r < n && col < nev;
                    const Elt<CPLX> x = ld_elt<CPLX>(Z, (r < n ? r : n - 1) + cc * ldz);
                    z[c].re[e] = ok ? x.re : 0.0;
                    if constexpr (CPLX) z[c].im[e] = ok ? x.im : 0.0;
                }
            }
            const bool in_p = upd && r0 >= jp + nbw;
            // Real blocks load all of their reflector operands before the
            // first product (one MFMA per operand: latency would dominate);
            // complex blocks (four MFMAs per operand, and no registers to
            // spare) load each operand just before its products.
            constexpr bool HOIST = !CPLX;
            constexpr int NU = HOIST ? PW / 4 : 1, NA = HOIST ? 4 : 1, NPT = HOIST ? PT : 1;
            // update operands: A[i][k] = V[r0+i][jp+4kk+k]
            Elt<CPLX> vu[NU];
            // accumulation operands: A[i][k] = conj(V[r0+4u+k][jn+16a+i])
            Elt<CPLX> va[NA][NPT];
            if constexpr (HOIST) {
                if (in_p) {
#pragma unroll
                    for (int kk = 0; kk < PW / 4; ++kk)
                        vu[kk] = v_sel<CPLX>(V, ldv, n, nbw, J, r0 + i16, jp + 4 * kk + g4);
                }
                if (acc) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int a = 0; a < PT; ++a)
                            va[u][a] = v_sel<CPLX>(V, ldv, n, nbw, J, r0 + 4 * u + g4,
                                                   jn + 16 * a + i16);
                }
            }
            auto v_upd = [&](int kk) -> Elt<CPLX> {
                if constexpr (HOIST) return vu[kk];
                else return v_sel<CPLX>(V, ldv, n, nbw, J, r0 + i16, jp + 4 * kk + g4);
            };
            auto v_acc = [&](int u, int a) -> Elt<CPLX> {
                if constexpr (HOIST) return va[u][a];
                else return v_sel<CPLX>(V, ldv, n, nbw, J, r0 + 4 * u + g4, jn + 16 * a + i16);
            };
            if (in_p) {
                // Z -= V_p W'_p: A[i][k] = V[r0+i][jp+k0+k], B = W'_p rows k0..k0+3
#pragma unroll
                for (int k0 = 0; k0 < PW; k0 += 4) {
                    const Elt<CPLX> v = v_upd(k0 / 4);
                    const int bt = k0 / 16, be = (k0 % 16) / 4;
#pragma unroll
                    for (int c = 0; c < CT; ++c) {
                        const double br = S.Wp[bt][c][be][0][lane];
                        z[c].re = mfma_n<1>(v.re, br, z[c].re);
                        if constexpr (CPLX) {
                            const double bi = S.Wp[bt][c][be][NP - 1][lane];
                            z[c].re = mfma(v.im, bi, z[c].re);
                            z[c].im = mfma_n<1>(v.re, bi, z[c].im);
                            z[c].im = mfma_n<1>(v.im, br, z[c].im);
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const int64_t col = col0 + 16 * c + i16;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t r = r0 + g4 + 4 * e;
                        if (r < n && col < nev) {
                            if constexpr (CPLX)
                                st_elt<CPLX>(Z, r + col * ldz, z[c].re[e], z[c].im[e]);
                            else
                                st_elt<CPLX>(Z, r + col * ldz, z[c].re[e], 0.0);
                        }
                    }
                }
            }
            if (acc) {
                // W_{p-1} += V_{p-1}^H Z: A[i][k] = conj(V[r0+4u+k][jn+16a+i]),
                // B = element u of the block (rows 4u..4u+3)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
#pragma unroll
                    for (int a = 0; a < PT; ++a) {
                        const Elt<CPLX> v = v_acc(u, a);
#pragma unroll
                        for (int c = 0; c < CT; ++c) {
                            w[a][c].re = mfma(v.re, z[c].re[u], w[a][c].re);
                            if constexpr (CPLX) {
                                w[a][c].re = mfma(v.im, z[c].im[u], w[a][c].re);
                                w[a][c].im = mfma(v.re, z[c].im[u], w[a][c].im);
                                w[a][c].im = mfma_n<1>(v.im, z[c].re[u], w[a][c].im);
                            }
                        }
                    }
                }
            }
        }
    }
}

template <bool CPLX>
int b2f_validate(int64_t n, int nbw, int64_t nev, const void* V, int64_t ldv, const void* tau,
                 const void* Z, int64_t ldz, const void* work, size_t work_bytes)
{
    if (n < 0) return -1;
    if (nbw < 1) return -2;
    if (nev < 0 || nev > n) return -3;
    const int64_t J = b2f_reflectors(n, nbw);
    const bool active = J > 0 && nev > 0;
    if (active && !V) return -4;
    if (ldv < (n > 1 ? n : 1)) return -5;
    if (active && !tau) return -6;
    if (nev > 0 && n > 0 && !Z) return -7;
    if (ldz < (n > 1 ? n : 1)) return -8;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -9;
    if (work_bytes && !work) return -9;
    return TRBT_SUCCESS;
}

size_t b2f_bytes(int64_t n, int nbw, bool cplx)
{
    const int64_t J = b2f_reflectors(n, nbw);
    if (J == 0) return 0;
    return B2F_HDR + (size_t)b2f_panels(J) * B2F_PW * B2F_PW * (cplx ? 16 : 8);
}

template <bool CPLX>
int b2f_run(int64_t n, int nbw, int64_t nev, const double* V, int64_t ldv, const double* tau,
            double* Z, int64_t ldz, void* work, size_t work_bytes, void* stream_v)
{
    int rc = b2f_validate<CPLX>(n, nbw, nev, V, ldv, tau, Z, ldz, work, work_bytes);
    if (rc) return rc;
    const int64_t J = b2f_reflectors(n, nbw);
    if (J == 0 || nev == 0) return TRBT_SUCCESS;
    if (!work || work_bytes < b2f_bytes(n, nbw, CPLX)) return TRBT_ERR_WORKSPACE;
    rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream_v;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (unsigned*)work, 64);
    double* Tw = (double*)((char*)work + B2F_HDR);
    const int64_t P = b2f_panels(J);
    hipLaunchKernelGGL((k_b2f_tfac<CPLX>), dim3((unsigned)P), dim3(256), 0, st, n, nbw, V, ldv,
                       tau, Tw);
    // complex: two 16-column tiles per workgroup when that still gives every
    // CU a strip; real: one (its block operands take the registers)
    const int64_t s2 = (nev + 31) / 32;
    if constexpr (CPLX) {
        if (s2 >= 256) {
            hipLaunchKernelGGL((k_b2f_apply<CPLX, 2, B2F_NW>), dim3((unsigned)s2),
                               dim3(64 * B2F_NW), 0, st, n, nbw, nev, V, ldv, (const double*)Tw,
                               Z, ldz);
            return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
        }
    }
    {
        const int64_t s1 = (nev + 15) / 16;
        hipLaunchKernelGGL((k_b2f_apply<CPLX, 1, B2F_NW>), dim3((unsigned)s1), dim3(64 * B2F_NW),
                           0, st, n, nbw, nev, V, ldv, (const double*)Tw, Z, ldz);
    }
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

// --------------------------------------------------------------------------
// Allocation-free variant (trans_ev_band_to_full_z_noalloc): the per-panel
// T factors go to a fixed array of device memory instead of a caller
// workspace.  Every device the library runs on holds its own copy of the
// array until the process ends; all calls on one device share it.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): it looks up the device address once per device
// and passes that.
// --------------------------------------------------------------------------
constexpr int B2F_MAX_DEVICES = 64;
std::mutex b2f_scratch_mu;
void* b2f_scratch_ptr[B2F_MAX_DEVICES];

}  // namespace

static_assert(TRBT_B2F_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[TRBT_B2F_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
int b2f_scratch(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TRBT_ERR_HIP;
    if (dev < 0 || dev >= B2F_MAX_DEVICES) return TRBT_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(b2f_scratch_mu);
    if (!b2f_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return TRBT_ERR_HIP;
        }
        b2f_scratch_ptr[dev] = p;
    }
    *out = b2f_scratch_ptr[dev];
    return TRBT_SUCCESS;
}

}  // namespace

extern "C" {

int trbt_band_to_full_workspace_bytes(int64_t n, int nbw, int64_t nev, int is_complex,
                                      size_t* bytes)
{
    if (n < 0) return -1;
    if (nbw < 1) return -2;
    if (nev < 0 || nev > n) return -3;
    if (!bytes) return -4;
    *bytes = nev > 0 ? b2f_bytes(n, nbw, is_complex != 0) : 0;
    return TRBT_SUCCESS;
}

int trans_ev_band_to_full_d(int64_t n, int nbw, int64_t nev, const double* hh_v, int64_t ldv,
                            const double* hh_tau, double* Z, int64_t ldz, void* work,
                            size_t work_bytes, void* stream)
{
    return b2f_run<false>(n, nbw, nev, hh_v, ldv, hh_tau, Z, ldz, work, work_bytes, stream);
}

int trans_ev_band_to_full_z(int64_t n, int nbw, int64_t nev, const trbt_z* hh_v, int64_t ldv,
                            const trbt_z* hh_tau, trbt_z* Z, int64_t ldz, void* work,
                            size_t work_bytes, void* stream)
{
    return b2f_run<true>(n, nbw, nev, (const double*)hh_v, ldv, (const double*)hh_tau,
                         (double*)Z, ldz, work, work_bytes, stream);
}

int trans_ev_band_to_full_z_noalloc(int64_t n, int nbw, int64_t nev, const trbt_z* hh_v,
                                    int64_t ldv, const trbt_z* hh_tau, trbt_z* Z, int64_t ldz,
                                    void* stream)
{
    int rc = b2f_validate<true>(n, nbw, nev, hh_v, ldv, hh_tau, Z, ldz, nullptr, 0);
    if (rc) return rc;
    if (b2f_reflectors(n, nbw) == 0 || nev == 0) return TRBT_SUCCESS;
    if (b2f_bytes(n, nbw, true) > TRBT_B2F_SCRATCH_BYTES) return TRBT_ERR_SCRATCH;
    rc = check_device();
    if (rc) return rc;
    void* s = nullptr;
    rc = b2f_scratch(&s);
    if (rc) return rc;
    return b2f_run<true>(n, nbw, nev, (const double*)hh_v, ldv, (const double*)hh_tau,
                         (double*)Z, ldz, s, TRBT_B2F_SCRATCH_BYTES, stream);
}

}  // extern "C"
