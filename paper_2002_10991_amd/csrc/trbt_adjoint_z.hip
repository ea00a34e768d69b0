// trbt_adjoint_z.hip -- adjoint of the complex back-transformation
// (Eq. 2stage_bkwd1 with complex reflectors H_k = I - tau_k v_k v_k^H) for
// a real loss, in the conjugate-Wirtinger convention: every gradient grad_x
// satisfies dL = Re sum conj(grad_x) dx.  For one column update
// z' = z - tau v (v^H z), with w = v^H z, gamma = v^H g (g = grad z'):
//   grad z   = g - conj(tau) gamma v
//   grad tau = -conj(w) gamma                       (summed over columns)
//   grad v   = -conj(tau) conj(w) g - tau conj(gamma) z   (summed over columns)
//
// Stage-parallel form.  The reflectors of one stage act on disjoint rows
// (Sec. 2.2.2), so a stage is one launch over (slot, 256-column chunk)
// workgroups, one thread per column.  Z and G are first transposed into a
// row-major working layout (row r of the working copy holds that row of every
// column, contiguous), so the threads of a workgroup read consecutive
// addresses.
//   forward:  stages n-3 .. 0; before each 16-stage segment [sbot, stop]
//             rows [sbot+1, n) (the only rows the segment touches) are
//             checkpointed;
//   backward: segments from the lowest stages up: restore the checkpoint,
//             recompute the segment writing each stage's input rows
//             [s+1, n) to the tape, then walk its stages in generation order
//             (ascending s), updating the gradient in place and writing each
//             workgroup's column sums of grad v, grad tau as a partial;
//   finish:   partials summed over the column chunks in chunk order (the
//             result is bitwise reproducible) and the gradient of Z_in
//             transposed back into the caller's G.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include "trbt.h"
#include "trbt_device.h"

namespace {

constexpr int ZC = 256;    // columns per workgroup (one per thread)
constexpr int ZSEG = 16;   // stages per checkpointed segment
constexpr int ZR = 16;     // gradient entries per LDS reduction round
constexpr int ZL = 16;     // rows loaded together (loads in flight per thread)

__host__ __device__ inline int64_t zseg_lo(int64_t n, int64_t t)   // lowest stage of segment t
{
    const int64_t stop = n - 3 - ZSEG * t;
    return stop - (ZSEG - 1) > 0 ? stop - (ZSEG - 1) : 0;
}

// column-major (ld) <-> row-major working layout, complex (2 doubles)
__global__ __launch_bounds__(256) void k_z_to_rows(int64_t n, int64_t nev,
                                                   const double* __restrict__ src, int64_t ld,
                                                   double* __restrict__ dst)
{
    __shared__ double tile[32][33 * 2];
    const int64_t c0 = (int64_t)blockIdx.y * 32, r0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int q = ty; q < 32; q += 8) {
        const int64_t c = c0 + q, r = r0 + tx;
        if (c < nev && r < n) {
            tile[q][2 * tx] = src[(c * ld + r) * 2];
            tile[q][2 * tx + 1] = src[(c * ld + r) * 2 + 1];
        }
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t r = r0 + q, c = c0 + tx;
        if (c < nev && r < n) {
            dst[(r * nev + c) * 2] = tile[tx][2 * q];
            dst[(r * nev + c) * 2 + 1] = tile[tx][2 * q + 1];
        }
    }
}

__global__ __launch_bounds__(256) void k_rows_to_z(int64_t n, int64_t nev,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ dst, int64_t ld)
{
    __shared__ double tile[32][33 * 2];
    const int64_t c0 = (int64_t)blockIdx.y * 32, r0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int q = ty; q < 32; q += 8) {
        const int64_t r = r0 + q, c = c0 + tx;
        if (c < nev && r < n) {
            tile[q][2 * tx] = src[(r * nev + c) * 2];
            tile[q][2 * tx + 1] = src[(r * nev + c) * 2 + 1];
        }
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t c = c0 + q, r = r0 + tx;
        if (c < nev && r < n) {
            dst[(c * ld + r) * 2] = tile[tx][2 * q];
            dst[(c * ld + r) * 2 + 1] = tile[tx][2 * q + 1];
        }
    }
}

// One stage of the forward transformation on the working copy W (rows
// [0, n)); with tape != null the stage's input rows [s+1, n) are also
// written to tape (row-major, row s+1 first).
__global__ __launch_bounds__(ZC) void k_zstage_fwd(int64_t n, int nbw, int64_t nev, int64_t s,
                                                   const double* __restrict__ hv,
                                                   const double* __restrict__ ht,
                                                   double* __restrict__ W,
                                                   double* __restrict__ tape)
{
    const int64_t j = blockIdx.x;
    const int64_t c = (int64_t)blockIdx.y * ZC + threadIdx.x;
    const int64_t r0 = s + 1 + j * nbw;
    const int len = (int)(n - r0 < nbw ? n - r0 : nbw);
    const int64_t k = stage_offset(n, nbw, s) + j;
    const double* v = hv + k * nbw * 2;
    if (c >= nev) return;
    // rows are read ZL at a time, all loads issued before any is used
    double dr = 0.0, di = 0.0;   // v^H z
    for (int i0 = 0; i0 < len; i0 += ZL) {
        double zr[ZL], zi[ZL];
#pragma unroll
        for (int q = 0; q < ZL; ++q) {
            zr[q] = zi[q] = 0.0;
            if (i0 + q < len) {
                const double* zp = &W[((r0 + i0 + q) * nev + c) * 2];
                zr[q] = zp[0];
                zi[q] = zp[1];
            }
        }
#pragma unroll
        for (int q = 0; q < ZL; ++q) {
            if (i0 + q < len) {
                const int i = i0 + q;
                if (tape) {
                    double* tp = &tape[((r0 + i - s - 1) * nev + c) * 2];
                    tp[0] = zr[q];
                    tp[1] = zi[q];
                }
                const double vr = v[2 * i], vi = v[2 * i + 1];
                dr = fma(vr, zr[q], fma(vi, zi[q], dr));
                di = fma(vr, zi[q], fma(-vi, zr[q], di));
            }
        }
    }
    const double tr = ht[2 * k], ti = ht[2 * k + 1];
    const double ar = tr * dr - ti * di, ai = tr * di + ti * dr;   // tau (v^H z)
    for (int i0 = 0; i0 < len; i0 += ZL) {
        double zr[ZL], zi[ZL];
#pragma unroll
        for (int q = 0; q < ZL; ++q) {
            zr[q] = zi[q] = 0.0;
            if (i0 + q < len) {
                const double* zp = &W[((r0 + i0 + q) * nev + c) * 2];
                zr[q] = zp[0];
                zi[q] = zp[1];
            }
        }
#pragma unroll
        for (int q = 0; q < ZL; ++q) {
            if (i0 + q < len) {
                const int i = i0 + q;
                double* zp = &W[((r0 + i) * nev + c) * 2];
                const double vr = v[2 * i], vi = v[2 * i + 1];
                zp[0] = zr[q] - (ar * vr - ai * vi);
                zp[1] = zi[q] - (ar * vi + ai * vr);
            }
        }
    }
}

// One stage of the reverse sweep: the gradient rows of every column through
// the stage's reflectors, and this workgroup's column sums of grad v (entries
// 0..len-1) and grad tau (entry nbw):
//   part[((chunk * K + k) * (nbw + 1) + e) * 2 + {re, im}]
__global__ __launch_bounds__(ZC) void k_zstage_bwd(int64_t n, int nbw, int64_t nev, int64_t s,
                                                   int64_t K, const double* __restrict__ hv,
                                                   const double* __restrict__ ht,
                                                   const double* __restrict__ tape,
                                                   double* __restrict__ Gw,
                                                   double* __restrict__ part)
{
    __shared__ double red[ZC][2 * ZR + 1];
    const int tid = threadIdx.x;
    const int64_t j = blockIdx.x, chunk = blockIdx.y;
    const int64_t c = chunk * ZC + tid;
    const bool valid = c < nev;
    const int64_t cc = valid ? c : 0;
    const int64_t r0 = s + 1 + j * nbw;
    const int len = (int)(n - r0 < nbw ? n - r0 : nbw);
    const int64_t k = stage_offset(n, nbw, s) + j;
    const double* v = hv + k * nbw * 2;
    const double tr = ht[2 * k], ti = ht[2 * k + 1];
    auto gp = [&](int i) { return &Gw[((r0 + i) * nev + cc) * 2]; };
    auto zp = [&](int i) { return &tape[((r0 + i - s - 1) * nev + cc) * 2]; };
    double gr = 0.0, gi = 0.0, wr = 0.0, wi = 0.0;   // gamma = v^H g, w = v^H z
    if (valid)
        for (int i0 = 0; i0 < len; i0 += ZL) {   // ZL rows of g and z in flight
            double xr[ZL], xi[ZL], yr[ZL], yi[ZL];
#pragma unroll
            for (int q = 0; q < ZL; ++q) {
                xr[q] = xi[q] = yr[q] = yi[q] = 0.0;
                if (i0 + q < len) {
                    const double* x = gp(i0 + q);
                    const double* z = zp(i0 + q);
                    xr[q] = x[0];
                    xi[q] = x[1];
                    yr[q] = z[0];
                    yi[q] = z[1];
                }
            }
#pragma unroll
            for (int q = 0; q < ZL; ++q) {
                if (i0 + q < len) {
                    const double vr = v[2 * (i0 + q)], vi = v[2 * (i0 + q) + 1];
                    gr = fma(vr, xr[q], fma(vi, xi[q], gr));
                    gi = fma(vr, xi[q], fma(-vi, xr[q], gi));
                    wr = fma(vr, yr[q], fma(vi, yi[q], wr));
                    wi = fma(vr, yi[q], fma(-vi, yr[q], wi));
                }
            }
        }
    // a = -conj(tau) conj(w), b = -tau conj(gamma)
    const double ar = -(tr * wr - ti * wi), ai = -(-tr * wi - ti * wr);
    const double br = -(tr * gr + ti * gi), bi = -(ti * gr - tr * gi);
    const double fr = tr * gr + ti * gi, fi = tr * gi - ti * gr;   // conj(tau) gamma
    for (int e0 = 0; e0 <= len; e0 += ZR) {
        // this round's rows of g and z (loads issued together); the
        // contributions use the incoming g, which is then updated in place:
        // g <- g - conj(tau) gamma v
        double xr[ZR], xi[ZR], yr[ZR], yi[ZR];
#pragma unroll
        for (int q = 0; q < ZR; ++q) {
            xr[q] = xi[q] = yr[q] = yi[q] = 0.0;
            if (valid && e0 + q < len) {
                const double* x = gp(e0 + q);
                const double* z = zp(e0 + q);
                xr[q] = x[0];
                xi[q] = x[1];
                yr[q] = z[0];
                yi[q] = z[1];
            }
        }
#pragma unroll
        for (int q = 0; q < ZR; ++q) {
            const int e = e0 + q;
            double vr = 0.0, vi = 0.0;
            if (valid && e < len) {
                vr = ar * xr[q] - ai * xi[q] + br * yr[q] - bi * yi[q];
                vi = ar * xi[q] + ai * xr[q] + br * yi[q] + bi * yr[q];
                const double wvr = v[2 * e], wvi = v[2 * e + 1];
                double* x = gp(e);
                x[0] = xr[q] - (fr * wvr - fi * wvi);
                x[1] = xi[q] - (fr * wvi + fi * wvr);
            } else if (valid && e == len) {   // -conj(w) gamma
                vr = -(wr * gr + wi * gi);
                vi = -(wr * gi - wi * gr);
            }
            red[tid][2 * q] = vr;
            red[tid][2 * q + 1] = vi;
        }
        __syncthreads();
        if (tid < 2 * ZR && e0 + tid / 2 <= len) {
            double acc = 0.0;
            for (int l = 0; l < ZC; ++l) acc += red[l][tid];
            const int e = e0 + tid / 2;
            part[((chunk * K + k) * (nbw + 1) + (e < len ? e : nbw)) * 2 + (tid & 1)] = acc;
        }
        __syncthreads();
    }
}

// grad v, grad tau = sums of the chunks' partials in chunk order; zero
// beyond each reflector's length.
__global__ __launch_bounds__(256) void k_zfinish(int64_t n, int nbw, int64_t K, int64_t nchunk,
                                                 const double* __restrict__ part,
                                                 double* __restrict__ dv,
                                                 double* __restrict__ dtau)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= K * (nbw + 1)) return;
    const int64_t k = idx / (nbw + 1);
    const int e = (int)(idx % (nbw + 1));
    int64_t lo = 0, hi = n - 2;   // the reflector's stage: largest s with offset <= k
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (stage_offset(n, nbw, mid) <= k) lo = mid; else hi = mid;
    }
    const int64_t r0 = lo + 1 + (k - stage_offset(n, nbw, lo)) * nbw;
    const int len = (int)(n - r0 < nbw ? n - r0 : nbw);
    for (int q = 0; q < 2; ++q) {
        if (e < nbw && e >= len) {
            dv[(k * nbw + e) * 2 + q] = 0.0;
            continue;
        }
        double acc = 0.0;
        for (int64_t ch = 0; ch < nchunk; ++ch)
            acc += part[((ch * K + k) * (nbw + 1) + e) * 2 + q];
        if (e == nbw) dtau[k * 2 + q] = acc;
        else dv[(k * nbw + e) * 2 + q] = acc;
    }
}

__global__ void k_zfill(double* p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

struct ZLayout {
    size_t zw = 0, gw = 0, ck = 0, tape = 0, part = 0, total = 0;
    int64_t nseg = 0, nchunk = 0;
};

size_t zal(size_t x) { return (x + 255) / 256 * 256; }

ZLayout zlayout(int64_t n, int nbw, int64_t nev)
{
    ZLayout L;
    const size_t row = (size_t)nev * 16;   // one row of the working layout
    size_t off = 256;
    L.zw = off;
    off = zal(off + (size_t)n * row);
    L.gw = off;
    off = zal(off + (size_t)n * row);
    L.nseg = (n - 2 + ZSEG - 1) / ZSEG;
    size_t ckrows = 0, taperows = 0;
    for (int64_t t = 0; t < L.nseg; ++t) {
        const int64_t lo = zseg_lo(n, t), stop = n - 3 - ZSEG * t;
        ckrows += (size_t)(n - lo - 1);
        size_t rows = 0;
        for (int64_t s = lo; s <= stop; ++s) rows += (size_t)(n - s - 1);
        taperows = rows > taperows ? rows : taperows;
    }
    L.ck = off;
    off = zal(off + ckrows * row);
    L.tape = off;
    off = zal(off + taperows * row);
    L.nchunk = (nev + ZC - 1) / ZC;
    L.part = off;
    off = zal(off + (size_t)L.nchunk * num_reflectors(n, nbw) * (nbw + 1) * 16);
    L.total = off;
    return L;
}

}  // namespace

// The blocked (compact-WY, FP64 MFMA) complex adjoint of trbt_adjoint.hip,
// taken for nbw in {16, 32, 48, 64}.
size_t trbt_adjoint_blocked_bytes_z(int64_t n, int nbw, int64_t nev);
int trbt_adjoint_blocked_z(int64_t n, int nbw, int64_t nev, const double* hv, const double* ht,
                           const double* Z_in, int64_t ldz, double* G, int64_t ldg, double* dv,
                           double* dtau, void* work, size_t work_bytes, hipStream_t st);

extern "C" {

int trbt_adjoint_workspace_bytes_z(int64_t n, int nbw, int64_t nev, int ckpt_every,
                                   size_t* bytes)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (nev < 0 || nev > n) return -3;
    if (ckpt_every != 0 && ckpt_every != 16) return -4;
    if (!bytes) return -5;
    if (num_reflectors(n, nbw) == 0 || nev == 0)
        *bytes = 0;
    else if (use_blocked(n, nbw, true))
        *bytes = trbt_adjoint_blocked_bytes_z(n, nbw, nev);
    else
        *bytes = zlayout(n, nbw, nev).total;
    return TRBT_SUCCESS;
}

int trans_ev_tridi_to_band_adjoint_z(int64_t n, int nbw, int64_t nev, const trbt_z* hh_v,
                                     const trbt_z* hh_tau, const trbt_z* Z_in, int64_t ldz,
                                     trbt_z* G, int64_t ldg, trbt_z* dv, trbt_z* dtau,
                                     int ckpt_every, void* work, size_t work_bytes,
                                     void* stream)
{
    // argument checks in the order (and with the codes) of the real adjoint
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (nev < 0 || nev > n) return -3;
    const int64_t K = num_reflectors(n, nbw);
    const bool cols = nev > 0 && n > 0;
    if (K > 0 && !hh_v) return -4;
    if (K > 0 && !hh_tau) return -5;
    if (cols && K > 0 && !Z_in) return -6;
    if (ldz < (n > 1 ? n : 1)) return -7;
    if (cols && K > 0 && !G) return -8;
    if (ldg < (n > 1 ? n : 1)) return -9;
    if (K > 0 && !dv) return -10;
    if (K > 0 && !dtau) return -11;
    if (ckpt_every != 0 && ckpt_every != 16) return -12;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -13;
    if (work_bytes && !work) return -13;
    if (K == 0) return TRBT_SUCCESS;   // grad Z_in = G, nothing else to write
    int rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    double* dvp = (double*)dv;
    double* dtp = (double*)dtau;
    if (nev == 0) {
        hipLaunchKernelGGL(k_zfill, dim3((unsigned)((2 * K * nbw + 255) / 256)), dim3(256), 0, st,
                           dvp, 2 * K * nbw);
        hipLaunchKernelGGL(k_zfill, dim3((unsigned)((2 * K + 255) / 256)), dim3(256), 0, st, dtp,
                           2 * K);
        return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
    }
    if (use_blocked(n, nbw, true))
        return trbt_adjoint_blocked_z(n, nbw, nev, (const double*)hh_v, (const double*)hh_tau,
                                      (const double*)Z_in, ldz, (double*)G, ldg, dvp, dtp, work,
                                      work_bytes, st);
    const ZLayout L = zlayout(n, nbw, nev);
    if (!work || work_bytes < L.total) return TRBT_ERR_WORKSPACE;
    char* ws = (char*)work;
    // fault word: this form has no inter-workgroup waits, so it stays clear
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (unsigned*)work, 64);
    double* Zw = (double*)(ws + L.zw);
    double* Gw = (double*)(ws + L.gw);
    double* ck = (double*)(ws + L.ck);
    double* tape = (double*)(ws + L.tape);
    double* part = (double*)(ws + L.part);
    const double* hv = (const double*)hh_v;
    const double* ht = (const double*)hh_tau;
    const size_t row = (size_t)nev * 16;
    const dim3 tg((unsigned)((n + 31) / 32), (unsigned)((nev + 31) / 32));
    hipLaunchKernelGGL(k_z_to_rows, tg, dim3(256), 0, st, n, nev, (const double*)Z_in, ldz, Zw);
    hipLaunchKernelGGL(k_z_to_rows, tg, dim3(256), 0, st, n, nev, (const double*)G, ldg, Gw);
    const unsigned nch = (unsigned)L.nchunk;

    // forward with a checkpoint before every segment
    size_t ckoff = 0;
    for (int64_t t = 0; t < L.nseg; ++t) {
        const int64_t lo = zseg_lo(n, t), stop = n - 3 - ZSEG * t;
        const size_t bytes = (size_t)(n - lo - 1) * row;
        if (hipMemcpyAsync((char*)ck + ckoff, (char*)Zw + (size_t)(lo + 1) * row, bytes,
                           hipMemcpyDeviceToDevice, st) != hipSuccess)
            return TRBT_ERR_HIP;
        ckoff += bytes;
        for (int64_t s = stop; s >= lo; --s)
            hipLaunchKernelGGL(k_zstage_fwd, dim3((unsigned)sweeps_in_stage(n, nbw, s), nch),
                               dim3(ZC), 0, st, n, nbw, nev, s, hv, ht, Zw, (double*)nullptr);
    }
    // reverse sweep, segments from the lowest stages up
    for (int64_t t = L.nseg - 1; t >= 0; --t) {
        const int64_t lo = zseg_lo(n, t), stop = n - 3 - ZSEG * t;
        const size_t bytes = (size_t)(n - lo - 1) * row;
        ckoff -= bytes;
        if (hipMemcpyAsync((char*)Zw + (size_t)(lo + 1) * row, (char*)ck + ckoff, bytes,
                           hipMemcpyDeviceToDevice, st) != hipSuccess)
            return TRBT_ERR_HIP;
        // tape: stage s's input rows [s+1, n), stages stop .. lo in this order
        size_t toff = 0;
        for (int64_t s = stop; s >= lo; --s) {
            hipLaunchKernelGGL(k_zstage_fwd, dim3((unsigned)sweeps_in_stage(n, nbw, s), nch),
                               dim3(ZC), 0, st, n, nbw, nev, s, hv, ht, Zw,
                               (double*)((char*)tape + toff));
            toff += (size_t)(n - s - 1) * row;
        }
        for (int64_t s = lo; s <= stop; ++s) {
            toff -= (size_t)(n - s - 1) * row;
            hipLaunchKernelGGL(k_zstage_bwd, dim3((unsigned)sweeps_in_stage(n, nbw, s), nch),
                               dim3(ZC), 0, st, n, nbw, nev, s, K, hv, ht,
                               (const double*)((char*)tape + toff), Gw, part);
        }
    }
    const int64_t cnt = K * (nbw + 1);
    hipLaunchKernelGGL(k_zfinish, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, n, nbw,
                       K, L.nchunk, (const double*)part, dvp, dtp);
    hipLaunchKernelGGL(k_rows_to_z, tg, dim3(256), 0, st, n, nev, (const double*)Gw, (double*)G,
                       ldg);
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

}  // extern "C"
