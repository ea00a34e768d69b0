// trbt_tridiag.hip -- the lowest nev eigenpairs of a real symmetric
// tridiagonal matrix T = diag(d) + subdiag(e) on AMD Instinct MI355X
// (gfx950): the tridiagonal step of the two-stage solver (Eq. 2stage_solve),
// between the bulge chasing and the back-transformation.  Only the wanted
// eigenvectors are computed.
//
// Method (the classical pair, one thread per wanted eigenpair; the paper's
// solver is divide and conquer, which reaches the same eigenpairs):
//   * eigenvalue i by multisection on the Sturm count: the number of
//     negative pivots of the LDL^T factorisation of T - x I equals the number
//     of eigenvalues below x (Sylvester's law of inertia); the interval
//     starts from the Gershgorin bounds and is cut into 17 by 16 lanes per
//     eigenvalue until it is no wider than a few ulps of its end points;
//   * eigenvector i by inverse iteration with that eigenvalue: two solves
//     (T - lambda I) x_{k+1} = x_k / ||x_k|| by Gaussian elimination with
//     partial pivoting (the tridiagonal LU: U with two superdiagonals), from
//     a fixed pseudo-random start; an exactly zero pivot is replaced by
//     eps ||T||.  The factors live in the workspace, row-major across the
//     eigenvectors, so the threads of a wave read and write consecutive
//     addresses; the vectors are transposed into Z at the end.
// Accuracy: residual ||T x - lambda x|| ~ eps ||T||; the angle between
// computed eigenvectors of eigenvalues a gap apart ~ eps ||T|| / gap.
// Eigenvalues closer than 1e-6 ||T|| to their predecessor form a cluster:
// its vectors (each an inverse iterate from a different start, so together
// spanning the cluster's invariant subspace) are orthonormalised by modified
// Gram-Schmidt, one workgroup per cluster, so (near-)degenerate eigenvalues
// get an orthonormal basis of their subspace.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "trbt.h"
#include "trbt_device.h"
#include "trbt_lanes.h"

namespace {

constexpr int TD_THREADS = 64;
constexpr int TD_ITERS = 2;
// eigenvalues closer than this times ||T|| to their predecessor are one
// cluster, whose vectors are orthonormalised together afterwards; outside
// clusters the angle error of inverse iteration is below about eps / TD_CLUSTER
constexpr double TD_CLUSTER = 1e-6;

// number of eigenvalues of T strictly below x
__device__ inline int64_t sturm_count(int64_t n, const double* __restrict__ d,
                                      const double* __restrict__ e2, double x, double pivmin)
{
    int64_t cnt = 0;
    double t = d[0] - x;
    if (fabs(t) < pivmin) t = -pivmin;
    cnt += t < 0.0;
    for (int64_t k = 1; k < n; ++k) {
        t = d[k] - x - e2[k - 1] / t;
        if (fabs(t) < pivmin) t = -pivmin;
        cnt += t < 0.0;
    }
    return cnt;
}

// e2 = e^2; bounds[0..1] = Gershgorin interval, bounds[2] = max |T|-ish
// norm estimate (max row sum), bounds[3] = pivmin.  One workgroup.
__global__ __launch_bounds__(256) void k_td_prep(int64_t n, const double* __restrict__ d,
                                                 const double* __restrict__ e,
                                                 double* __restrict__ e2,
                                                 double* __restrict__ bounds)
{
    __shared__ double lo_s[256], hi_s[256], nm_s[256], em_s[256];
    double lo = INFINITY, hi = -INFINITY, nm = 0.0, em = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += 256) {
        const double a = k > 0 ? fabs(e[k - 1]) : 0.0, b = k + 1 < n ? fabs(e[k]) : 0.0;
        lo = fmin(lo, d[k] - a - b);
        hi = fmax(hi, d[k] + a + b);
        nm = fmax(nm, fabs(d[k]) + a + b);
        if (k + 1 < n) {
            e2[k] = e[k] * e[k];
            em = fmax(em, e2[k]);
        }
    }
    lo_s[threadIdx.x] = lo;
    hi_s[threadIdx.x] = hi;
    nm_s[threadIdx.x] = nm;
    em_s[threadIdx.x] = em;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256; ++i) {
            lo = fmin(lo, lo_s[i]);
            hi = fmax(hi, hi_s[i]);
            nm = fmax(nm, nm_s[i]);
            em = fmax(em, em_s[i]);
        }
        const double eps = 2.220446049250313e-16;
        const double pad = 2.0 * eps * fmax(fabs(lo), fabs(hi)) + 2.0 * eps * n * nm + 1e-300;
        bounds[0] = lo - pad;
        bounds[1] = hi + pad;
        bounds[2] = nm > 0.0 ? nm : 1.0;
        bounds[3] = fmax(2.2250738585072014e-308 * fmax(em, 1.0), 1e-290);
    }
}

// eigenvalue i (0-based, ascending) by multisection: TD_MS consecutive lanes
// share one eigenvalue and evaluate the Sturm count at TD_MS interior points
// of its interval, x_k = lo + (hi - lo)(k+1)/(TD_MS+1); the new interval is
// [x_{k*-1}, x_{k*}] for the first point k* with count > i, read from the
// group's bits of a wave ballot (every lane of the group computes the same
// end points from the same formula).
constexpr int TD_MS = 16;

__global__ __launch_bounds__(TD_THREADS) void k_td_bisect(int64_t n, int64_t nev,
                                                          const double* __restrict__ d,
                                                          const double* __restrict__ e2,
                                                          const double* __restrict__ bounds,
                                                          double* __restrict__ w)
{
    const int64_t gid = (int64_t)blockIdx.x * TD_THREADS + threadIdx.x;
    const int64_t i = gid / TD_MS;
    const int k = (int)(gid % TD_MS);
    const int gbit = (threadIdx.x & 63) & ~(TD_MS - 1);   // the group's first lane in the wave
    if (i >= nev) return;   // whole groups leave together
    double lo = bounds[0], hi = bounds[1];
    const double pivmin = bounds[3];
    const double eps = 2.220446049250313e-16;
    // invariant: count(lo) <= i < count(hi)
    for (int it = 0; it < 100; ++it) {
        if (hi - lo <= 4.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) break;
        const double step = (hi - lo) / (TD_MS + 1);
        const double x = lo + step * (k + 1);
        const bool above = sturm_count(n, d, e2, x, pivmin) > i;
        const unsigned grp = (unsigned)((__ballot(above) >> gbit) & ((1u << TD_MS) - 1));
        double nlo = lo, nhi = hi;
        if (grp) {
            const int ks = __builtin_ctz(grp);
            nhi = lo + step * (ks + 1);
            if (ks > 0) nlo = lo + step * ks;
        } else {
            nlo = lo + step * TD_MS;
        }
        if (nlo == lo && nhi == hi) break;   // no representable progress
        lo = nlo;
        hi = nhi;
    }
    if (k == 0) w[i] = 0.5 * (lo + hi);
}

// a fixed pseudo-random start in [-1, 1) (splitmix64 of (vector, row))
__device__ inline double td_start(int64_t i, int64_t r)
{
    uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + (uint64_t)r * 0xD1B54A32D192ED03ull + 1;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// eigenvector i by inverse iteration.  Row-major across the eigenvectors:
//   X[r * nev + i]        the iterate,
//   F[(r * 4 + q) * nev + i]  row r of the LU of T - lambda I: q = 0 the
//                          pivot (U's diagonal), 1 and 2 U's superdiagonals,
//                          3 the multiplier,
//   P[r * nev + i]        1 when rows r and r+1 were swapped.
// The recurrences run row by row, with the loads of TD_CH rows issued
// together (one thread per eigenvector leaves few waves to hide latency).
constexpr int TD_CH = 16;

__global__ __launch_bounds__(TD_THREADS) void k_td_invit(int64_t n, int64_t nev,
                                                         const double* __restrict__ d,
                                                         const double* __restrict__ e,
                                                         const double* __restrict__ bounds,
                                                         const double* __restrict__ w,
                                                         double* __restrict__ X,
                                                         double* __restrict__ F,
                                                         unsigned char* __restrict__ P)
{
    const int64_t i = (int64_t)blockIdx.x * TD_THREADS + threadIdx.x;
    if (i >= nev) return;
    const double lam = w[i];
    const double eps = 2.220446049250313e-16;
    const double tiny = eps * bounds[2];
    double* Xi = X + i;
    double* Fi = F + i;
    unsigned char* Pi = P + i;
    const int64_t s4 = 4 * nev;   // stride of a row of F

    // LU with partial pivoting of T - lam I.  The current row (to become
    // U's row k, or to be swapped with row k+1) has pivot candidate a in
    // column k and bsup in column k+1.
    double a = d[0] - lam;
    double bsup = n > 1 ? e[0] : 0.0;
    for (int64_t k = 0; k + 1 < n; ++k) {
        const double sub = e[k];                      // T(k+1, k)
        const double dn = d[k + 1] - lam;             // T(k+1, k+1)
        const double en = k + 2 < n ? e[k + 1] : 0.0; // T(k+1, k+2)
        double* fr = Fi + k * s4;
        if (fabs(a) >= fabs(sub)) {
            const double piv = a != 0.0 ? a : tiny;
            const double l = sub / piv;
            fr[0] = piv;
            fr[nev] = bsup;
            fr[2 * nev] = 0.0;
            fr[3 * nev] = l;
            Pi[k * nev] = 0;
            a = dn - l * bsup;
            bsup = en;
        } else {
            const double l = a / sub;   // rows k and k+1 swapped
            fr[0] = sub;
            fr[nev] = dn;
            fr[2 * nev] = en;
            fr[3 * nev] = l;
            Pi[k * nev] = 1;
            a = bsup - l * dn;
            bsup = -l * en;
        }
    }
    {
        double* fr = Fi + (n - 1) * s4;
        fr[0] = a != 0.0 ? a : tiny;
        fr[nev] = fr[2 * nev] = fr[3 * nev] = 0.0;
    }
    for (int64_t r = 0; r < n; ++r) Xi[r * nev] = td_start(i, r);

    for (int it = 0; it <= TD_ITERS; ++it) {
        // 1 / ||x||
        double ss = 0.0;
        for (int64_t r0 = 0; r0 < n; r0 += TD_CH) {
            double v[TD_CH];
#pragma unroll
            for (int q = 0; q < TD_CH; ++q) v[q] = r0 + q < n ? Xi[(r0 + q) * nev] : 0.0;
#pragma unroll
            for (int q = 0; q < TD_CH; ++q) ss = fma(v[q], v[q], ss);
        }
        const double inv = 1.0 / sqrt(ss);
        if (it == TD_ITERS) {
            // normalise; sign: the largest-magnitude entry positive (the
            // first of equal ones)
            double big = 0.0, sg = 1.0;
            for (int64_t r0 = 0; r0 < n; r0 += TD_CH) {
                double v[TD_CH];
#pragma unroll
                for (int q = 0; q < TD_CH; ++q) v[q] = r0 + q < n ? Xi[(r0 + q) * nev] : 0.0;
#pragma unroll
                for (int q = 0; q < TD_CH; ++q)
                    if (fabs(v[q]) > big) {
                        big = fabs(v[q]);
                        sg = v[q] < 0.0 ? -1.0 : 1.0;
                    }
            }
            const double sc = sg * inv;
            for (int64_t r = 0; r < n; ++r) Xi[r * nev] *= sc;
            break;
        }
        // forward: row swaps and multipliers on x / ||x|| (in place: row k
        // of the result is written once row k+1 has been read)
        double carry = Xi[0] * inv;
        for (int64_t k0 = 0; k0 + 1 < n; k0 += TD_CH) {
            double nx[TD_CH], lq[TD_CH];
            unsigned char pq[TD_CH];
#pragma unroll
            for (int q = 0; q < TD_CH; ++q) {
                const int64_t k = k0 + q;
                nx[q] = lq[q] = 0.0;
                pq[q] = 0;
                if (k + 1 < n) {
                    nx[q] = Xi[(k + 1) * nev] * inv;
                    lq[q] = Fi[k * s4 + 3 * nev];
                    pq[q] = Pi[k * nev];
                }
            }
#pragma unroll
            for (int q = 0; q < TD_CH; ++q) {
                const int64_t k = k0 + q;
                if (k + 1 < n) {
                    if (pq[q]) {
                        Xi[k * nev] = nx[q];
                        carry = carry - lq[q] * nx[q];
                    } else {
                        Xi[k * nev] = carry;
                        carry = nx[q] - lq[q] * carry;
                    }
                }
            }
        }
        Xi[(n - 1) * nev] = carry;
        // backward with U
        double x1 = 0.0, x2 = 0.0;   // solution rows k+1, k+2
        for (int64_t k0 = n - 1; k0 >= 0; k0 -= TD_CH) {
            double yq[TD_CH], u0[TD_CH], u1[TD_CH], u2[TD_CH];
#pragma unroll
            for (int q = 0; q < TD_CH; ++q) {
                const int64_t k = k0 - q;
                yq[q] = u1[q] = u2[q] = 0.0;
                u0[q] = 1.0;
                if (k >= 0) {
                    yq[q] = Xi[k * nev];
                    u0[q] = Fi[k * s4];
                    u1[q] = Fi[k * s4 + nev];
                    u2[q] = Fi[k * s4 + 2 * nev];
                }
            }
#pragma unroll
            for (int q = 0; q < TD_CH; ++q) {
                const int64_t k = k0 - q;
                if (k >= 0) {
                    const double v = (yq[q] - u1[q] * x1 - u2[q] * x2) / u0[q];
                    Xi[k * nev] = v;
                    x2 = x1;
                    x1 = v;
                }
            }
        }
    }
}

// Modified Gram-Schmidt over each cluster of size >= 2 (one workgroup per
// eigenvalue index; only cluster starts with a successor in the cluster do
// work).  Vectors in the output Z (column-major, vector j = Z[j * ldz ..],
// contiguous, so the workgroup's threads read consecutive rows), already
// unit.
__global__ __launch_bounds__(256) void k_td_ortho(int64_t n, int64_t nev,
                                                  const double* __restrict__ w,
                                                  const double* __restrict__ bounds,
                                                  double* __restrict__ Z, int64_t ldz)
{
    // one partial per wave, double-buffered by call parity: each thread only
    // ever touches its own rows of Z (r = tid mod 256), so the sums are the
    // only exchange, and one barrier per sum suffices (a wave can reach the
    // next sum's writes only after every wave has passed this one's barrier)
    __shared__ double red[2][4];
    const int64_t i = blockIdx.x;
    const double thr = TD_CLUSTER * bounds[2];
    if (i > 0 && w[i] - w[i - 1] <= thr) return;            // not a cluster start
    if (i + 1 >= nev || w[i + 1] - w[i] > thr) return;       // a single eigenvalue
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int parity = 0;
    auto block_sum = [&](double v) {
        v = wave_sum(v);
        if (lane == 0) red[parity][wv] = v;
        __syncthreads();
        const double s = (red[parity][0] + red[parity][1]) + (red[parity][2] + red[parity][3]);
        parity ^= 1;
        return s;
    };
    for (int64_t j = i + 1; j < nev && w[j] - w[j - 1] <= thr; ++j) {
        double* __restrict__ zj = Z + j * ldz;
        for (int64_t m = i; m < j; ++m) {
            const double* __restrict__ zm = Z + m * ldz;
            double p = 0.0;
            for (int64_t r = tid; r < n; r += 256) p = fma(zj[r], zm[r], p);
            const double dt = block_sum(p);
            for (int64_t r = tid; r < n; r += 256) zj[r] = fma(-dt, zm[r], zj[r]);
        }
        double p = 0.0;
        for (int64_t r = tid; r < n; r += 256) p = fma(zj[r], zj[r], p);
        const double inv = 1.0 / sqrt(block_sum(p));
        for (int64_t r = tid; r < n; r += 256) zj[r] *= inv;
    }
}

// row-major X (n x nev) -> column-major Z (ldz)
__global__ __launch_bounds__(256) void k_td_out(int64_t n, int64_t nev,
                                                const double* __restrict__ X,
                                                double* __restrict__ Z, int64_t ldz)
{
    __shared__ double tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int q = ty; q < 32; q += 8) {
        const int64_t r = r0 + q, c = c0 + tx;
        if (r < n && c < nev) tile[q][tx] = X[r * nev + c];
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t c = c0 + q, r = r0 + tx;
        if (r < n && c < nev) Z[c * ldz + r] = tile[tx][q];
    }
}

struct TdLayout {
    size_t e2 = 0, bounds = 0, x = 0, f = 0, p = 0, total = 0;
};

size_t tdal(size_t v) { return (v + 255) / 256 * 256; }

TdLayout td_layout(int64_t n, int64_t nev)
{
    TdLayout L;
    size_t off = 0;
    L.e2 = off;
    off = tdal(off + (size_t)(n > 1 ? n - 1 : 1) * 8);
    L.bounds = off;
    off = tdal(off + 4 * 8);
    L.x = off;
    off = tdal(off + (size_t)n * nev * 8);
    L.f = off;
    off = tdal(off + (size_t)n * nev * 4 * 8);
    L.p = off;
    off = tdal(off + (size_t)n * nev);
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

int trbt_tridiag_eigh_workspace_bytes(int64_t n, int64_t nev, size_t* bytes)
{
    if (n < 0) return -1;
    if (nev < 0 || nev > n) return -2;
    if (!bytes) return -3;
    *bytes = (n > 0 && nev > 0) ? td_layout(n, nev).total : 0;
    return TRBT_SUCCESS;
}

int trbt_tridiag_eigh_d(int64_t n, int64_t nev, const double* d, const double* e, double* w,
                        double* Z, int64_t ldz, void* work, size_t work_bytes, void* stream)
{
    if (n < 0) return -1;
    if (nev < 0 || nev > n) return -2;
    if (nev > 0 && !d) return -3;
    if (nev > 0 && n > 1 && !e) return -4;
    if (nev > 0 && !w) return -5;
    if (nev > 0 && !Z) return -6;
    if (ldz < (n > 1 ? n : 1)) return -7;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -8;
    if (nev == 0) return TRBT_SUCCESS;
    const TdLayout L = td_layout(n, nev);
    if (!work || work_bytes < L.total) return TRBT_ERR_WORKSPACE;
    int rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)work;
    double* e2 = (double*)(ws + L.e2);
    double* bounds = (double*)(ws + L.bounds);
    double* X = (double*)(ws + L.x);
    double* F = (double*)(ws + L.f);
    unsigned char* P = (unsigned char*)(ws + L.p);
    const unsigned nb = (unsigned)((nev + TD_THREADS - 1) / TD_THREADS);
    const unsigned nbm = (unsigned)((nev * TD_MS + TD_THREADS - 1) / TD_THREADS);
    hipLaunchKernelGGL(k_td_prep, dim3(1), dim3(256), 0, st, n, d, e, e2, bounds);
    hipLaunchKernelGGL(k_td_bisect, dim3(nbm), dim3(TD_THREADS), 0, st, n, nev, d,
                       (const double*)e2, (const double*)bounds, w);
    hipLaunchKernelGGL(k_td_invit, dim3(nb), dim3(TD_THREADS), 0, st, n, nev, d, e,
                       (const double*)bounds, (const double*)w, X, F, P);
    hipLaunchKernelGGL(k_td_out, dim3((unsigned)((n + 31) / 32), (unsigned)((nev + 31) / 32)),
                       dim3(256), 0, st, n, nev, (const double*)X, Z, ldz);
    hipLaunchKernelGGL(k_td_ortho, dim3((unsigned)nev), dim3(256), 0, st, n, nev,
                       (const double*)w, (const double*)bounds, Z, ldz);
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

}  // extern "C"
