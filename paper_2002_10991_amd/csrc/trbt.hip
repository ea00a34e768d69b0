// trbt.hip -- single-problem entry points of the tridiagonal-to-banded
// eigenvector back-transformation for AMD Instinct MI355X (gfx950): the
// host side of trans_ev_tridi_to_band_{d,z}, trbt_prepare_* and trbt_apply_*.
// The kernels and the ordering argument are in trbt_device.h.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include "trbt.h"
#include "trbt_device.h"

namespace {

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------

// Slot groups: when a problem has fewer column strips than the device has
// CUs, G workgroups share each strip (at most GMAX), with G progress
// counters per strip in the workspace after the packed blocks (room for
// 16-column strips, the narrowest, plus 8 strips of padding).
constexpr int GMAX = 8;

inline size_t group_counter_bytes(int64_t nev)
{
    return ((size_t)((nev + 15) / 16 + 8) * GMAX * sizeof(int) + 255) / 256 * 256;
}

// Workspace of the single-problem forward: packed blocks + group counters.
inline size_t apply_bytes(int64_t n, int nbw, int64_t nev, bool cplx)
{
    return blocked_bytes(n, nbw, cplx) + group_counter_bytes(nev);
}

// CUs of the current device (looked up once per device id).
inline int device_cus()
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

// Launch the blocked forward kernel, with slot groups when the strips alone
// leave CUs idle and the grid fits on the device at once (a cooperative
// launch guarantees the workgroups of a strip run concurrently); otherwise
// one workgroup per strip.
template <int NB, int CT, bool CPLX, int D, int NW, bool ROT>
int launch_blocked(int64_t n, int64_t nev, const double* ws, double* Z, int64_t ldz,
                   unsigned* err, int* gprog, hipStream_t st)
{
    const int64_t strips = (nev + 16 * CT - 1) / (16 * CT);
    const int64_t rounds = (sweeps_in_stage(n, NB, 0) + NW - 1) / NW;
    const int cus = device_cus();
    int64_t G = 1;
    if (cus > 0 && strips < cus) {
        G = cus / strips;
        if (G > rounds) G = rounds;
        if (G > GMAX) G = GMAX;
    }
    if (G > 1) {
        auto kern = k_blocked<NB, CT, CPLX, D, NW, ROT, true>;
        const int64_t grid = (strips + 7) / 8 * 8 * G;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * NW, 0) ==
                hipSuccess &&
            (int64_t)per_cu * cus >= grid) {
            const int cnt = (int)(strips * G);
            hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
                               (unsigned*)gprog, cnt);
            int g32 = (int)G;
            void* args[] = {&n, &nev, &ws, &Z, &ldz, &err, &g32, &gprog};
            if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3((unsigned)grid),
                                           dim3(64 * NW), args, 0, st) == hipSuccess)
                return TRBT_SUCCESS;
        }
        (void)hipGetLastError();   // fall back to one workgroup per strip
    }
    hipLaunchKernelGGL((k_blocked<NB, CT, CPLX, D, NW, ROT, false>), dim3((unsigned)strips),
                       dim3(64 * NW), 0, st, n, nev, ws, Z, ldz, err, 1, (int*)nullptr);
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}
template <bool CPLX>
int prepare(int64_t n, int nbw, const double* hv, const double* ht, void* work,
            size_t work_bytes, void* stream_v)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    const int64_t K = num_reflectors(n, nbw);
    if (K > 0 && !hv) return -3;
    if (K > 0 && !ht) return -4;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -5;
    if (work_bytes && !work) return -5;
    if (K == 0 || !use_blocked_apply(n, nbw, CPLX)) return TRBT_SUCCESS;
    if (!work || work_bytes < blocked_bytes(n, nbw, CPLX)) return TRBT_ERR_WORKSPACE;
    int rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream_v;
    double* ws = (double*)work;
    const int64_t nblocks = blocked_num_blocks(n, nbw);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (unsigned*)work, 64);
#define TRBT_PACK(NBV)                                                                         \
    case NBV:                                                                                  \
        hipLaunchKernelGGL((k_pack<NBV, CPLX, rotating_window<NBV, CPLX>()>),                  \
                           dim3((unsigned)nblocks), dim3(256), 0, st, n, hv, ht,               \
                           ws + HDR_BYTES / sizeof(double));                                   \
        break;
    switch (nbw) {
        TRBT_PACK(16)
        TRBT_PACK(32)
        TRBT_PACK(48)
        TRBT_PACK(64)
        TRBT_PACK(80)
        TRBT_PACK(96)
        TRBT_PACK(112)
        TRBT_PACK(128)
        default: return TRBT_ERR_INTERNAL;
    }
#undef TRBT_PACK
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

template <bool CPLX>
int apply(int64_t n, int nbw, int64_t nev, const double* hv, const double* ht, double* Z,
          int64_t ldz, void* work, size_t work_bytes, void* stream_v)
{
    int rc = validate(n, nbw, nev, hv, ht, Z, ldz, work, work_bytes);
    if (rc) return rc;
    if (num_reflectors(n, nbw) == 0 || nev == 0) return TRBT_SUCCESS;
    rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream_v;

    if (use_blocked_apply(n, nbw, CPLX)) {
        if (work_bytes < apply_bytes(n, nbw, nev, CPLX) || !work) return TRBT_ERR_WORKSPACE;
        const double* ws = (const double*)work;
        unsigned* err = (unsigned*)work;
        int* gprog = (int*)((char*)work + blocked_bytes(n, nbw, CPLX));
        // nbw > 64: windows of 6..9 tiles need one wave per SIMD (4 waves,
        // all 512 registers) and a half-block operand ring; real nbw <= 64:
        // two column tiles per wave
#define TRBT_MAIN(NBV)                                                                         \
    case NBV: {                                                                                \
        constexpr bool ROT = rotating_window<NBV, CPLX>();                                     \
        constexpr int CTV = (!CPLX && NBV <= 64) ? 2 : 1;                                       \
        constexpr int NW = NBV <= 64 ? WAVES : 4;                                              \
        constexpr int D = (NBV <= 64 || CPLX) ? ring_depth<NBV, CPLX, CTV>()                   \
                                              : 4 * (NBV / 16 + 1);                            \
        return launch_blocked<NBV, CTV, CPLX, D, NW, ROT>(n, nev, ws, Z, ldz, err, gprog, st); \
    }
        switch (nbw) {
            TRBT_MAIN(16)
            TRBT_MAIN(32)
            TRBT_MAIN(48)
            TRBT_MAIN(64)
            TRBT_MAIN(80)
            TRBT_MAIN(96)
            TRBT_MAIN(112)
            TRBT_MAIN(128)
            default: return TRBT_ERR_INTERNAL;
        }
#undef TRBT_MAIN
    } else {
        // the streaming kernel has no waits: its fault word is always clear
        if (work && work_bytes >= sizeof(unsigned))
            hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (unsigned*)work, 1);
        const unsigned grid = (unsigned)((nev + 63) / 64);
        if (CPLX)
            hipLaunchKernelGGL((k_unblocked<cd>), dim3(grid), dim3(64), 0, st, n, nbw, nev,
                               (const cd*)hv, (const cd*)ht, (cd*)Z, ldz);
        else
            hipLaunchKernelGGL((k_unblocked<double>), dim3(grid), dim3(64), 0, st, n, nbw, nev,
                               hv, ht, Z, ldz);
    }
    return hipGetLastError() == hipSuccess ? TRBT_SUCCESS : TRBT_ERR_HIP;
}

template <bool CPLX>
int run(int64_t n, int nbw, int64_t nev, const double* hv, const double* ht, double* Z,
        int64_t ldz, void* work, size_t work_bytes, void* stream_v)
{
    int rc = validate(n, nbw, nev, hv, ht, Z, ldz, work, work_bytes);
    if (rc) return rc;
    if (num_reflectors(n, nbw) == 0 || nev == 0) return TRBT_SUCCESS;
    rc = prepare<CPLX>(n, nbw, hv, ht, work, work_bytes, stream_v);
    if (rc == -5) return -8;           // work argument position differs
    if (rc) return rc;
    return apply<CPLX>(n, nbw, nev, hv, ht, Z, ldz, work, work_bytes, stream_v);
}

}  // namespace

extern "C" {

int trbt_num_reflectors(int64_t n, int nbw, int64_t* K)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (!K) return -3;
    *K = num_reflectors(n, nbw);
    return TRBT_SUCCESS;
}

int trbt_stage_offsets(int64_t n, int nbw, int64_t* off)
{
    if (n < 2) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (!off) return -3;
    for (int64_t s = 0; s <= n - 2; ++s) off[s] = stage_offset(n, nbw, s);
    return TRBT_SUCCESS;
}

int trbt_workspace_bytes(int64_t n, int nbw, int64_t nev, int is_complex, size_t* bytes)
{
    if (n < 0) return -1;
    if (nbw < 1 || nbw > TRBT_NBW_MAX) return -2;
    if (nev < 0 || nev > n) return -3;
    if (!bytes) return -4;
    *bytes = (use_blocked_apply(n, nbw, is_complex != 0) && num_reflectors(n, nbw) > 0 && nev > 0)
                 ? apply_bytes(n, nbw, nev, is_complex != 0)
                 : 0;
    return TRBT_SUCCESS;
}

int trans_ev_tridi_to_band_d(int64_t n, int nbw, int64_t nev, const double* hh_v,
                             const double* hh_tau, double* Z, int64_t ldz, void* work,
                             size_t work_bytes, void* stream)
{
    return run<false>(n, nbw, nev, hh_v, hh_tau, Z, ldz, work, work_bytes, stream);
}

int trans_ev_tridi_to_band_z(int64_t n, int nbw, int64_t nev, const trbt_z* hh_v,
                             const trbt_z* hh_tau, trbt_z* Z, int64_t ldz, void* work,
                             size_t work_bytes, void* stream)
{
    return run<true>(n, nbw, nev, (const double*)hh_v, (const double*)hh_tau, (double*)Z, ldz,
                     work, work_bytes, stream);
}

int trbt_prepare_d(int64_t n, int nbw, const double* hh_v, const double* hh_tau, void* work,
                   size_t work_bytes, void* stream)
{
    return prepare<false>(n, nbw, hh_v, hh_tau, work, work_bytes, stream);
}

int trbt_prepare_z(int64_t n, int nbw, const trbt_z* hh_v, const trbt_z* hh_tau, void* work,
                   size_t work_bytes, void* stream)
{
    return prepare<true>(n, nbw, (const double*)hh_v, (const double*)hh_tau, work, work_bytes,
                         stream);
}

int trbt_apply_d(int64_t n, int nbw, int64_t nev, const double* hh_v, const double* hh_tau,
                 double* Z, int64_t ldz, void* work, size_t work_bytes, void* stream)
{
    return apply<false>(n, nbw, nev, hh_v, hh_tau, Z, ldz, work, work_bytes, stream);
}

int trbt_apply_z(int64_t n, int nbw, int64_t nev, const trbt_z* hh_v, const trbt_z* hh_tau,
                 trbt_z* Z, int64_t ldz, void* work, size_t work_bytes, void* stream)
{
    return apply<true>(n, nbw, nev, (const double*)hh_v, (const double*)hh_tau, (double*)Z, ldz,
                       work, work_bytes, stream);
}

int trbt_work_check(const void* work, int* fault, void* stream)
{
    if (!fault) return -2;
    *fault = 0;
    if (work && ((uintptr_t)work % TRBT_WORK_ALIGN)) return -1;
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamSynchronize(st) != hipSuccess) return TRBT_ERR_HIP;
    if (!work) return TRBT_SUCCESS;
    unsigned word = 0;
    if (hipMemcpy(&word, work, sizeof word, hipMemcpyDeviceToHost) != hipSuccess)
        return TRBT_ERR_HIP;
    *fault = word != 0u;
    return TRBT_SUCCESS;
}

const char* trbt_strerror(int status)
{
    switch (status) {
        case TRBT_SUCCESS: return "success";
        case TRBT_ERR_DEVICE: return "current device is not gfx950";
        case TRBT_ERR_WORKSPACE: return "workspace too small or missing";
        case TRBT_ERR_HIP: return "HIP runtime error";
        case TRBT_ERR_INTERNAL: return "internal error";
        case TRBT_ERR_SCRATCH: return "problem too large for the fixed scratch of an allocation-free entry point";
        default: break;
    }
    if (status < 0 && status > -20) return "invalid argument (see the argument position)";
    return "unknown status";
}

}  // extern "C"
