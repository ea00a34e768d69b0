// trbt_batched.hip -- batched back-transformation of many independent
// eigenproblems of uneven size (k-points, spin channels), all real or all
// complex Hermitian, in one persistent, graph-captured launch per band width.
//
// The operation per problem is the single-problem one (Yu et al., CPC 2020,
// Sec. 2.2.2, Eq. 2stage_bkwd1): columns are independent and the reflector
// DAG lives inside one column strip, so the unit of work is a
// (problem, column strip) task that one workgroup runs start to finish with
// the same per-strip body as the single-problem kernel.
//
// Plan creation lays out, once, in one device allocation:
//   header      per-launch state: the fault word and one task counter per
//               XCD queue of every group (cleared by a fill kernel at the
//               start of every execution; no memset nodes in the graph);
//   packed      the compact-WY blocks of every problem (written by the
//               batched pack kernel at every execution, so hh_v / hh_tau may
//               change between executions);
//   tables      per group: problem descriptors, the task list and the
//               queue boundaries.
// Problems are grouped by form and band width (one template instance per
// group).  Blocked groups run a persistent kernel: every workgroup pulls
// tasks from the queue of its home XCD (blockIdx % 8; workgroups are
// dealt to the 8 XCDs round robin) and steals from the others once that
// queue is empty.  Problems are dealt to XCD queues largest first onto the
// least-loaded queue, so the strips of one problem, which stream the same
// packed operands, share one L2; inside a queue tasks run largest first.
// The launch sequence is captured once into a hipGraph and replayed by
// trbt_plan_exec.
//
// Tuning: without a fixed configuration, plan creation times every
// candidate (strip width 16 or 32 columns (complex: 16), 4 or 8 waves per
// workgroup, 16-stage compact-WY blocks; one reflector at a time as well
// when no problem can take the blocked form or all have n <= 256) on scratch
// copies of the problems' Z and keeps the fastest.  With the environment
// variable TRBT_TUNE_CACHE naming a file, the result is kept there, keyed by
// a signature of the problem set (device architecture and CU count, real or
// complex, and the sorted (n, nbw, nev) of every problem), and a later plan
// of the same signature takes it without timing anything.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <new>
#include <tuple>
#include <vector>

#include "trbt.h"
#include "trbt_device.h"

namespace {

constexpr int NXCD = 8;             // XCDs of MI355X (locality only)
constexpr int QSTRIDE = 16;         // ints between two queue counters (64 B)
constexpr int MAX_GROUPS = 5;       // nbw 16, 32, 48, 64 blocked + streaming
constexpr size_t HDR = 256 + MAX_GROUPS * NXCD * QSTRIDE * sizeof(int);

struct BProb {   // complex problems: interleaved (re, im) doubles
    int64_t n, nev, ldz;
    const double* hv;
    const double* ht;
    double* Z;
    double* ws;       // packed blocks (blocked groups)
    int64_t first;    // first pack block (blocked) / first workgroup (streaming)
    int64_t nbw;
};

struct BTask {
    int prob, strip;
};

__device__ inline int find_problem(const BProb* __restrict__ probs, int nprob, int64_t b)
{
    int lo = 0, hi = nprob;   // largest p with probs[p].first <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (probs[mid].first <= b) lo = mid; else hi = mid;
    }
    return lo;
}

template <int NB, bool CPLX>
__global__ __launch_bounds__(256) void k_pack_batched(const BProb* __restrict__ probs, int nprob)
{
    __shared__ int s_p;
    if (threadIdx.x == 0) s_p = find_problem(probs, nprob, blockIdx.x);
    __syncthreads();
    const BProb& P = probs[s_p];
    pack_block<NB, CPLX, rotating_window<NB, CPLX>()>(P.n, P.hv, P.ht, P.ws,
                                                      (int64_t)blockIdx.x - P.first);
}

// Persistent blocked kernel: one (problem, strip) task at a time per
// workgroup until every queue is empty.
template <int NB, int CT, int NW, bool CPLX>
__global__ __launch_bounds__(64 * NW) void k_blocked_batched(const BProb* __restrict__ probs,
                                                             const BTask* __restrict__ tasks,
                                                             const int* __restrict__ qbegin,
                                                             int* __restrict__ qnext,
                                                             unsigned* __restrict__ err)
{
    constexpr int D = ring_depth<NB, CPLX, CT>();
    __shared__ StripLds<NB, CT, CPLX, NW> S;
    __shared__ int s_task;
    const int home = blockIdx.x % NXCD;
    for (;;) {
        if (threadIdx.x == 0) {
            int task = -1;
            for (int k = 0; k < NXCD && task < 0; ++k) {
                const int x = (home + k) % NXCD;
                const int cnt = qbegin[x + 1] - qbegin[x];
                // a drained queue stays drained: skip it without an atomic
                if (__hip_atomic_load(&qnext[QSTRIDE * x], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT) >= cnt)
                    continue;
                const int i = atomicAdd(&qnext[QSTRIDE * x], 1);
                if (i < cnt) task = qbegin[x] + i;
            }
            s_task = task;
        }
        S.reset();
        __syncthreads();
        const int task = s_task;
        if (task < 0) return;
        const BTask tk = tasks[task];
        const BProb& P = probs[tk.prob];
        blocked_strip<NB, CT, CPLX, D, NW, false, rotating_window<NB, CPLX>()>(
            P.n, P.nev, P.ws, P.Z, P.ldz, err, tk.strip, S);
        __syncthreads();
    }
}

// Streaming form: one lane per column, problems back to back in the grid.
template <typename T>
__global__ __launch_bounds__(64) void k_unblocked_batched(const BProb* __restrict__ probs,
                                                          int nprob)
{
    const BProb& P = probs[find_problem(probs, nprob, blockIdx.x)];
    const int64_t col = ((int64_t)blockIdx.x - P.first) * 64 + threadIdx.x;
    if (col >= P.nev) return;
    unblocked_column<T>(P.n, (int)P.nbw, (const T*)P.hv, (const T*)P.ht,
                        (T*)P.Z + col * P.ldz);
}

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Group {
    bool blocked = false;
    int nbw = 0;                 // template band width (blocked groups)
    std::vector<int> members;    // problem indices, in table order
    // device table offsets (bytes into the plan allocation) and sizes
    size_t off_probs = 0, off_tasks = 0, off_qbegin = 0;
    int ntasks = 0;
    int64_t grid = 0;            // pack blocks (blocked) / streaming workgroups
    int64_t apply_grid = 0;
};

bool valid_config(const trbt_plan_config& c, bool cplx)
{
    return (c.strip_cols == 16 || (c.strip_cols == 32 && !cplx)) &&
           (c.waves == 4 || c.waves == 8) && (c.block_stages == 16 || c.block_stages == 1);
}

}  // namespace

struct trbt_plan {
    int device = 0;
    int cus = 0;
    bool cplx = false;                 // all problems complex (else all real)
    std::vector<trbt_problem_d> probs; // complex: pointers to interleaved doubles
    std::vector<size_t> ws_off;   // packed-block offset of each problem (or 0)
    size_t ws_bytes = 0;          // total packed-block bytes
    size_t table_off = 0;         // start of the tables region
    char* dmem = nullptr;
    size_t dbytes = 0;
    trbt_plan_config cfg{16, 8, 16};
    double tuned_ms = 0.0;
    std::vector<Group> groups;
    hipStream_t priv = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int64_t problem_cost(const trbt_problem_d& p, bool cplx)
{   // MFMA work of one strip ~ number of packed blocks; streaming ~ L
    return use_blocked(p.n, p.nbw, cplx) ? blocked_num_blocks(p.n, p.nbw)
                                         : num_reflectors(p.n, p.nbw) * p.nbw / 16;
}

template <int NB, int CT, int NW, bool CPLX>
int occupancy_grid(int cus, int64_t ntasks, int64_t* grid)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void*)k_blocked_batched<NB, CT, NW, CPLX>, 64 * NW, 0) !=
        hipSuccess)
        return TRBT_ERR_HIP;
    if (per_cu < 1) per_cu = 1;
    const int64_t slots = (int64_t)per_cu * cus;
    *grid = std::max<int64_t>(1, std::min<int64_t>(slots, ntasks));
    return TRBT_SUCCESS;
}

template <int NB, int CT, int NW, bool CPLX>
void launch_blocked(const Group& g, char* dmem, unsigned* err, int* qnext, hipStream_t st)
{
    hipLaunchKernelGGL((k_blocked_batched<NB, CT, NW, CPLX>), dim3((unsigned)g.apply_grid),
                       dim3(64 * NW), 0, st, (const BProb*)(dmem + g.off_probs),
                       (const BTask*)(dmem + g.off_tasks), (const int*)(dmem + g.off_qbegin),
                       qnext, err);
}

template <int NB>
int dispatch_blocked(const trbt_plan& P, const Group& g, unsigned* err, int* qnext,
                     hipStream_t st, bool grid_only, int64_t* grid)
{
    const int CT = P.cfg.strip_cols / 16, NW = P.cfg.waves;
    if (P.cplx) {   // complex: one 16-column tile per wave
        if (grid_only)
            return NW == 4 ? occupancy_grid<NB, 1, 4, true>(P.cus, g.ntasks, grid)
                           : occupancy_grid<NB, 1, 8, true>(P.cus, g.ntasks, grid);
        hipLaunchKernelGGL((k_pack_batched<NB, true>), dim3((unsigned)g.grid), dim3(256), 0, st,
                           (const BProb*)(P.dmem + g.off_probs), (int)g.members.size());
        if (NW == 4) launch_blocked<NB, 1, 4, true>(g, P.dmem, err, qnext, st);
        else launch_blocked<NB, 1, 8, true>(g, P.dmem, err, qnext, st);
        return TRBT_SUCCESS;
    }
    if (grid_only) {
        if (CT == 1 && NW == 4) return occupancy_grid<NB, 1, 4, false>(P.cus, g.ntasks, grid);
        if (CT == 1 && NW == 8) return occupancy_grid<NB, 1, 8, false>(P.cus, g.ntasks, grid);
        if (CT == 2 && NW == 4) return occupancy_grid<NB, 2, 4, false>(P.cus, g.ntasks, grid);
        return occupancy_grid<NB, 2, 8, false>(P.cus, g.ntasks, grid);
    }
    hipLaunchKernelGGL((k_pack_batched<NB, false>), dim3((unsigned)g.grid), dim3(256), 0, st,
                       (const BProb*)(P.dmem + g.off_probs), (int)g.members.size());
    if (CT == 1 && NW == 4) launch_blocked<NB, 1, 4, false>(g, P.dmem, err, qnext, st);
    else if (CT == 1 && NW == 8) launch_blocked<NB, 1, 8, false>(g, P.dmem, err, qnext, st);
    else if (CT == 2 && NW == 4) launch_blocked<NB, 2, 4, false>(g, P.dmem, err, qnext, st);
    else launch_blocked<NB, 2, 8, false>(g, P.dmem, err, qnext, st);
    return TRBT_SUCCESS;
}

int dispatch_group(const trbt_plan& P, const Group& g, int gi, hipStream_t st, bool grid_only,
                   int64_t* grid)
{
    unsigned* err = (unsigned*)P.dmem;
    int* qnext = (int*)(P.dmem + 256) + gi * NXCD * QSTRIDE;
    if (!g.blocked) {
        if (!grid_only) {
            if (P.cplx)
                hipLaunchKernelGGL(k_unblocked_batched<cd>, dim3((unsigned)g.grid), dim3(64), 0,
                                   st, (const BProb*)(P.dmem + g.off_probs),
                                   (int)g.members.size());
            else
                hipLaunchKernelGGL(k_unblocked_batched<double>, dim3((unsigned)g.grid),
                                   dim3(64), 0, st, (const BProb*)(P.dmem + g.off_probs),
                                   (int)g.members.size());
        }
        return TRBT_SUCCESS;
    }
    switch (g.nbw) {
        case 16: return dispatch_blocked<16>(P, g, err, qnext, st, grid_only, grid);
        case 32: return dispatch_blocked<32>(P, g, err, qnext, st, grid_only, grid);
        case 48: return dispatch_blocked<48>(P, g, err, qnext, st, grid_only, grid);
        case 64: return dispatch_blocked<64>(P, g, err, qnext, st, grid_only, grid);
        default: return TRBT_ERR_INTERNAL;
    }
}

// Group the active problems, build the device tables for P.cfg with the
// given Z pointers (the caller's, or scratch copies while tuning), and
// upload them.
int build_tables(trbt_plan& P, const std::vector<double*>& zptr)
{
    const int count = (int)P.probs.size();
    P.groups.clear();
    const bool stream_all = P.cfg.block_stages == 1;
    const int nbws[4] = {16, 32, 48, 64};
    for (int gi = 0; gi < 5; ++gi) {
        Group g;
        g.blocked = gi < 4 && !stream_all;
        g.nbw = gi < 4 ? nbws[gi] : 0;
        for (int i = 0; i < count; ++i) {
            const trbt_problem_d& p = P.probs[i];
            if (num_reflectors(p.n, p.nbw) == 0 || p.nev == 0) continue;
            const bool elig = use_blocked(p.n, p.nbw, P.cplx) && !stream_all;
            if (g.blocked ? (elig && p.nbw == g.nbw) : (gi == 4 && !elig)) g.members.push_back(i);
        }
        if (!g.members.empty()) P.groups.push_back(g);
    }

    std::vector<char> host;
    size_t off = 0;
    auto reserve = [&](size_t bytes) {
        off = align_up(off, 256);
        const size_t at = off;
        off += bytes;
        return at;
    };
    for (size_t gi = 0; gi < P.groups.size(); ++gi) {
        Group& g = P.groups[gi];
        // largest problems first: their strips start first
        std::stable_sort(g.members.begin(), g.members.end(), [&](int a, int b) {
            return problem_cost(P.probs[a], P.cplx) > problem_cost(P.probs[b], P.cplx);
        });
        const int np = (int)g.members.size();
        std::vector<BProb> bp(np);
        int64_t first = 0;
        for (int m = 0; m < np; ++m) {
            const int i = g.members[m];
            const trbt_problem_d& p = P.probs[i];
            bp[m].n = p.n;
            bp[m].nev = p.nev;
            bp[m].ldz = p.ldz;
            bp[m].hv = p.hh_v;
            bp[m].ht = p.hh_tau;
            bp[m].Z = zptr[i];
            bp[m].ws = (double*)(P.dmem + P.ws_off[i]);
            bp[m].nbw = p.nbw;
            bp[m].first = first;
            first += g.blocked ? blocked_num_blocks(p.n, p.nbw) : (p.nev + 63) / 64;
        }
        g.grid = first;
        std::vector<BTask> tasks;
        std::vector<int> qbegin(NXCD + 1, 0);
        if (g.blocked) {
            const int cols = P.cfg.strip_cols;
            // deal problems to XCD queues: largest total work onto the
            // least-loaded queue (members are already sorted by strip cost)
            std::vector<int> order(np);
            for (int m = 0; m < np; ++m) order[m] = m;
            auto total = [&](int m) {
                const trbt_problem_d& p = P.probs[g.members[m]];
                return problem_cost(p, P.cplx) * ((p.nev + cols - 1) / cols);
            };
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return total(a) > total(b); });
            std::vector<int64_t> load(NXCD, 0);
            std::vector<std::vector<int>> q(NXCD);
            for (int m : order) {
                const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                load[x] += total(m);
                q[x].push_back(m);
            }
            for (int x = 0; x < NXCD; ++x) {
                qbegin[x] = (int)tasks.size();
                std::stable_sort(q[x].begin(), q[x].end(), [&](int a, int b) {
                    return problem_cost(P.probs[g.members[a]], P.cplx) >
                           problem_cost(P.probs[g.members[b]], P.cplx);
                });
                for (int m : q[x]) {
                    const int64_t strips = (P.probs[g.members[m]].nev + cols - 1) / cols;
                    for (int64_t s = 0; s < strips; ++s) tasks.push_back({m, (int)s});
                }
            }
            qbegin[NXCD] = (int)tasks.size();
        }
        g.ntasks = (int)tasks.size();
        g.off_probs = reserve(bp.size() * sizeof(BProb));
        g.off_tasks = reserve(tasks.size() * sizeof(BTask));
        g.off_qbegin = reserve(qbegin.size() * sizeof(int));
        host.resize(off);
        memcpy(host.data() + g.off_probs, bp.data(), bp.size() * sizeof(BProb));
        if (!tasks.empty())
            memcpy(host.data() + g.off_tasks, tasks.data(), tasks.size() * sizeof(BTask));
        memcpy(host.data() + g.off_qbegin, qbegin.data(), qbegin.size() * sizeof(int));
        g.off_probs += P.table_off;
        g.off_tasks += P.table_off;
        g.off_qbegin += P.table_off;
        if (g.blocked) {
            const int rc = dispatch_group(P, g, (int)gi, nullptr, true, &g.apply_grid);
            if (rc) return rc;
        }
    }
    if (P.table_off + host.size() > P.dbytes) return TRBT_ERR_INTERNAL;
    if (!host.empty() &&
        hipMemcpy(P.dmem + P.table_off, host.data(), host.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
        return TRBT_ERR_HIP;
    return TRBT_SUCCESS;
}

// Capture: clear the header, then per group the pack and apply kernels.
int capture(trbt_plan& P)
{
    if (P.exec) (void)hipGraphExecDestroy(P.exec);
    if (P.graph) (void)hipGraphDestroy(P.graph);
    P.exec = nullptr;
    P.graph = nullptr;
    if (P.groups.empty()) return TRBT_SUCCESS;
    if (hipStreamBeginCapture(P.priv, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return TRBT_ERR_HIP;
    const int words = (int)(HDR / sizeof(unsigned));
    hipLaunchKernelGGL(k_zero_words, dim3((words + 255) / 256), dim3(256), 0, P.priv,
                       (unsigned*)P.dmem, words);
    int rc = TRBT_SUCCESS;
    for (size_t gi = 0; gi < P.groups.size() && !rc; ++gi)
        rc = dispatch_group(P, P.groups[gi], (int)gi, P.priv, false, nullptr);
    const hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(P.priv, &graph);
    if (rc || le != hipSuccess || ce != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc ? rc : TRBT_ERR_HIP;
    }
    P.graph = graph;
    if (hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0) != hipSuccess) {
        P.exec = nullptr;
        return TRBT_ERR_HIP;
    }
    return TRBT_SUCCESS;
}

int time_exec(trbt_plan& P, double best_ms, double* ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return TRBT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TRBT_ERR_HIP;
    }
    int rc = TRBT_SUCCESS;
    double best = 1e300;
    for (int rep = 0; rep < 3 && !rc; ++rep) {   // rep 0 warms up
        float t = 0.f;
        if (hipEventRecord(e0, P.priv) != hipSuccess ||
            (P.exec && hipGraphLaunch(P.exec, P.priv) != hipSuccess) ||
            hipEventRecord(e1, P.priv) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            rc = TRBT_ERR_HIP;
            break;
        }
        if (rep > 0) best = std::min(best, (double)t);
        if (rep == 0 && t > 3.0 * best_ms) {   // far off the best so far: stop early
            best = t;
            break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return rc;
}

void release(trbt_plan* P)
{
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->priv) (void)hipStreamDestroy(P->priv);
    if (P->dmem) (void)hipFree(P->dmem);
    delete P;
}

int tune_by_timing(trbt_plan& P);

// --------------------------------------------------------------------------
// Tuning cache (TRBT_TUNE_CACHE): one text line per tuned problem set,
//   trbt-tune-v1 <signature> <strip_cols> <waves> <block_stages> <best ms>
// appended after tuning; the last line of a signature wins.
// --------------------------------------------------------------------------
uint64_t plan_signature(const trbt_plan& P)
{
    hipDeviceProp_t prop;
    const char* arch = "unknown";
    if (hipGetDeviceProperties(&prop, P.device) == hipSuccess) arch = prop.gcnArchName;
    std::vector<std::tuple<int64_t, int, int64_t>> shapes;
    for (const trbt_problem_d& p : P.probs) shapes.emplace_back(p.n, p.nbw, p.nev);
    std::sort(shapes.begin(), shapes.end());
    uint64_t h = 1469598103934665603ull;   // FNV-1a, 64 bit
    auto mix = [&h](const void* data, size_t len) {
        const unsigned char* c = (const unsigned char*)data;
        for (size_t i = 0; i < len; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    mix(arch, strlen(arch));
    mix(&P.cus, sizeof P.cus);
    const int cp = P.cplx ? 1 : 0;
    mix(&cp, sizeof cp);
    for (const auto& t : shapes) {
        const int64_t a = std::get<0>(t), c = std::get<2>(t);
        const int b = std::get<1>(t);
        mix(&a, sizeof a);
        mix(&b, sizeof b);
        mix(&c, sizeof c);
    }
    return h;
}

bool cache_lookup(const char* path, uint64_t sig, bool cplx, trbt_plan_config* cfg, double* ms)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        unsigned long long s = 0;
        trbt_plan_config c{};
        double t = 0.0;
        if (sscanf(line, "trbt-tune-v1 %llx %d %d %d %lf", &s, &c.strip_cols, &c.waves,
                   &c.block_stages, &t) == 5 &&
            s == sig && valid_config(c, cplx)) {
            *cfg = c;
            *ms = t;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char* path, uint64_t sig, const trbt_plan_config& c, double ms)
{
    FILE* f = fopen(path, "a");
    if (!f) return;   // an unwritable cache only costs the next plan its tuning
    fprintf(f, "trbt-tune-v1 %016llx %d %d %d %.6f\n", (unsigned long long)sig, c.strip_cols,
            c.waves, c.block_stages, ms);
    fclose(f);
}

int tune(trbt_plan& P)
{
    const char* cache = getenv("TRBT_TUNE_CACHE");
    const uint64_t sig = (cache && *cache) ? plan_signature(P) : 0;
    if (cache && *cache) {
        trbt_plan_config c;
        double ms = 0.0;
        if (cache_lookup(cache, sig, P.cplx, &c, &ms)) {
            P.cfg = c;
            P.tuned_ms = ms;
            return TRBT_SUCCESS;
        }
    }
    const int rc = tune_by_timing(P);
    if (!rc && cache && *cache) cache_store(cache, sig, P.cfg, P.tuned_ms);
    return rc;
}

int tune_by_timing(trbt_plan& P)
{
    // scratch copies of every Z, so that timing leaves the caller's data alone
    // (the last column is copied only up to row n: the caller's buffer may
    // end there)
    std::vector<size_t> zoff(P.probs.size(), 0), zlen(P.probs.size(), 0);
    size_t zbytes = 0;
    for (size_t i = 0; i < P.probs.size(); ++i) {
        const trbt_problem_d& p = P.probs[i];
        zoff[i] = zbytes;
        if (p.nev > 0 && p.n > 0)
            zlen[i] = ((size_t)(p.nev - 1) * p.ldz + p.n) * sizeof(double) * (P.cplx ? 2 : 1);
        zbytes = align_up(zbytes + zlen[i], 256);
    }
    char* scratch = nullptr;
    if (zbytes && hipMalloc(&scratch, zbytes) != hipSuccess) return TRBT_ERR_HIP;
    std::vector<double*> zs(P.probs.size(), nullptr);
    int rc = TRBT_SUCCESS;
    for (size_t i = 0; i < P.probs.size() && !rc; ++i) {
        const trbt_problem_d& p = P.probs[i];
        if (p.nev > 0 && p.n > 0) {
            zs[i] = (double*)(scratch + zoff[i]);
            if (hipMemcpyAsync(zs[i], p.Z, zlen[i], hipMemcpyDeviceToDevice, P.priv) !=
                hipSuccess)
                rc = TRBT_ERR_HIP;
        }
    }
    bool any_blocked = false;
    int64_t max_n = 0;
    for (const trbt_problem_d& p : P.probs) {
        const bool active = num_reflectors(p.n, p.nbw) > 0 && p.nev > 0;
        any_blocked |= active && use_blocked(p.n, p.nbw, P.cplx);
        if (active) max_n = std::max(max_n, p.n);
    }
    std::vector<trbt_plan_config> cands;
    if (any_blocked) {
        for (int cols : {16, 32})
            for (int waves : {8, 4})
                if (cols == 16 || !P.cplx) cands.push_back({cols, waves, 16});
    }
    // The streaming form (one lane per column, a dependent chain of K
    // reflectors per lane) only competes on tiny problems; beyond that a
    // single timing of it costs more than the whole plan's other candidates.
    if (!any_blocked || max_n <= 256) cands.push_back({16, 8, 1});
    trbt_plan_config best{16, 8, 16};
    double best_ms = 1e300;
    for (const trbt_plan_config& c : cands) {
        if (rc) break;
        P.cfg = c;
        rc = build_tables(P, zs);
        if (!rc) rc = capture(P);
        double ms = 0.0;
        if (!rc) rc = time_exec(P, best_ms, &ms);
        if (!rc && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    if (hipStreamSynchronize(P.priv) != hipSuccess && !rc) rc = TRBT_ERR_HIP;
    if (scratch) (void)hipFree(scratch);
    P.cfg = best;
    P.tuned_ms = best_ms < 1e300 ? best_ms : 0.0;
    return rc;
}

// Plan creation for real (cplx = false) or complex problems, given as
// real-typed descriptors (complex pointers reinterpreted as interleaved
// doubles).
int create_plan(const trbt_problem_d* probs, int count, bool cplx,
                const trbt_plan_config* cfg, trbt_plan** plan, void* stream)
{
    if (count < 0 || (count > 0 && !probs)) return count < 0 ? -2 : -1;
    if (cfg && !valid_config(*cfg, cplx)) return -3;
    if (!plan) return -4;
    *plan = nullptr;
    for (int i = 0; i < count; ++i) {
        const trbt_problem_d& p = probs[i];
        if (validate(p.n, p.nbw, p.nev, p.hh_v, p.hh_tau, p.Z, p.ldz, nullptr, 0))
            return TRBT_ERR_PROBLEM(i);
    }
    int rc = check_device();
    if (rc) return rc;

    trbt_plan* P = new (std::nothrow) trbt_plan;
    if (!P) return TRBT_ERR_HIP;
    P->cplx = cplx;
    P->probs.assign(probs, probs + count);
    hipDeviceProp_t prop;
    if (hipGetDevice(&P->device) != hipSuccess ||
        hipGetDeviceProperties(&prop, P->device) != hipSuccess) {
        release(P);
        return TRBT_ERR_HIP;
    }
    P->cus = prop.multiProcessorCount;

    // device allocation: header, packed blocks, tables (sized for the
    // largest task list: 16-column strips)
    P->ws_off.assign(count, 0);
    size_t off = HDR;
    size_t tables = 0;
    for (int i = 0; i < count; ++i) {
        const trbt_problem_d& p = probs[i];
        const bool active = num_reflectors(p.n, p.nbw) > 0 && p.nev > 0;
        if (active && use_blocked(p.n, p.nbw, cplx)) {
            off = align_up(off, 256);
            P->ws_off[i] = off;
            off += blocked_bytes(p.n, p.nbw, cplx) - HDR_BYTES;
        }
        tables += sizeof(BProb) + sizeof(BTask) * (size_t)((p.nev + 15) / 16);
    }
    P->table_off = align_up(off, 256);
    P->dbytes = P->table_off + tables + MAX_GROUPS * (3 * 256 + (NXCD + 1) * sizeof(int));
    if (hipMalloc(&P->dmem, P->dbytes) != hipSuccess) {
        P->dmem = nullptr;
        release(P);
        return TRBT_ERR_HIP;
    }
    if (hipStreamCreateWithFlags(&P->priv, hipStreamNonBlocking) != hipSuccess) {
        P->priv = nullptr;
        release(P);
        return TRBT_ERR_HIP;
    }
    // the caller's stream may still be producing Z and the reflectors
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
        release(P);
        return TRBT_ERR_HIP;
    }
    if (cfg) {
        P->cfg = *cfg;
    } else {
        rc = tune(*P);
        if (rc) {
            release(P);
            return rc;
        }
    }
    std::vector<double*> zs(count);
    for (int i = 0; i < count; ++i) zs[i] = probs[i].Z;
    rc = build_tables(*P, zs);
    if (!rc) rc = capture(*P);
    if (rc) {
        release(P);
        return rc;
    }
    *plan = P;
    return TRBT_SUCCESS;
}

}  // namespace

extern "C" {

int trbt_plan_create_batched_d(const trbt_problem_d* probs, int count,
                               const trbt_plan_config* cfg, trbt_plan** plan, void* stream)
{
    return create_plan(probs, count, false, cfg, plan, stream);
}

int trbt_plan_create_batched_z(const trbt_problem_z* probs, int count,
                               const trbt_plan_config* cfg, trbt_plan** plan, void* stream)
{
    if (count < 0 || (count > 0 && !probs)) return count < 0 ? -2 : -1;
    std::vector<trbt_problem_d> d(count > 0 ? count : 0);
    for (int i = 0; i < count; ++i) {
        const trbt_problem_z& p = probs[i];
        d[i] = trbt_problem_d{p.n, p.nbw, p.nev, (const double*)p.hh_v, (const double*)p.hh_tau,
                              (double*)p.Z, p.ldz};
    }
    return create_plan(d.data(), count, true, cfg, plan, stream);
}

int trbt_plan_exec(trbt_plan* plan, void* stream)
{
    if (!plan) return -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TRBT_ERR_HIP;
    if (dev != plan->device) return TRBT_ERR_DEVICE;
    if (!plan->exec) return TRBT_SUCCESS;
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? TRBT_SUCCESS
                                                                         : TRBT_ERR_HIP;
}

int trbt_plan_get_config(const trbt_plan* plan, trbt_plan_config* cfg, double* tuned_ms)
{
    if (!plan) return -1;
    if (cfg) *cfg = plan->cfg;
    if (tuned_ms) *tuned_ms = plan->tuned_ms;
    return TRBT_SUCCESS;
}

int trbt_plan_check(trbt_plan* plan, int* fault)
{
    if (!plan) return -1;
    if (!fault) return -2;
    unsigned word = 0;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&word, plan->dmem, sizeof(word), hipMemcpyDeviceToHost) != hipSuccess)
        return TRBT_ERR_HIP;
    *fault = (int)word;
    return TRBT_SUCCESS;
}

int trbt_plan_destroy(trbt_plan* plan)
{
    if (!plan) return TRBT_SUCCESS;
    if (hipDeviceSynchronize() != hipSuccess) {
        release(plan);
        return TRBT_ERR_HIP;
    }
    release(plan);
    return TRBT_SUCCESS;
}

}  // extern "C"
