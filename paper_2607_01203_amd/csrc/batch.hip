// batch.hip -- many uneven bound problems in one graph launch.
//
// A batch mixes analytic (chain, any number of nodes) and ReLU-MLP
// problems, each one trajectory of its own horizon.  At creation the
// problems are grouped by launch shape:
//   analytic: by node count and dynamics constants; every group is one
//     launch of the path-based bound kernel over a table of tiles (a tile is
//     up to T consecutive steps of one problem, with that problem's pointers);
//   MLP: by network; the problems' inputs are gathered into batch-owned
//     staging arrays, bounded in chunks of CB boxes, and scattered back.
// T and CB are chosen by timing candidates on the batch's own data (the
// autotuner), with results cached in a text file keyed by GPU
// architecture and group shape.  The tiles of every analytic group then
// form one work queue, bounded by one persistent launch (workgroups take
// tiles from a device counter, largest tiles first); it and the MLP groups'
// launches are captured on two streams (the VALU-bound and MFMA-bound work
// overlap) into one hipGraph; a submit is one graph launch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "leb.h"
#include "leb_internal.hpp"

namespace leb {

struct NNProbPtrs {
    const double *z, *v, *mu, *sigma;
    double *r_lo, *r_hi;
    int64_t off;       // first staged unit
    int N;
    int pad_;
};

// one thread per (staged unit, input component)
__global__ void nn_gather_kernel(const NNProbPtrs* P, const int* unit_prob, int64_t units, int nx, int nu,
                                 double* zS, double* vS, double* muS, double* sgS) {
    const int n0 = nx + nu;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= units * n0) return;
    const int64_t u = q / n0;
    const int c = (int)(q - u * n0);
    const NNProbPtrs& p = P[unit_prob[u]];
    const int64_t k = u - p.off;
    if (c < nx) zS[u * nx + c] = p.z[k * nx + c];
    else vS[u * nu + (c - nx)] = p.v[k * nu + (c - nx)];
    sgS[q] = p.sigma[k * n0 + c];
    muS[q] = p.mu ? p.mu[k * n0 + c] : 0.0;
}

__global__ void nn_scatter_kernel(const NNProbPtrs* P, const int* unit_prob, int64_t units, int m, const double* loS,
                                  const double* hiS) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= units * m) return;
    const int64_t u = q / m;
    const int c = (int)(q - u * m);
    const NNProbPtrs& p = P[unit_prob[u]];
    const int64_t k = u - p.off;
    p.r_lo[k * m + c] = loS[q];
    p.r_hi[k * m + c] = hiS[q];
}

static unsigned nbk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace leb

using namespace leb;

struct PbhGroup {
    leb_dynamics dyn;
    std::vector<int> probs;
    int64_t units = 0;
    int T = 0;
    PbhTile* tiles = nullptr;   // device
    int n_tiles = 0;
    bool cached = false;
};

struct NNGroup {
    leb_mlp net = nullptr;
    int nx = 0, nu = 0, m = 0;
    std::vector<int> probs;
    int64_t units = 0;
    int CB = 0;
    NNProbPtrs* ptrs = nullptr;   // device
    int* unit_prob = nullptr;     // device [units]
    double *zS = nullptr, *vS = nullptr, *muS = nullptr, *sgS = nullptr, *loS = nullptr, *hiS = nullptr;
    double* buf[NN_NBUF] = {};
    bool cached = false;
};

struct leb_batch_s {
    std::vector<leb_problem> probs;
    std::vector<PbhGroup> pbh;
    std::vector<NNGroup> nn;
    std::vector<void*> allocs;
    hipStream_t s0 = nullptr, s1 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    PbhQueueArgs queue = {nullptr, 0, 0, nullptr};   // every analytic group's tiles in one persistent launch
    size_t queue_smem = 0;
    int queue_grid = 0;
    std::string info;
};

static void batch_free(leb_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void* p : b->allocs)
        if (p) (void)hipFree(p);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->s0) (void)hipStreamDestroy(b->s0);
    if (b->s1) (void)hipStreamDestroy(b->s1);
    delete b;
}

static int balloc(leb_batch_s* b, size_t bytes, void** out) {
    *out = nullptr;
    if (bytes == 0) bytes = 8;
    if (hipMalloc(out, bytes) != hipSuccess) { *out = nullptr; return LEB_ENOMEM; }
    b->allocs.push_back(*out);
    return LEB_OK;
}

// ------------------------------------------------------------ tune cache

static std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

static int64_t bucket(int64_t x) {    // next power of two
    int64_t b = 1;
    while (b < x) b <<= 1;
    return b;
}

static std::map<std::string, int> read_cache(const char* path) {
    std::map<std::string, int> m;
    if (!path) return m;
    FILE* f = fopen(path, "r");
    if (!f) return m;
    char key[256];
    int v;
    while (fscanf(f, "%255s %d", key, &v) == 2) m[key] = v;
    fclose(f);
    return m;
}

static void append_cache(const char* path, const std::string& key, int v) {
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d\n", key.c_str(), v);
    fclose(f);
}

// ------------------------------------------------------------ group work

static int pbh_build_tiles(leb_batch_s* b, PbhGroup& g, int T, PbhTile** dev, int* n_tiles) {
    std::vector<PbhTile> h;
    const int nx = g.dyn.nx, nu = g.dyn.nu, n = nx + nu;
    for (int pi : g.probs) {
        const leb_problem& p = b->probs[pi];
        for (int u0 = 0; u0 < p.N; u0 += T) {
            PbhTile t = {};
            t.z = p.z + (int64_t)u0 * nx;
            t.v = p.v ? p.v + (int64_t)u0 * nu : nullptr;
            t.mu = p.mu ? p.mu + (int64_t)u0 * n : nullptr;
            t.sigma = p.sigma + (int64_t)u0 * n;
            t.r_lo = p.r_lo + (int64_t)u0 * nx;
            t.r_hi = p.r_hi + (int64_t)u0 * nx;
            t.n = std::min(T, p.N - u0);
            h.push_back(t);
        }
    }
    int rc = balloc(b, h.size() * sizeof(PbhTile), (void**)dev);
    if (rc) return rc;
    if (hipMemcpy(*dev, h.data(), h.size() * sizeof(PbhTile), hipMemcpyHostToDevice) != hipSuccess) return LEB_EDEVICE;
    *n_tiles = (int)h.size();
    return LEB_OK;
}

static int pbh_run(const PbhGroup& g, hipStream_t s) { return launch_pbh_tiles(&g.dyn, g.tiles, g.n_tiles, g.T, s); }

static int nn_run(const NNGroup& g, hipStream_t s) {
    const int n0 = g.nx + g.nu;
    hipLaunchKernelGGL(nn_gather_kernel, dim3(nbk(g.units * n0)), dim3(256), 0, s, g.ptrs, g.unit_prob, g.units, g.nx,
                       g.nu, g.zS, g.vS, g.muS, g.sgS);
    if (hipGetLastError() != hipSuccess) return LEB_EDEVICE;
    int rc = nn_bound_run(g.net, g.units, g.zS, g.vS, g.muS, g.sgS, nullptr, g.loS, g.hiS, nullptr, nullptr, 0.0, nullptr, g.CB,
                          g.buf, s);
    if (rc) return rc;
    hipLaunchKernelGGL(nn_scatter_kernel, dim3(nbk(g.units * g.m)), dim3(256), 0, s, g.ptrs, g.unit_prob, g.units, g.m,
                       g.loS, g.hiS);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

// median of 3 timed runs after one warm-up, in microseconds
template <class F>
static int time_us(F run, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* us) {
    int rc = run();
    if (rc) return rc;
    float t[3];
    for (int r = 0; r < 3; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) return LEB_EDEVICE;
        if ((rc = run())) return rc;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t[r], e0, e1) != hipSuccess)
            return LEB_EDEVICE;
    }
    std::sort(t, t + 3);
    *us = t[1] * 1e3f;
    return LEB_OK;
}

static bool same_chain(const leb_dynamics& a, const leb_dynamics& b) {
    return a.n_units == b.n_units && a.dt == b.dt && a.m == b.m && a.k_spring == b.k_spring &&
           a.rest_len == b.rest_len;
}

extern "C" int leb_batch_create(const leb_problem* probs, int32_t count, const char* tune_cache, leb_batch* out) {
    if (!out || count < 0 || (count > 0 && !probs)) return LEB_EINVAL;
    *out = nullptr;
    // validate
    for (int i = 0; i < count; ++i) {
        const leb_problem& p = probs[i];
        if (p.N < 1 || !p.z || !p.sigma || !p.r_lo || !p.r_hi) return LEB_EINVAL;
        const void* ptrs[] = {p.z, p.v, p.mu, p.sigma, p.r_lo, p.r_hi};
        for (const void* q : ptrs)
            if (q && !aligned8(q)) return LEB_EINVAL;
        if (p.type == LEB_PROBLEM_ANALYTIC) {
            int rc = check_chain_dynamics(p.dyn);
            if (rc) return rc;
            if (p.dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_ENOTSUP;
            if (!p.v) return LEB_EINVAL;
        } else if (p.type == LEB_PROBLEM_NN) {
            if (!p.net) return LEB_EINVAL;
            int nx, nu, m;
            nn_dims(p.net, &nx, &nu, &m);
            if (nu > 0 && !p.v) return LEB_EINVAL;
        } else {
            return LEB_EINVAL;
        }
    }
    leb_batch_s* b = new (std::nothrow) leb_batch_s;
    if (!b) return LEB_ENOMEM;
    b->probs.assign(probs, probs + count);
    int rc = LEB_OK;
    if (hipStreamCreateWithFlags(&b->s0, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&b->s1, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess) {
        batch_free(b);
        return LEB_EDEVICE;
    }
    // group
    for (int i = 0; i < count; ++i) {
        const leb_problem& p = b->probs[i];
        if (p.type == LEB_PROBLEM_ANALYTIC) {
            auto it = std::find_if(b->pbh.begin(), b->pbh.end(), [&](const PbhGroup& g) { return same_chain(g.dyn, *p.dyn); });
            if (it == b->pbh.end()) {
                b->pbh.emplace_back();
                b->pbh.back().dyn = *p.dyn;
                it = b->pbh.end() - 1;
            }
            it->probs.push_back(i);
            it->units += p.N;
        } else {
            auto it = std::find_if(b->nn.begin(), b->nn.end(), [&](const NNGroup& g) { return g.net == p.net; });
            if (it == b->nn.end()) {
                b->nn.emplace_back();
                NNGroup& g = b->nn.back();
                g.net = p.net;
                nn_dims(p.net, &g.nx, &g.nu, &g.m);
                it = b->nn.end() - 1;
            }
            it->probs.push_back(i);
            it->units += p.N;
        }
    }
    const std::string arch = arch_name();
    std::map<std::string, int> cache = read_cache(tune_cache);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        batch_free(b);
        return LEB_EDEVICE;
    }
    char key[256];
    // analytic groups: T in {256/U, 128/U, 64/U}
    for (PbhGroup& g : b->pbh) {
        if (rc) break;
        const int U = g.dyn.n_units;
        snprintf(key, sizeof key, "%s|pbh|U=%d|units=%lld", arch.c_str(), U, (long long)bucket(g.units));
        std::vector<int> cand;
        for (int lanes : {PBH_BLOCK_LANES, PBH_BLOCK_LANES / 2, PBH_BLOCK_LANES / 4})
            if (lanes / U >= 1 && std::find(cand.begin(), cand.end(), lanes / U) == cand.end()) cand.push_back(lanes / U);
        auto hit = cache.find(key);
        if (hit != cache.end() && std::find(cand.begin(), cand.end(), hit->second) != cand.end()) {
            g.T = hit->second;
            g.cached = true;
            rc = pbh_build_tiles(b, g, g.T, &g.tiles, &g.n_tiles);
            continue;
        }
        float best = 1e30f;
        for (int T : cand) {
            PbhGroup trial = g;
            trial.T = T;
            if ((rc = pbh_build_tiles(b, trial, T, &trial.tiles, &trial.n_tiles))) break;
            float us = 0;
            if ((rc = time_us([&] { return pbh_run(trial, b->s0); }, b->s0, e0, e1, &us))) break;
            if (us < best) { best = us; g.T = T; g.tiles = trial.tiles; g.n_tiles = trial.n_tiles; }
        }
        if (!rc) append_cache(tune_cache, key, g.T);
    }
    // MLP groups: staging, work buffers, CB in {256, ..., 4096}
    for (NNGroup& g : b->nn) {
        if (rc) break;
        const int n0 = g.nx + g.nu;
        std::vector<NNProbPtrs> hp;
        std::vector<int> up;
        int64_t off = 0;
        for (int pi : g.probs) {
            const leb_problem& p = b->probs[pi];
            NNProbPtrs q = {p.z, p.v, p.mu, p.sigma, p.r_lo, p.r_hi, off, p.N, 0};
            for (int k = 0; k < p.N; ++k) up.push_back((int)hp.size());
            hp.push_back(q);
            off += p.N;
        }
        if ((rc = balloc(b, hp.size() * sizeof(NNProbPtrs), (void**)&g.ptrs)) ||
            (rc = balloc(b, up.size() * sizeof(int), (void**)&g.unit_prob)) ||
            (rc = balloc(b, g.units * g.nx * 8, (void**)&g.zS)) || (rc = balloc(b, g.units * g.nu * 8, (void**)&g.vS)) ||
            (rc = balloc(b, g.units * n0 * 8, (void**)&g.muS)) || (rc = balloc(b, g.units * n0 * 8, (void**)&g.sgS)) ||
            (rc = balloc(b, g.units * g.m * 8, (void**)&g.loS)) || (rc = balloc(b, g.units * g.m * 8, (void**)&g.hiS)))
            break;
        if (hipMemcpy(g.ptrs, hp.data(), hp.size() * sizeof(NNProbPtrs), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g.unit_prob, up.data(), up.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
            rc = LEB_EDEVICE;
            break;
        }
        std::vector<int> cand;
        for (int CB : {256, 512, 1024, 2048, 4096}) cand.push_back((int)std::min<int64_t>(CB, g.units));
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        const int cbmax = *std::max_element(cand.begin(), cand.end());
        size_t sizes[NN_NBUF];
        nn_buffer_sizes(g.net, cbmax, sizes);
        for (int q = 0; q < NN_NBUF && !rc; ++q) rc = balloc(b, sizes[q], (void**)&g.buf[q]);
        if (rc) break;
        const int widest = (int)lround(sqrt((double)(sizes[14] / ((size_t)cbmax * 3 * 8))));
        snprintf(key, sizeof key, "%s|nn|nx=%d|m=%d|units=%lld|maxw=%d", arch.c_str(), g.nx, g.m,
                 (long long)bucket(g.units), widest);
        auto hit = cache.find(key);
        if (hit != cache.end() && std::find(cand.begin(), cand.end(), hit->second) != cand.end()) {
            g.CB = hit->second;
            g.cached = true;
            continue;
        }
        float best = 1e30f;
        int best_cb = cand[0];
        for (int CB : cand) {
            g.CB = CB;
            float us = 0;
            if ((rc = time_us([&] { return nn_run(g, b->s1); }, b->s1, e0, e1, &us))) break;
            if (us < best) { best = us; best_cb = CB; }
        }
        g.CB = best_cb;
        if (!rc) append_cache(tune_cache, key, g.CB);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the analytic groups' tiles as one work queue, largest tiles first
    if (!rc && !b->pbh.empty()) {
        std::vector<const PbhGroup*> order;
        for (const PbhGroup& g : b->pbh) order.push_back(&g);
        std::stable_sort(order.begin(), order.end(), [](const PbhGroup* x, const PbhGroup* y) {
            return x->T * x->dyn.n_units > y->T * y->dyn.n_units;
        });
        std::vector<PbhQueueGroup> hq;
        int first = 0;
        for (const PbhGroup* g : order) {
            PbhQueueGroup q;
            q.tiles = g->tiles; q.first = first; q.n_tiles = g->n_tiles;
            q.U = g->dyn.n_units; q.T = g->T;
            q.c = g->dyn.dt / g->dyn.m; q.kL = g->dyn.k_spring * g->dyn.rest_len; q.L0 = g->dyn.rest_len;
            hq.push_back(q);
            first += g->n_tiles;
            b->queue_smem = std::max(b->queue_smem, pbh_smem_bytes_T(q.U, q.T));
        }
        PbhQueueGroup* dq = nullptr;
        int* cnt = nullptr;
        if ((rc = balloc(b, hq.size() * sizeof(PbhQueueGroup), (void**)&dq)) ||
            (rc = balloc(b, sizeof(int), (void**)&cnt))) {
        } else if (hipMemcpy(dq, hq.data(), hq.size() * sizeof(PbhQueueGroup), hipMemcpyHostToDevice) != hipSuccess) {
            rc = LEB_EDEVICE;
        } else {
            b->queue = PbhQueueArgs{dq, (int)hq.size(), first, cnt};
            b->queue_grid = pbh_queue_grid(b->queue_smem, first);
            if (b->queue_grid < 1) rc = LEB_EDEVICE;
        }
    }
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = LEB_EDEVICE;
    // capture: analytic groups on s0, MLP groups on s1, joined
    if (!rc) {
        if (hipStreamBeginCapture(b->s0, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = LEB_EDEVICE;
        bool capturing = !rc;
        if (!rc && (hipEventRecord(b->fork, b->s0) != hipSuccess || hipStreamWaitEvent(b->s1, b->fork, 0) != hipSuccess))
            rc = LEB_EDEVICE;
        if (!rc && b->queue.total > 0) rc = launch_pbh_queue(b->queue, b->queue_smem, b->queue_grid, b->s0);
        for (const NNGroup& g : b->nn)
            if (!rc) rc = nn_run(g, b->s1);
        if (!rc && (hipEventRecord(b->join, b->s1) != hipSuccess || hipStreamWaitEvent(b->s0, b->join, 0) != hipSuccess))
            rc = LEB_EDEVICE;
        if (capturing) {
            hipGraph_t gr = nullptr;
            const hipError_t e = hipStreamEndCapture(b->s0, &gr);
            if (!rc && e != hipSuccess) rc = LEB_EDEVICE;
            if (gr) b->graph = gr;
        }
        if (!rc && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) rc = LEB_EDEVICE;
    }
    if (rc) {
        batch_free(b);
        return rc;
    }
    char line[256];
    if (b->queue.total > 0) {
        snprintf(line, sizeof line, "pbh work queue: %d tiles of %d groups, %d persistent workgroups\n", b->queue.total,
                 b->queue.n_groups, b->queue_grid);
        b->info += line;
    }
    for (const PbhGroup& g : b->pbh) {
        snprintf(line, sizeof line, "pbh U=%d problems=%zu units=%lld T=%d%s\n", g.dyn.n_units, g.probs.size(),
                 (long long)g.units, g.T, g.cached ? " (cached)" : "");
        b->info += line;
    }
    for (const NNGroup& g : b->nn) {
        snprintf(line, sizeof line, "nn nx=%d m=%d problems=%zu units=%lld CB=%d%s\n", g.nx, g.m, g.probs.size(),
                 (long long)g.units, g.CB, g.cached ? " (cached)" : "");
        b->info += line;
    }
    *out = b;
    return LEB_OK;
}

extern "C" int leb_batch_submit(leb_batch b, void* stream) {
    if (!b || !b->exec) return LEB_EINVAL;
    return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_batch_destroy(leb_batch b) {
    if (!b) return LEB_OK;
    (void)hipDeviceSynchronize();
    batch_free(b);
    return LEB_OK;
}

extern "C" int leb_batch_info(leb_batch b, char* buf, int32_t len) {
    if (!b || !buf || len < 1) return LEB_EINVAL;
    snprintf(buf, (size_t)len, "%s", b->info.c_str());
    return LEB_OK;
}
