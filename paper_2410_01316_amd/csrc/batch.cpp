// Batched form of libfastsum: many independent kernel-sum problems run by one
// persistent launch per phase, captured into a HIP graph and replayed.
#include "fastsum.h"
#include "fastsum_impl.h"
#include "host_common.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

using namespace fastsum;
using namespace fastsum::host;

namespace {

struct ProblemPlan {
    Resolved r;
    GridGeom geom;
    int dpad = 0;
    int64_t n_max = 0, m_max = 0, ldx = 0, ldy = 0, ldm = 0;
    int nchunk_cap = 1, ngroup_cap = 1;
    // arena offsets (bytes); fused batches hold split tiles (at, xt, yt)
    // in place of A and the projections
    size_t off_A = 0, off_xproj = 0, off_yproj = 0, off_partial = 0, off_grid = 0,
           off_spart = 0, off_exp = 0, off_mult = 0, off_tw = 0;
    float bound = 0.f;
    float norm2_max = 0.f;     // fused range check: |x / R|^2 bound
    float norm_lim = 1.f;      // bound check: (1 + 1e-5) / max_p |xi_p|
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

struct fastsum_batch_s {
    fastsum_params common{};
    WindowPoly win;
    WindowArgs win_args{};
    int P = 0, W = 4, pstage = 8, nprob = 0, device = 0, num_cu = 256;
    // projections computed inside spread and gather (every d <= 64, unless
    // FASTSUM_FLAG_MATERIALIZE asks for stored projections)
    bool fused = false;
    fastsum_batch_tuning tuning{};
    std::vector<ProblemPlan> plans;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    // descriptors and task lists on the device, staging copies on the host
    BatchProblem* d_probs = nullptr;
    BatchTask* d_tasks = nullptr;
    BatchProblem* h_probs = nullptr;   // pinned
    BatchTask* h_tasks = nullptr;      // pinned
    size_t task_cap = 0;
    int task_off[kBatchPhases] = {};
    int task_cnt[kBatchPhases] = {};
    size_t lds_spread = 0, lds_fft = 0, lds_gather = 0;
    int* flag = nullptr;
    unsigned* norms = nullptr;         // bound check slots, kNormUints per problem
    bool norms_dirty = false;          // a direct launch stopped before the checks cleared them
    // replay state
    std::vector<fastsum_problem_io> last_io;
    bool have_tasks = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // recorded after every upload from the staging buffers and every launch:
    // waited for before the staging buffers are rewritten or the graph is
    // destroyed, on whichever stream the earlier calls ran
    hipEvent_t last_use = nullptr;
    bool used = false;
};

namespace {

// Wait until nothing enqueued earlier still reads the staging buffers or
// runs the graph.
hipError_t wait_idle(fastsum_batch_s* b) {
    if (!b->used) return hipSuccess;
    const hipError_t e = hipEventSynchronize(b->last_use);
    if (e == hipSuccess) b->used = false;
    return e;
}

hipError_t mark_used(fastsum_batch_s* b, hipStream_t st) {
    const hipError_t e = hipEventRecord(b->last_use, st);
    if (e == hipSuccess) b->used = true;
    return e;
}

void drop_graph(fastsum_batch_s* b) {
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
}

void free_batch(fastsum_batch_s* b) {
    if (!b) return;
    if (b->last_use) (void)wait_idle(b);
    drop_graph(b);
    if (b->last_use) (void)hipEventDestroy(b->last_use);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->arena) (void)hipFree(b->arena);
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->d_tasks) (void)hipFree(b->d_tasks);
    if (b->flag) (void)hipFree(b->flag);
    if (b->norms) (void)hipFree(b->norms);
    if (b->h_probs) (void)hipHostFree(b->h_probs);
    if (b->h_tasks) (void)hipHostFree(b->h_tasks);
    delete b;
}

// Fused batches: default chunks of 4 slices; a task covers 16 directions,
// so a batch of many problems has ample tasks at this length.
constexpr int64_t kFusedBatchChunk = 4 * kSliceLen;

int chunks_for(const fastsum_batch_s* b, int64_t N) {
    if (b->fused) {
        const int64_t len = b->tuning.spread_chunk > 0 ? b->tuning.spread_chunk : kFusedBatchChunk;
        const int64_t nc = std::max<int64_t>((N + len - 1) / len, (N + kMaxChunk - 1) / kMaxChunk);
        return (int)std::max<int64_t>(nc, 1);
    }
    int nc = spread_chunks(N, b->P);
    if (b->tuning.spread_chunk > 0) nc = (int)((N + b->tuning.spread_chunk - 1) / b->tuning.spread_chunk);
    nc = std::min<int>(nc, std::max<int>(spread_chunks(N, b->P), (int)((N + 4095) / 4096)));
    nc = std::max<int>(nc, (int)((N + kMaxChunk - 1) / kMaxChunk));
    return std::max(nc, 1);
}

int group_for(const fastsum_batch_s* b, int64_t M) {
    if (b->fused)    // one range of all directions unless tuned: targets read once
        return (int)round_up(b->tuning.gather_group > 0 ? b->tuning.gather_group : b->P, kFuseDirs);
    if (b->tuning.gather_group > 0) return (int)round_up(b->tuning.gather_group, b->pstage);
    return gather_group(M, b->P, b->pstage);
}

fastsum_status validate_tuning(const fastsum_batch_tuning* t) {
    if (!t) return FASTSUM_OK;
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64) return FASTSUM_EINVAL;
    if (t->spread_chunk < 0 || (t->spread_chunk % 4096) != 0) return FASTSUM_EINVAL;
    if (t->gather_group < 0 || (t->gather_group % 8) != 0 || t->gather_group > 1024)
        return FASTSUM_EINVAL;
    if (t->use_graph < -1 || t->use_graph > 1) return FASTSUM_EINVAL;
    return FASTSUM_OK;
}

// Task lists of one problem of a fused batch, with a cost estimate per
// spread and gather task (sources or targets times directions) by which
// those phases are ordered, largest first.
void fused_tasks(int i, const BatchProblem& d, const fastsum_problem_io& q, int P,
                 std::vector<BatchTask>* ph, std::vector<int64_t>* cost) {
    const int64_t xtiles = (q.N + 15) / 16, ytiles = (q.M + 15) / 16;
    for (int64_t t = 0; t < (xtiles + kSplitTaskTiles - 1) / kSplitTaskTiles; ++t)
        ph[kBatchProject].push_back({i, 0, (int)t, 0});
    if (!d.same_xy)
        for (int64_t t = 0; t < (ytiles + kSplitTaskTiles - 1) / kSplitTaskTiles; ++t)
            ph[kBatchProject].push_back({i, 1, (int)t, 0});
    for (int c = 0; c < (int)((q.N + kSliceLen - 1) / kSliceLen); ++c)
        ph[kBatchScale].push_back({i, c, 0, 0});
    const int groups = (P + kFuseDirs - 1) / kFuseDirs;
    for (int c = 0; c < d.nchunk; ++c) {
        const int64_t len = std::min<int64_t>(d.chunk_len, q.N - (int64_t)c * d.chunk_len);
        for (int g = 0; g < groups; ++g) {
            ph[kBatchSpread].push_back({i, g, c, 0});
            cost[kBatchSpread].push_back(len * std::min(kFuseDirs, P - g * kFuseDirs));
        }
    }
    for (int a = 0; a < (P + 1) / 2; ++a) ph[kBatchFftconv].push_back({i, a, 0, 0});
    const int64_t tile = fused_gather_tile(0, 4);    // batched plans: narrow grids
    const int gtiles = (int)((q.M + tile - 1) / tile);
    for (int r = 0; r < d.ngroup; ++r)
        for (int t = 0; t < gtiles; ++t) {
            ph[kBatchGather].push_back({i, t, r, 0});
            cost[kBatchGather].push_back(std::min<int64_t>(tile, q.M - t * tile) *
                                         std::min(d.pg, P - r * d.pg));
        }
    const int rt = (int)((q.M + kBlock - 1) / kBlock);
    for (int t = 0; t < rt; ++t) ph[kBatchReduce].push_back({i, t, 0, 0});
}

void sort_by_cost(std::vector<BatchTask>& tasks, const std::vector<int64_t>& cost) {
    std::vector<size_t> idx(tasks.size());
    for (size_t k = 0; k < idx.size(); ++k) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    std::vector<BatchTask> out(tasks.size());
    for (size_t k = 0; k < idx.size(); ++k) out[k] = tasks[idx[k]];
    tasks.swap(out);
}

// Fill h_probs / h_tasks for the given io and record per-phase ranges.
fastsum_status build_tasks(fastsum_batch_s* b, const fastsum_problem_io* io) {
    const int P = b->P;
    std::vector<BatchTask> ph[kBatchPhases];
    std::vector<int64_t> cost[kBatchPhases];
    for (int i = 0; i < b->nprob; ++i) {
        const ProblemPlan& pp = b->plans[i];
        const fastsum_problem_io& q = io[i];
        BatchProblem& d = b->h_probs[i];
        std::memset(&d, 0, sizeof(d));
        d.x = q.x;
        d.w = q.w;
        d.y = q.y;
        d.s = q.s;
        d.N = q.N;
        d.M = q.M;
        d.same_xy = (q.x == q.y) ? 1 : 0;
        if (b->fused) {
            d.at = reinterpret_cast<const uint16_t*>(b->arena + pp.off_A);
            d.xt = reinterpret_cast<uint16_t*>(b->arena + pp.off_xproj);
            d.yt = reinterpret_cast<uint16_t*>(b->arena + pp.off_yproj);
            d.pscale = (float)(pp.r.tau * pp.r.p.R);
            d.norm2_max = pp.norm2_max;
            d.kb = split_kblocks(pp.r.p.d);
        } else {
            d.A = reinterpret_cast<const float*>(b->arena + pp.off_A);
            d.xproj = reinterpret_cast<float*>(b->arena + pp.off_xproj);
            d.yproj = reinterpret_cast<float*>(b->arena + pp.off_yproj);
        }
        d.inv_r = (float)(1.0 / pp.r.p.R);
        d.norms = b->norms + (size_t)kNormUints * i;
        d.norm_lim = pp.norm_lim;
        d.partial = reinterpret_cast<float*>(b->arena + pp.off_partial);
        d.grid = reinterpret_cast<float*>(b->arena + pp.off_grid);
        d.spart = reinterpret_cast<double*>(b->arena + pp.off_spart);
        d.slice_max = reinterpret_cast<float*>(b->arena + pp.off_exp);
        d.mult = reinterpret_cast<const float2*>(b->arena + pp.off_mult);
        d.tw = reinterpret_cast<const float2*>(b->arena + pp.off_tw);
        d.ldx = pp.ldx;
        d.ldy = pp.ldy;
        d.ldm = pp.ldm;
        d.g = pp.geom;
        d.d = pp.r.p.d;
        d.dpad = pp.dpad;
        d.bound = pp.bound;
        d.nchunk = chunks_for(b, q.N);
        if (d.nchunk > pp.nchunk_cap) return FASTSUM_EINVAL;
        d.chunk_len = spread_chunk_len(q.N, d.nchunk);
        d.pg = group_for(b, q.M);
        d.ngroup = (P + d.pg - 1) / d.pg;
        if (d.ngroup > pp.ngroup_cap) return FASTSUM_EINVAL;

        if (b->fused) {
            fused_tasks(i, d, q, P, ph, cost);
            continue;
        }
        const int ptiles = (P + kProjTileP - 1) / kProjTileP;
        const int nt = (int)((q.N + kProjTileN - 1) / kProjTileN);
        const int mt = (int)((q.M + kProjTileN - 1) / kProjTileN);
        for (int t = 0; t < nt; ++t)
            for (int c = 0; c < ptiles; ++c) ph[kBatchProject].push_back({i, 0, t, c});
        if (!d.same_xy)
            for (int t = 0; t < mt; ++t)
                for (int c = 0; c < ptiles; ++c) ph[kBatchProject].push_back({i, 1, t, c});
        for (int c = 0; c < (int)((q.N + kSliceLen - 1) / kSliceLen); ++c)
            ph[kBatchScale].push_back({i, c, 0, 0});
        for (int c = 0; c < d.nchunk; ++c)
            for (int p = 0; p < P; ++p) ph[kBatchSpread].push_back({i, p, c, 0});
        for (int a = 0; a < (P + 1) / 2; ++a) ph[kBatchFftconv].push_back({i, a, 0, 0});
        const int gtiles = (int)((q.M + kGatherTile - 1) / kGatherTile);
        for (int g = 0; g < d.ngroup; ++g)
            for (int t = 0; t < gtiles; ++t) ph[kBatchGather].push_back({i, t, g, 0});
        const int rt = (int)((q.M + kBlock - 1) / kBlock);
        for (int t = 0; t < rt; ++t) ph[kBatchReduce].push_back({i, t, 0, 0});
    }
    if (b->fused) {
        sort_by_cost(ph[kBatchSpread], cost[kBatchSpread]);
        sort_by_cost(ph[kBatchGather], cost[kBatchGather]);
    }
    size_t total = 0;
    for (int k = 0; k < kBatchPhases; ++k) total += ph[k].size();
    if (total > b->task_cap) return FASTSUM_EINVAL;
    size_t off = 0;
    for (int k = 0; k < kBatchPhases; ++k) {
        b->task_off[k] = (int)off;
        b->task_cnt[k] = (int)ph[k].size();
        if (!ph[k].empty()) std::memcpy(b->h_tasks + off, ph[k].data(), ph[k].size() * sizeof(BatchTask));
        off += ph[k].size();
    }
    return FASTSUM_OK;
}

fastsum_status launch_all(fastsum_batch_s* b, hipStream_t st) {
    const int bpc = b->tuning.blocks_per_cu > 0 ? b->tuning.blocks_per_cu : 4;
    const int grid_blocks = bpc * b->num_cu;
    const size_t lds[kBatchPhases] = {0, 0, b->lds_spread, b->lds_fft, b->lds_gather, 0};
    for (int k = 0; k < kBatchPhases; ++k) {
        hipError_t e = b->fused
            ? launch_batch_phase_fused(k, b->W, b->d_probs, b->d_tasks + b->task_off[k],
                                       b->task_cnt[k], b->P, b->win_args, b->flag, grid_blocks,
                                       lds[k], st)
            : launch_batch_phase(k, b->W, b->d_probs, b->d_tasks + b->task_off[k],
                                 b->task_cnt[k], b->P, b->pstage, b->win_args, b->flag,
                                 grid_blocks, lds[k], st);
        if (e != hipSuccess) return status_of(e);
    }
    return FASTSUM_OK;
}

bool same_io(const std::vector<fastsum_problem_io>& a, const fastsum_problem_io* b, int n) {
    if ((int)a.size() != n) return false;
    for (int i = 0; i < n; ++i)
        if (a[i].x != b[i].x || a[i].w != b[i].w || a[i].y != b[i].y || a[i].s != b[i].s ||
            a[i].N != b[i].N || a[i].M != b[i].M)
            return false;
    return true;
}

}  // namespace

extern "C" {

fastsum_status fastsum_choose_nft(const fastsum_params* prm, const int32_t* candidates,
                                  int32_t n_candidates, double tol, int32_t* chosen) {
    if (!prm || !candidates || n_candidates < 1 || !chosen || !(tol >= 0.0)) return FASTSUM_EINVAL;
    Resolved r;
    int32_t best = -1, largest = -1;
    for (int i = 0; i < n_candidates; ++i) {
        fastsum_params q = *prm;
        q.n_ft = candidates[i];
        fastsum_status st = resolve_params(&q, r);
        if (st != FASTSUM_OK) return st;
        largest = std::max(largest, candidates[i]);
    }
    const int kmax = 4096;
    std::vector<double> c;
    fourier_coefficients_upto(r.p.kernel, r.p.d, r.p.scale, r.tau, kmax, c);
    double total = std::fabs(c[0]);
    for (int k = 1; k <= kmax; ++k) total += 2.0 * std::fabs(c[k]);
    for (int i = 0; i < n_candidates; ++i) {
        const int K = candidates[i] / 2;
        double tail = 0.0;
        for (int k = K + 1; k <= kmax; ++k) tail += 2.0 * std::fabs(c[k]);
        if (tail <= tol * total && (best < 0 || candidates[i] < best)) best = candidates[i];
    }
    *chosen = best > 0 ? best : largest;
    return FASTSUM_OK;
}

fastsum_status fastsum_batch_create(const fastsum_params* common, const fastsum_problem_desc* probs,
                                    int32_t n_problems, const fastsum_batch_tuning* tuning,
                                    void* stream, fastsum_batch* out) {
    if (!common || !probs || n_problems < 1 || !out) return FASTSUM_EINVAL;
    if (common->proj != FASTSUM_PROJ_FP32 || (common->flags & ~FASTSUM_FLAG_MATERIALIZE) != 0)
        return FASTSUM_EUNSUPPORTED;
    if (validate_tuning(tuning) != FASTSUM_OK) return FASTSUM_EINVAL;
    hipStream_t hs = (hipStream_t)stream;
    fastsum_batch_s* b = new (std::nothrow) fastsum_batch_s();
    if (!b) return FASTSUM_ENOMEM;
    b->common = *common;
    b->nprob = n_problems;
    if (tuning) b->tuning = *tuning;
    b->plans.resize(n_problems);

    // per-problem FP64 precompute and arena layout
    size_t off = 0;
    int max_nr = 8, max_n = 8;
    std::vector<std::vector<float2>> mults(n_problems), tws(n_problems);
    std::vector<std::vector<float>> As(n_problems);
    std::vector<std::vector<uint16_t>> Ats(n_problems);
    for (int i = 0; i < n_problems; ++i) {
        const fastsum_problem_desc& pd = probs[i];
        if (!pd.xi || pd.n_max < 1 || pd.m_max < 1) { free_batch(b); return FASTSUM_EINVAL; }
        fastsum_params q = *common;
        q.d = pd.d;
        q.n_ft = pd.n_ft;
        q.scale = pd.scale;
        q.R = pd.R;
        ProblemPlan& pp = b->plans[i];
        if (resolve_params(&q, pp.r) != FASTSUM_OK) { free_batch(b); return FASTSUM_EINVAL; }
        if (i == 0) {
            b->P = pp.r.p.P;
            b->W = pp.r.p.window_w;
            if (!build_window(b->W, b->win)) { free_batch(b); return FASTSUM_EINVAL; }
            b->win_args = pack_window(b->win);
        }
        const int n = pp.r.n;
        pp.geom = make_geom(n, b->W, pp.r.tau * pp.r.p.R);
        pp.bound = (float)(pp.r.tau * pp.r.p.R * (1.0 + 1e-5) + 1e-7);
        pp.dpad = (int)round_up(pp.r.p.d, 4);
        pp.n_max = pd.n_max;
        pp.m_max = pd.m_max;
        pp.ldx = round_up(pd.n_max, 64);
        pp.ldy = round_up(pd.m_max, 64);
        pp.ldm = round_up(std::max(pd.n_max, pd.m_max), 64);
        max_nr = std::max(max_nr, pp.geom.nr);
        max_n = std::max(max_n, n);
        std::vector<float2> mult_d;
        build_tables(pp.r.p.kernel, pp.r.p.d, pp.r.p.scale, pp.r.tau, pp.r.p.n_ft, n, b->win,
                     mults[i], mult_d, tws[i]);
        As[i].assign((size_t)b->P * pp.dpad, 0.f);
        double xi_norm_max = 0.0;
        for (int p = 0; p < b->P; ++p) {
            double ss = 0.0;
            for (int k = 0; k < pp.r.p.d; ++k) {
                const double v = pd.xi[(size_t)k * b->P + p];
                As[i][(size_t)p * pp.dpad + k] = (float)(pp.r.tau * v);
                ss += v * v;
            }
            xi_norm_max = std::max(xi_norm_max, std::sqrt(ss));
        }
        if (!(xi_norm_max > 0.0)) xi_norm_max = 1.0;
        // |x~| <= tau R for every direction when |x| max|xi| <= R
        const double lim = (1.0 + 1e-5) / xi_norm_max;
        pp.norm2_max = (float)(lim * lim);
        // |x~ - y~| <= tau max|xi| (|x| + |y|) <= tau R when the bound holds
        pp.norm_lim = (float)lim;
    }
    b->fused = (common->flags & FASTSUM_FLAG_MATERIALIZE) == 0;
    for (int i = 0; i < n_problems; ++i)
        b->fused = b->fused && fused_supported(b->plans[i].r.p.d, b->plans[i].geom.nr) &&
                   !fused_wide(b->plans[i].geom.nr);
    if (b->fused)
        for (int i = 0; i < n_problems; ++i) {
            split_dirs_host(probs[i].xi, b->plans[i].r.p.d, b->P, Ats[i]);
            As[i].clear();
        }
    b->pstage = std::max(1, std::min(8, 12288 / max_nr));
    size_t tasks = 0;
    for (int i = 0; i < n_problems; ++i) {
        ProblemPlan& pp = b->plans[i];
        const int P = b->P;
        // caps: every admissible N and tuning (chunks of >= 4096 sources)
        int nc = std::max(chunks_for(b, pp.n_max), spread_chunks(pp.n_max, P));
        nc = std::max(nc, (int)((pp.n_max + 4095) / 4096));
        const int ng = (P + (b->fused ? kFuseDirs : b->pstage) - 1) /
                       (b->fused ? kFuseDirs : b->pstage);
        pp.nchunk_cap = nc;
        pp.ngroup_cap = ng;
        const int nr = pp.geom.nr, n = pp.r.n;
        if (b->fused) {
            pp.off_A = off; off = align256(off + Ats[i].size() * sizeof(uint16_t));
            pp.off_xproj = off; off = align256(off + (size_t)split_tiles_bytes(pp.n_max, pp.r.p.d));
            pp.off_yproj = off; off = align256(off + (size_t)split_tiles_bytes(pp.m_max, pp.r.p.d));
        } else {
            pp.off_A = off; off = align256(off + sizeof(float) * (size_t)P * pp.dpad);
            pp.off_xproj = off; off = align256(off + sizeof(float) * (size_t)P * pp.ldx);
            pp.off_yproj = off; off = align256(off + sizeof(float) * (size_t)P * pp.ldy);
        }
        pp.off_partial = off; off = align256(off + sizeof(float) * (size_t)nc * P * nr);
        pp.off_grid = off; off = align256(off + sizeof(float) * (size_t)P * nr);
        pp.off_spart = off; off = align256(off + sizeof(double) * (size_t)ng * pp.ldm);
        pp.off_exp = off; off = align256(off + sizeof(float) * (size_t)((pp.n_max + kSliceLen - 1) / kSliceLen));
        pp.off_mult = off; off = align256(off + sizeof(float2) * (size_t)n);
        pp.off_tw = off; off = align256(off + sizeof(float2) * (size_t)n);
        const size_t ptiles = (P + kProjTileP - 1) / kProjTileP;
        tasks += ptiles * ((pp.n_max + kProjTileN - 1) / kProjTileN + (pp.m_max + kProjTileN - 1) / kProjTileN);
        tasks += (size_t)nc * P + (pp.n_max + kSliceLen - 1) / kSliceLen;
        tasks += (P + 1) / 2;
        tasks += (size_t)ng * ((pp.m_max + kGatherTile - 1) / kGatherTile);
        tasks += (pp.m_max + kBlock - 1) / kBlock;
        if (b->fused)    // split tasks (the others are bounded by the stored form's)
            tasks += (size_t)((pp.n_max + 16 * kSplitTaskTiles - 1) / (16 * kSplitTaskTiles) +
                              (pp.m_max + 16 * kSplitTaskTiles - 1) / (16 * kSplitTaskTiles));
    }
    b->arena_bytes = off;
    b->task_cap = tasks;
    b->lds_spread = b->fused ? fused_spread_lds(max_nr) : stored_spread_lds(max_nr);
    b->lds_fft = fftconv_lds_bytes(max_n, false);
    b->lds_gather = b->fused ? fused_gather_lds(max_nr) : (size_t)b->pstage * max_nr * sizeof(float);

    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess) e = hipMalloc((void**)&b->arena, b->arena_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_probs, sizeof(BatchProblem) * n_problems);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_tasks, sizeof(BatchTask) * std::max<size_t>(tasks, 1));
    if (e == hipSuccess) e = hipMalloc((void**)&b->flag, sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void**)&b->norms, sizeof(unsigned) * kNormUints * n_problems);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_probs, sizeof(BatchProblem) * n_problems);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_tasks, sizeof(BatchTask) * std::max<size_t>(tasks, 1));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->last_use, hipEventDisableTiming);
    if (e != hipSuccess) { fastsum_status st = status_of(e); free_batch(b); return st; }
    for (int i = 0; i < n_problems && e == hipSuccess; ++i) {
        const ProblemPlan& pp = b->plans[i];
        e = b->fused ? hipMemcpyAsync(b->arena + pp.off_A, Ats[i].data(),
                                      Ats[i].size() * sizeof(uint16_t), hipMemcpyHostToDevice, hs)
                     : hipMemcpyAsync(b->arena + pp.off_A, As[i].data(), As[i].size() * sizeof(float),
                                      hipMemcpyHostToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->arena + pp.off_mult, mults[i].data(), mults[i].size() * sizeof(float2),
                               hipMemcpyHostToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->arena + pp.off_tw, tws[i].data(), tws[i].size() * sizeof(float2),
                               hipMemcpyHostToDevice, hs);
    }
    if (e == hipSuccess) e = hipMemsetAsync(b->flag, 0, sizeof(int), hs);
    if (e == hipSuccess) e = hipMemsetAsync(b->norms, 0, sizeof(unsigned) * kNormUints * n_problems, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) { free_batch(b); return FASTSUM_EDEVICE; }
    *out = b;
    return FASTSUM_OK;
}

fastsum_status fastsum_batch_set_tuning(fastsum_batch b, const fastsum_batch_tuning* tuning) {
    if (!b) return FASTSUM_EINVAL;
    if (validate_tuning(tuning) != FASTSUM_OK) return FASTSUM_EINVAL;
    if (wait_idle(b) != hipSuccess) return FASTSUM_EDEVICE;
    if (tuning) b->tuning = *tuning;
    else std::memset(&b->tuning, 0, sizeof(b->tuning));
    drop_graph(b);
    b->have_tasks = false;
    b->last_io.clear();
    return FASTSUM_OK;
}

fastsum_status fastsum_batch_exec(fastsum_batch b, const fastsum_problem_io* io, int32_t n,
                                  void* stream) {
    if (!b || !io || n != b->nprob) return FASTSUM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
        const fastsum_problem_io& q = io[i];
        const ProblemPlan& pp = b->plans[i];
        if (!q.x || !q.w || !q.y || !q.s) return FASTSUM_EINVAL;
        if (q.N < 1 || q.M < 1 || q.N > pp.n_max || q.M > pp.m_max) return FASTSUM_EINVAL;
        if (q.x == q.y && q.N != q.M) return FASTSUM_EINVAL;
    }
    const bool use_graph = b->tuning.use_graph != -1;
    if (!b->have_tasks || !same_io(b->last_io, io, n)) {
        // the staging buffers may still feed an earlier upload, the graph an
        // earlier replay
        if (wait_idle(b) != hipSuccess) return FASTSUM_EDEVICE;
        drop_graph(b);
        b->have_tasks = false;
        fastsum_status r = build_tasks(b, io);
        if (r != FASTSUM_OK) return r;
        size_t total = 0;
        for (int k = 0; k < kBatchPhases; ++k) total += b->task_cnt[k];
        hipError_t e = hipMemcpyAsync(b->d_probs, b->h_probs, sizeof(BatchProblem) * n,
                                      hipMemcpyHostToDevice, st);
        if (e == hipSuccess && total)
            e = hipMemcpyAsync(b->d_tasks, b->h_tasks, sizeof(BatchTask) * total,
                               hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = mark_used(b, st);
        if (e != hipSuccess) return FASTSUM_EDEVICE;
        b->last_io.assign(io, io + n);
        b->have_tasks = true;
        if (use_graph) {
            e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return FASTSUM_EDEVICE;
            fastsum_status lr = launch_all(b, b->cap_stream);
            e = hipStreamEndCapture(b->cap_stream, &b->graph);
            if (lr != FASTSUM_OK) { drop_graph(b); b->have_tasks = false; return lr; }
            if (e == hipSuccess) e = hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) { drop_graph(b); b->have_tasks = false; return FASTSUM_EDEVICE; }
        }
    }
    // every problem's first reduce task checks max |x| + max |y| <= R and
    // clears its norm slots; a direct launch that stopped early left them set
    if (b->norms_dirty &&
        hipMemsetAsync(b->norms, 0, sizeof(unsigned) * kNormUints * b->nprob, st) != hipSuccess)
        return FASTSUM_EDEVICE;
    b->norms_dirty = false;
    if (use_graph) {
        if (hipGraphLaunch(b->graph_exec, st) != hipSuccess) return FASTSUM_EDEVICE;
        return mark_used(b, st) == hipSuccess ? FASTSUM_OK : FASTSUM_EDEVICE;
    }
    b->norms_dirty = true;
    const fastsum_status r = launch_all(b, st);
    if (r == FASTSUM_OK) b->norms_dirty = false;
    if (mark_used(b, st) != hipSuccess) return FASTSUM_EDEVICE;
    return r;
}

fastsum_status fastsum_batch_check(fastsum_batch b) {
    if (!b) return FASTSUM_EINVAL;
    int h = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(&h, b->flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e == hipSuccess && h) e = hipMemset(b->flag, 0, sizeof(int));
    if (e != hipSuccess) return FASTSUM_EDEVICE;
    return h ? FASTSUM_ERANGE : FASTSUM_OK;
}

void fastsum_batch_destroy(fastsum_batch b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    free_batch(b);
}

}  // extern "C"
