// Continuous-batching reconstruction server.
//
// One loop thread owns all device work.  Requests (a sinogram, background and
// parameters for a loaded system matrix) are queued by appga_submit from any
// thread.  For every system matrix the loop keeps a pool of 64 lanes in the
// lane layout (iterates, extrapolation, ratio buffers and data stay resident
// on the device) and advances all occupied lanes together: one step is one
// APPGA iteration of the whole pool, replayed from a captured hipGraph (two
// graphs, for the two f~ buffers).  Each lane carries its own iteration
// counter on the device, from which the step kernel forms theta_{k+1}
// (eq. GNtheta) in FP64, so requests at different iterations share a step.
// A request is admitted as soon as its matrix's pool has a free lane and the
// pool fits the HBM budget; it leaves when its own budget of iterations is
// done, its lane is copied out and immediately reusable.  Pools run on their
// own streams, so pools of different geometries overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "appga.h"
#include "appga_impl.h"

using namespace appga;

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kLanes = 64;

struct Request {
    uint64_t ticket = 0;
    const appga_matrix *mat = nullptr;
    std::vector<float> g, gamma;  // gamma empty: params.gamma_scalar in every bin
    appga_params p{};
    Clock::time_point t_submit;
    std::vector<float> result;
    appga_stats stats{};
    appga_status status = APPGA_OK;
    std::string error;            // message of a failed request (set by the loop thread)
    bool done = false;
};

// Pinned host staging of one admission: data, background and the lane's
// small state, copied to the device in stream order; reusable once `ev` has
// completed.
struct Stage {
    float *h = nullptr;      // g (m), gamma (m), then LaneParams, {a, b, omega, none}, k0, clamps
    hipEvent_t ev = nullptr;
    bool used = false;
};
constexpr int kStageRing = 8;
constexpr int kDepth = 16;   // steps in flight per pool

struct Pool {
    const appga_matrix *mat = nullptr;
    hipStream_t stream = nullptr;
    void *arena = nullptr;
    int64_t bytes = 0;
    float *g = nullptr, *gamma = nullptr, *f = nullptr, *ft[2] = {nullptr, nullptr}, *e = nullptr;
    float *gf = nullptr;                              // A^T e of the tile kernel (or null)
    float *tile_part = nullptr;                       // partial sums of split forward tiles (or null)
    LaneParams *lp = nullptr;
    double *mom = nullptr;
    int *lane_k = nullptr;
    float *theta = nullptr;                           // [64] theta_{k+1}
    unsigned long long *clamps = nullptr;
    float *stage_in = nullptr, *stage_out = nullptr;  // device staging (m floats, d floats)
    Stage stages[kStageRing];
    int next_stage = 0;
    float *h_res = nullptr;                           // pinned results: 64 x (d + 4) floats
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int parity = 0;                                   // which ft buffer holds f~^k
    std::shared_ptr<Request> lane_req[kLanes];
    int lane_done_iters[kLanes] = {};
    bool lane_out[kLanes] = {};                       // result copy of the lane not yet collected
    std::deque<hipEvent_t> inflight;                  // events of launched steps
    std::vector<hipEvent_t> free_events;
    int pending_out = 0;                              // result copies not yet completed
};

struct Extraction {
    std::shared_ptr<Request> req;
    Pool *pool = nullptr;
    hipEvent_t ev = nullptr;
    int lane = 0;
    int d = 0;                       // image size of the request's matrix
};

}  // namespace

struct appga_server {
    appga_ctx *ctx = nullptr;
    appga_server_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> arrivals;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::thread loop;
    // loop-thread state, keyed by the matrix's serial number (an address can be
    // reused by a later load after a free)
    std::map<uint64_t, std::unique_ptr<Pool>> pools;
    std::map<uint64_t, std::deque<std::shared_ptr<Request>>> waiting;
    std::vector<Extraction> extractions;
    int64_t bytes_in_use = 0;
    std::string loop_error;
    bool use_graphs = true;    // replay captured graphs (else launch the kernels directly)
};

namespace {

// Byte offsets of one pool's buffers inside its arena.
struct PoolLayout {
    size_t g, gamma, f, ft0, ft1, e, gf, tp, lp, mom, k, theta, clamps, stage_in, stage_out, total;
};

PoolLayout pool_layout(const appga_matrix *mat) {
    const size_t m = static_cast<size_t>(mat->A.n_rows), d = static_cast<size_t>(mat->A.n_cols);
    PoolLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    L.g = take(4 * m * kLanes);
    L.gamma = take(4 * m * kLanes);
    L.f = take(4 * d * kLanes);
    L.ft0 = take(4 * d * kLanes);
    L.ft1 = take(4 * d * kLanes);
    L.e = take(4 * m * kLanes);
    L.gf = mat->bt.valid ? take(4 * d * kLanes * mat->bt_split) : 0;
    L.tp = mat->ft.valid && mat->ft.n_pslots > 0 ? take(4 * fwd_tile_part_floats(mat->ft, kLanes)) : 0;
    L.lp = take(sizeof(LaneParams) * kLanes);
    L.mom = take(sizeof(double) * 4 * kLanes);
    L.k = take(sizeof(int) * kLanes);
    L.theta = take(sizeof(float) * kLanes);
    L.clamps = take(sizeof(unsigned long long) * kLanes);
    L.stage_in = take(4 * m);
    L.stage_out = take(4 * d);
    L.total = off;
    return L;
}

int64_t pool_bytes(const appga_matrix *mat) { return static_cast<int64_t>(pool_layout(mat).total); }

void destroy_pool(Pool *p) {
    if (!p) return;
    hipStreamSynchronize(p->stream);
    for (auto ev : p->inflight) hipEventDestroy(ev);
    for (auto ev : p->free_events) hipEventDestroy(ev);
    for (auto &st : p->stages) {
        if (st.ev) hipEventDestroy(st.ev);
        if (st.h) hipHostFree(st.h);
    }
    for (auto &gx : p->graph)
        if (gx) hipGraphExecDestroy(gx);
    hipFree(p->arena);
    if (p->h_res) hipHostFree(p->h_res);
    hipStreamDestroy(p->stream);
}

// Enqueues one APPGA iteration of the pool reading f~ from buffer `cur` on the
// pool's stream (per-lane theta, forward + ratio, back projection + update).
hipError_t enqueue_step(Pool *p, int cur) {
    const appga_matrix *mat = p->mat;
    FwdArgs fa{};
    fa.row_ptr = mat->A.row_ptr;
    fa.col = mat->A.col;
    fa.col32 = mat->A.col32;
    fa.nnz_padded = mat->A.nnz_padded;
    fa.val = mat->A.val;
    fa.row_scale = mat->A.row_scale;
    fa.m = mat->A.n_rows;
    fa.n_x = mat->A.n_cols;
    fa.B = kLanes;
    fa.Bp = kLanes;
    fa.x = p->ft[cur];
    fa.g = p->g;
    fa.gamma = p->gamma;
    fa.gamma_lane = nullptr;
    fa.out = p->e;
    fa.mode = FM_RATIO;
    fa.scale_out = 1;
    fa.fwd_wgs = mat->fwd_wgs;
    fa.clamps = p->clamps;
    fa.tile_part = p->tile_part;
    StepArgs sa{};
    sa.row_ptr = mat->AT.row_ptr;
    sa.col = mat->AT.col;
    sa.col32 = mat->AT.col32;
    sa.nnz_padded = mat->AT.nnz_padded;
    sa.val = mat->AT.val;
    sa.row_scale = mat->AT.row_scale;
    sa.n = mat->geom.n;
    sa.m = mat->A.n_rows;
    sa.B = kLanes;
    sa.Bp = kLanes;
    sa.e = p->e;
    sa.ft = p->ft[cur];
    sa.f = p->f;
    sa.ft_next = p->ft[cur ^ 1];
    sa.lam = mat->lam;
    sa.lp = p->lp;
    sa.theta_next = p->theta;
    sa.pbuf = nullptr;
    sa.pmode = PM_EM;
    sa.out_mode = SO_STEP;
    sa.re_part = nullptr;
    sa.tiles_x = (mat->geom.n + 3) / 4;
    sa.xcd_remap = mat->xcd_remap;
    sa.gf_in = p->gf;
    sa.gf_split = mat->bt_split;
    hipError_t e1 = launch_lane_theta(p->lane_k, p->mom, p->theta, p->stream);
    if (e1 == hipSuccess) e1 = launch_forward_mat(mat, fa, p->stream);
    if (e1 == hipSuccess && p->gf)
        e1 = launch_back_tiles(mat->bt, mat->AT.vtype, mat->geom.n, mat->A.n_rows, kLanes, mat->bt_remap,
                               mat->bt_split, p->e, p->gf, p->stream);
    if (e1 == hipSuccess) e1 = launch_step(mat->AT, sa, mat->group_back, p->stream);
    return e1;
}

// Captures enqueue_step(p, cur) into an executable graph.
hipError_t capture_step(Pool *p, int cur, hipGraphExec_t *out) {
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t e1 = enqueue_step(p, cur);
    e = hipStreamEndCapture(p->stream, &graph);
    if (e1 != hipSuccess) return e1;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    return e;
}

appga_status create_pool(appga_server *srv, const appga_matrix *mat, std::unique_ptr<Pool> &out) {
    auto p = std::make_unique<Pool>();
    p->mat = mat;
    const int64_t m = mat->A.n_rows, d = mat->A.n_cols;
    hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(APPGA_E_DEVICE, "stream: %s", hipGetErrorString(e));
    const PoolLayout L = pool_layout(mat);
    e = hipMalloc(&p->arena, L.total);
    if (e != hipSuccess) {
        hipStreamDestroy(p->stream);
        return fail(APPGA_E_OOM, "pool allocation of %zu bytes failed", L.total);
    }
    p->bytes = static_cast<int64_t>(L.total);
    char *base = static_cast<char *>(p->arena);
    p->g = reinterpret_cast<float *>(base + L.g);
    p->gamma = reinterpret_cast<float *>(base + L.gamma);
    p->f = reinterpret_cast<float *>(base + L.f);
    p->ft[0] = reinterpret_cast<float *>(base + L.ft0);
    p->ft[1] = reinterpret_cast<float *>(base + L.ft1);
    p->e = reinterpret_cast<float *>(base + L.e);
    p->gf = mat->bt.valid ? reinterpret_cast<float *>(base + L.gf) : nullptr;
    p->tile_part = mat->ft.valid && mat->ft.n_pslots > 0 ? reinterpret_cast<float *>(base + L.tp) : nullptr;
    p->lp = reinterpret_cast<LaneParams *>(base + L.lp);
    p->mom = reinterpret_cast<double *>(base + L.mom);
    p->lane_k = reinterpret_cast<int *>(base + L.k);
    p->theta = reinterpret_cast<float *>(base + L.theta);
    p->clamps = reinterpret_cast<unsigned long long *>(base + L.clamps);
    p->stage_in = reinterpret_cast<float *>(base + L.stage_in);
    p->stage_out = reinterpret_cast<float *>(base + L.stage_out);
    e = hipSuccess;
    for (auto &st : p->stages) {
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&st.h), sizeof(float) * 2 * m + 256,
                                               hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st.ev, hipEventDisableTiming);
    }
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&p->h_res), sizeof(float) * (d + 4) * kLanes,
                          hipHostMallocDefault);
    if (e == hipSuccess) e = launch_fill(p->g, static_cast<size_t>(m) * kLanes, 0.0f, p->stream);
    // idle lanes: g = 0 with background 1, so A f + gamma never reaches the floor
    // (a floored bin costs an atomic on the lane's counter)
    if (e == hipSuccess) e = launch_fill(p->gamma, static_cast<size_t>(m) * kLanes, 1.0f, p->stream);
    for (float *buf : {p->f, p->ft[0], p->ft[1], p->e})
        if (e == hipSuccess)
            e = launch_fill(buf, static_cast<size_t>(buf == p->e ? m : d) * kLanes, 0.0f, p->stream);
    if (e == hipSuccess) e = launch_fill(p->theta, kLanes, 0.0f, p->stream);
    // idle lanes: no regulariser, beta = 1, eps = 1, no momentum
    std::vector<LaneParams> lp(kLanes, LaneParams{0.f, 0.f, 1.f, 1.f, 0.f, 0.f, 0.f, 0.f});
    std::vector<double> mom(4 * kLanes, 0.0);
    for (int l = 0; l < kLanes; ++l) {
        mom[4 * l] = 0.125;
        mom[4 * l + 1] = 1.0;
        mom[4 * l + 2] = 1.0;
        mom[4 * l + 3] = 1.0;
    }
    std::vector<int> ks(kLanes, 0);
    std::vector<unsigned long long> cl(kLanes, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->lp, lp.data(), sizeof(LaneParams) * kLanes, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->mom, mom.data(), sizeof(double) * 4 * kLanes, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->lane_k, ks.data(), sizeof(int) * kLanes, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->clamps, cl.data(), sizeof(unsigned long long) * kLanes, hipMemcpyHostToDevice,
                           p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess && srv->use_graphs) e = capture_step(p.get(), 0, &p->graph[0]);
    if (e == hipSuccess && srv->use_graphs) e = capture_step(p.get(), 1, &p->graph[1]);
    if (e != hipSuccess) {
        destroy_pool(p.get());
        return fail(APPGA_E_DEVICE, "pool set-up failed: %s", hipGetErrorString(e));
    }
    srv->bytes_in_use += p->bytes;
    out = std::move(p);
    return APPGA_OK;
}

// Places request r into lane l of pool p, in stream order on the pool's
// stream, through the next pinned staging buffer of the ring (no host wait
// unless that buffer's previous copies are still in flight).
hipError_t admit(Pool *p, int l, const std::shared_ptr<Request> &r) {
    const appga_matrix *mat = p->mat;
    const int m = mat->A.n_rows, n = mat->geom.n;
    Stage &st = p->stages[p->next_stage];
    p->next_stage = (p->next_stage + 1) % kStageRing;
    hipError_t e = hipSuccess;
    if (st.used) e = hipEventSynchronize(st.ev);
    if (e != hipSuccess) return e;
    float *hg = st.h, *hgam = st.h + m;
    char *tail = reinterpret_cast<char *>(st.h + 2 * m);
    auto *hlp = reinterpret_cast<LaneParams *>(tail);
    auto *hmom = reinterpret_cast<double *>(tail + 64);
    auto *hk = reinterpret_cast<int *>(tail + 128);
    auto *hcl = reinterpret_cast<unsigned long long *>(tail + 136);
    std::memcpy(hg, r->g.data(), sizeof(float) * m);
    if (!r->gamma.empty()) std::memcpy(hgam, r->gamma.data(), sizeof(float) * m);
    *hlp = LaneParams{static_cast<float>(r->p.lambda1), static_cast<float>(r->p.lambda2),
                      static_cast<float>(r->p.eps), static_cast<float>(r->p.beta),
                      static_cast<float>(r->p.fixed_p), 0.f, 0.f, 0.f};
    hmom[0] = r->p.a;
    hmom[1] = r->p.b;
    hmom[2] = r->p.omega;
    hmom[3] = r->p.momentum == APPGA_MOMENTUM_NONE ? 1.0 : 0.0;
    *hk = 0;
    *hcl = 0;
    // data and background into the lane (the device staging buffer is reused in stream order)
    e = hipMemcpyAsync(p->stage_in, hg, sizeof(float) * m, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = launch_lane_scatter(p->stage_in, p->g, m, l, p->stream);
    if (e == hipSuccess) {
        if (!r->gamma.empty()) {
            e = hipMemcpyAsync(p->stage_in, hgam, sizeof(float) * m, hipMemcpyHostToDevice, p->stream);
            if (e == hipSuccess) e = launch_lane_scatter(p->stage_in, p->gamma, m, l, p->stream);
        } else {
            e = launch_lane_fill(p->gamma, m, l, static_cast<float>(r->p.gamma_scalar), p->stream);
        }
    }
    if (e != hipSuccess) return e;
    // initial image of Section 4.1 (ACTc from the host copy of the data, FP64)
    double actc = 0.0;
    for (int i = 0; i < m; ++i)
        actc += static_cast<double>(r->g[i]) -
                (r->gamma.empty() ? static_cast<double>(static_cast<float>(r->p.gamma_scalar))
                                  : static_cast<double>(r->gamma[i]));
    const double ctr = (n - 1) / 2.0, rad2 = (n / 2.0) * (n / 2.0);
    int64_t npfov = 0;
    for (int rr = 0; rr < n; ++rr)
        for (int cc = 0; cc < n; ++cc) npfov += (cc - ctr) * (cc - ctr) + (rr - ctr) * (rr - ctr) <= rad2;
    const double tmc = actc / (static_cast<double>(npfov) * mat->geom.n_angles);
    e = launch_lane_disk_init(n, l, tmc, p->f, p->ft[p->parity], p->stream);
    // per-lane parameters, iteration counter and clamp counter
    if (e == hipSuccess) e = hipMemcpyAsync(p->lp + l, hlp, sizeof(LaneParams), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->mom + 4 * l, hmom, 4 * sizeof(double), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(p->lane_k + l, hk, sizeof(int), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->clamps + l, hcl, sizeof(unsigned long long), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipEventRecord(st.ev, p->stream);
    if (e != hipSuccess) return e;
    st.used = true;
    p->lane_req[l] = r;
    p->lane_done_iters[l] = 0;
    return hipSuccess;
}

bool pool_active(const Pool *p) {
    for (int l = 0; l < kLanes; ++l)
        if (p->lane_req[l]) return true;
    return false;
}

// A pool may be freed only when no lane is occupied and no result copy reads it.
bool pool_idle(const Pool *p) { return !pool_active(p) && p->pending_out == 0; }

void finish(appga_server *srv, const std::shared_ptr<Request> &r, appga_status st) {
    r->mat->inflight.fetch_sub(1);
    std::lock_guard<std::mutex> lk(srv->mu);
    r->status = st;
    if (st != APPGA_OK) r->error = appga_last_error();
    r->done = true;
    srv->cv_done.notify_all();
}

// One pass of the loop thread; returns true if it did any work.
bool loop_pass(appga_server *srv) {
    bool worked = false;
    // 1. new arrivals into per-matrix queues
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        while (!srv->arrivals.empty()) {
            auto r = srv->arrivals.front();
            srv->arrivals.pop_front();
            srv->waiting[r->mat->serial].push_back(r);
            worked = true;
        }
    }
    // 2. admission: free lanes of existing pools, new pools within the budget
    for (auto &wq : srv->waiting) {
        auto &q = wq.second;
        if (q.empty()) continue;
        const appga_matrix *mat = q.front()->mat;
        auto it = srv->pools.find(wq.first);
        if (it == srv->pools.end()) {
            if (srv->bytes_in_use + pool_bytes(mat) > srv->cfg.hbm_budget_bytes) {
                // make room: free idle pools of other matrices
                for (auto pit = srv->pools.begin(); pit != srv->pools.end();) {
                    if (pool_idle(pit->second.get())) {
                        srv->bytes_in_use -= pit->second->bytes;
                        destroy_pool(pit->second.get());
                        pit = srv->pools.erase(pit);
                    } else {
                        ++pit;
                    }
                }
                if (srv->bytes_in_use + pool_bytes(mat) > srv->cfg.hbm_budget_bytes) continue;
            }
            std::unique_ptr<Pool> np;
            appga_status st = create_pool(srv, mat, np);
            if (st != APPGA_OK) {
                while (!q.empty()) {
                    finish(srv, q.front(), st);
                    q.pop_front();
                }
                continue;
            }
            it = srv->pools.emplace(wq.first, std::move(np)).first;
        }
        Pool *p = it->second.get();
        const int cap = std::max(1, std::min(kLanes, srv->cfg.slots_per_matrix));
        for (int l = 0; l < cap && !q.empty(); ++l) {
            if (p->lane_req[l] || p->lane_out[l]) continue;
            auto r = q.front();
            q.pop_front();
            hipError_t e = admit(p, l, r);
            if (e != hipSuccess) {
                p->lane_req[l].reset();
                finish(srv, r, fail(APPGA_E_DEVICE, "admission failed: %s", hipGetErrorString(e)));
            }
            worked = true;
        }
    }
    // 3. one more step of every pool with occupied lanes and fewer than kDepth
    //    steps in flight (never waits: a busy pool is visited again next pass)
    for (auto &pp : srv->pools) {
        Pool *p = pp.second.get();
        while (!p->inflight.empty() && hipEventQuery(p->inflight.front()) == hipSuccess) {
            p->free_events.push_back(p->inflight.front());
            p->inflight.pop_front();
        }
        if (!pool_active(p) || p->inflight.size() >= static_cast<size_t>(kDepth)) continue;
        hipEvent_t ev = nullptr;
        hipError_t e = hipSuccess;
        if (!p->free_events.empty()) {
            ev = p->free_events.back();
            p->free_events.pop_back();
        } else {
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        }
        if (e == hipSuccess)
            e = p->graph[p->parity] ? hipGraphLaunch(p->graph[p->parity], p->stream) : enqueue_step(p, p->parity);
        if (e == hipSuccess) e = hipEventRecord(ev, p->stream);
        if (e != hipSuccess) {
            if (ev) p->free_events.push_back(ev);
            srv->loop_error = hipGetErrorString(e);
            for (int l = 0; l < kLanes; ++l)
                if (p->lane_req[l]) {
                    finish(srv, p->lane_req[l], fail(APPGA_E_DEVICE, "step failed: %s", srv->loop_error.c_str()));
                    p->lane_req[l].reset();
                }
            continue;
        }
        p->inflight.push_back(ev);
        p->parity ^= 1;
        worked = true;
        // lanes whose budget is done: copy out into the lane's pinned result slot
        const int d = p->mat->A.n_cols;
        for (int l = 0; l < kLanes; ++l) {
            auto &r = p->lane_req[l];
            if (!r) continue;
            if (++p->lane_done_iters[l] < r->p.iterations) continue;
            Extraction x;
            x.req = r;
            x.pool = p;
            x.lane = l;
            x.d = d;
            float *h_out = p->h_res + static_cast<size_t>(l) * (d + 4);
            auto *h_cl = reinterpret_cast<unsigned long long *>(h_out + d + (d & 1));
            hipError_t ee = launch_lane_gather(p->f, p->stage_out, d, l, p->stream);
            if (ee == hipSuccess)
                ee = hipMemcpyAsync(h_out, p->stage_out, sizeof(float) * d, hipMemcpyDeviceToHost, p->stream);
            if (ee == hipSuccess)
                ee = hipMemcpyAsync(h_cl, p->clamps + l, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                    p->stream);
            if (ee == hipSuccess) ee = hipEventCreateWithFlags(&x.ev, hipEventDisableTiming);
            if (ee == hipSuccess) ee = hipEventRecord(x.ev, p->stream);
            if (ee != hipSuccess) {
                if (x.ev) hipEventDestroy(x.ev);
                finish(srv, r, fail(APPGA_E_DEVICE, "result copy failed: %s", hipGetErrorString(ee)));
            } else {
                ++p->pending_out;
                p->lane_out[l] = true;
                srv->extractions.push_back(x);
            }
            r.reset();  // the lane takes a new request once its result is collected
        }
    }
    // 4. completed result copies
    for (size_t i = 0; i < srv->extractions.size();) {
        Extraction &x = srv->extractions[i];
        if (hipEventQuery(x.ev) != hipSuccess) {
            ++i;
            continue;
        }
        const int d = x.d;
        const float *h_out = x.pool->h_res + static_cast<size_t>(x.lane) * (d + 4);
        const auto *h_cl = reinterpret_cast<const unsigned long long *>(h_out + d + (d & 1));
        auto r = x.req;
        r->result.assign(h_out, h_out + d);
        r->stats.iterations_done = r->p.iterations;
        r->stats.objective0 = 0.0;
        r->stats.objective = 0.0;
        r->stats.re = 0.0;
        r->stats.guard_clamps = static_cast<int64_t>(*h_cl);
        r->stats.seconds = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
        bool finite = true;
        for (float v : r->result)
            if (!std::isfinite(v)) finite = false;
        hipEventDestroy(x.ev);
        --x.pool->pending_out;
        x.pool->lane_out[x.lane] = false;
        finish(srv, r, finite ? APPGA_OK : APPGA_E_NONFINITE);
        srv->extractions.erase(srv->extractions.begin() + static_cast<long>(i));
        worked = true;
    }
    return worked;
}

void run_loop(appga_server *srv) {
    hipSetDevice(srv->ctx->device);
    while (true) {
        const bool worked = loop_pass(srv);
        bool busy = !srv->extractions.empty();
        for (auto &pp : srv->pools) busy = busy || pool_active(pp.second.get());
        for (auto &wq : srv->waiting) busy = busy || !wq.second.empty();
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->stopping && !busy && srv->arrivals.empty()) break;
        if (!worked && !busy && srv->arrivals.empty()) {
            srv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        } else if (!worked) {
            // device work in flight and nothing to launch: poll again at once
            lk.unlock();
            std::this_thread::yield();
        }
    }
    for (auto &pp : srv->pools) destroy_pool(pp.second.get());
    srv->pools.clear();
}

}  // namespace

extern "C" appga_status appga_server_footprint(const appga_matrix *mat, int64_t *bytes) {
    clear_error();
    if (!mat || !bytes) return fail(APPGA_E_INVALID_ARG, "NULL matrix or output");
    *bytes = pool_bytes(mat);
    return APPGA_OK;
}

extern "C" appga_status appga_server_start(appga_ctx *ctx, const appga_server_cfg *cfg,
                                           appga_server **out) {
    clear_error();
    if (!ctx || !cfg || !out) return fail(APPGA_E_INVALID_ARG, "NULL ctx, config or output");
    if (cfg->hbm_budget_bytes <= 0 || cfg->slots_per_matrix <= 0)
        return fail(APPGA_E_INVALID_ARG, "budget and slots must be positive");
    auto *srv = new appga_server();
    srv->ctx = ctx;
    srv->cfg = *cfg;
    const char *gs = std::getenv("APPGA_SERVER_GRAPHS");
    srv->use_graphs = !(gs && gs[0] == '0');
    srv->loop = std::thread(run_loop, srv);
    *out = srv;
    return APPGA_OK;
}

extern "C" appga_status appga_submit(appga_server *srv, const appga_matrix *mat, const float *g,
                                     const float *gamma, const appga_params *params,
                                     uint64_t *ticket) {
    clear_error();
    if (!srv || !mat || !g || !params || !ticket) return fail(APPGA_E_INVALID_ARG, "NULL argument");
    if (mat->ctx != srv->ctx) return fail(APPGA_E_INVALID_ARG, "matrix belongs to another context");
    if (mat && mat->psf_R >= 0)
        return fail(APPGA_E_INVALID_ARG, "serving does not model a PSF; use a session for this matrix");
    appga_status st = validate_params(params);
    if (st != APPGA_OK) return st;
    if (params->precond != APPGA_PRECOND_EM)
        return fail(APPGA_E_INVALID_ARG, "the server runs the EM preconditioner only");
    if (params->iterations < 1) return fail(APPGA_E_DOMAIN, "served requests need iterations >= 1");
    if (pool_bytes(mat) > srv->cfg.hbm_budget_bytes)
        return fail(APPGA_E_OOM, "a lane pool for this matrix needs %lld bytes, above the budget of %lld",
                    static_cast<long long>(pool_bytes(mat)), static_cast<long long>(srv->cfg.hbm_budget_bytes));
    const int64_t m = mat->A.n_rows;
    st = validate_data(g, m, "sinogram");
    if (st == APPGA_OK && gamma) st = validate_data(gamma, m, "background");
    if (st != APPGA_OK) return st;
    double actc = 0.0;
    for (int64_t i = 0; i < m; ++i) actc += static_cast<double>(g[i]) - (gamma ? gamma[i] : params->gamma_scalar);
    if (!(actc > 0)) return fail(APPGA_E_DOMAIN, "ACTc = sum(g) - sum(gamma) <= 0");
    auto r = std::make_shared<Request>();
    r->mat = mat;
    r->g.assign(g, g + m);
    if (gamma) r->gamma.assign(gamma, gamma + m);
    r->p = *params;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stopping) return fail(APPGA_E_INVALID_ARG, "server is stopping");
        r->ticket = srv->next_ticket++;
        srv->tickets[r->ticket] = r;
        mat->inflight.fetch_add(1);
        srv->arrivals.push_back(r);
    }
    srv->cv_work.notify_one();
    *ticket = r->ticket;
    return APPGA_OK;
}

extern "C" appga_status appga_wait(appga_server *srv, uint64_t ticket, float *f_out,
                                   appga_stats *stats, int32_t timeout_ms) {
    clear_error();
    if (!srv) return fail(APPGA_E_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(APPGA_E_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    auto r = it->second;
    auto pred = [&] { return r->done; };
    if (timeout_ms < 0)
        srv->cv_done.wait(lk, pred);
    else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
        return fail(APPGA_E_TIMEOUT, "ticket %llu not done", (unsigned long long)ticket);
    srv->tickets.erase(it);
    if (r->status != APPGA_OK && r->status != APPGA_E_NONFINITE)
        return fail(r->status, "ticket %llu: %s", (unsigned long long)ticket, r->error.c_str());
    if (f_out) std::memcpy(f_out, r->result.data(), sizeof(float) * r->result.size());
    if (stats) *stats = r->stats;
    return r->status == APPGA_OK ? APPGA_OK : fail(APPGA_E_NONFINITE, "non-finite result");
}

extern "C" appga_status appga_server_stop(appga_server *srv) {
    clear_error();
    if (!srv) return fail(APPGA_E_INVALID_ARG, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    if (srv->loop.joinable()) srv->loop.join();
    delete srv;
    return APPGA_OK;
}
