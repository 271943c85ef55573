// Batched solves: many independent problems of uneven sizes, replayed from
// captured hipGraphs.
//
// Every problem is planned on its own (tables, FP64 column set, workspace:
// the planning done once and reused every timestep, paper Section 2.1, with
// the per-problem reusable buffers of its uneven-decomposition plan), so a
// batched solve runs exactly the kernels a standalone solve of that problem
// runs and gives the same result bit for bit.
//
// Mode PS_BATCH_LANES: the problems are dealt to a few lanes, largest first,
// each to the lane with the fewest points so far (LPT).  Each lane has its
// own stream; the solves of a lane's problems are captured one after another
// into one graph on that stream, with the stream as the capture's origin.
// By default each plan's FP64 columns run in order on the lane (placement 0
// of the plan), so a lane's graph is one chain on one stream; otherwise each
// plan keeps its own placement and its FP64 columns fork onto the plan's
// second stream and join back inside the capture.  The in-order form is the
// faster one for the uneven batch: the plans' second streams share the
// device's few hardware queues with the lanes, so their forks tie the lanes'
// progress together, while the lanes themselves already overlap one
// problem's FP64 columns with other problems' passes.  A batched solve forks
// the lanes from the caller's stream, launches every lane's graph on its
// stream and joins them back, so problems of different lanes run side by
// side and the small problems fill the gaps the large ones leave.  Before the
// first capture every plan solves once eagerly on the stream it will be
// captured on, so no kernel is first launched inside a capture.
//
// Earlier forms, refused by ps_batch_set_mode (their code is removed):
//   PS_BATCH_PERSISTENT: one persistent launch whose blocks took (problem,
//     phase, tile) tickets and waited per problem for the previous phase.
//     After a fix of an out-of-bounds coefficient read it still did not
//     complete on the GPU; the cause was not found.
//   PS_BATCH_PHASES: one kernel per phase over the tiles of every problem,
//     sharing the persistent kernel's tile work list; never run.
//   PS_BATCH_PLANS: every plan's solve captured into ONE graph, the plans'
//     streams being lanes forked from the capture's origin; its first run
//     ended in a host segmentation fault during that capture.  It was the
//     only capture in which a plan's own stream was itself a forked capture
//     stream (the plan's stream then waits on events its second stream
//     recorded); the lanes mode never does that.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "ps_internal.h"
#include "ps_plan_impl.h"
#include "../../include/pressure_solve.h"

namespace {

constexpr int kMaxLanes = 8;
constexpr int kDefaultLanes = 4;

} // namespace

struct ps_batch {
    int count = 0, precision = 0;
    hipStream_t stream = nullptr;           // caller's stream
    std::vector<ps_plan *> plans;
    std::vector<long long> points;          // nx ny nz per problem
    std::vector<int> order;                 // problems, most points first
    std::vector<int> lane_of;               // problem -> lane
    int nlanes = kDefaultLanes;
    hipStream_t lanes[kMaxLanes] = {};
    hipEvent_t ev_in = nullptr, ev_join[kMaxLanes] = {};
    hipGraphExec_t exec[kMaxLanes] = {};    // one graph per lane (null: empty lane)
    int fp64_in_order = 1;                  // FP64 columns in order on the lanes
    std::vector<int> tuned_side;            // each plan's own FP64-column placement
    bool captured = false;
    std::vector<const void *> cap_rhs;
    std::vector<void *> cap_out;
};

static int bfail(int code, const std::string &msg) { return ps::set_error(code, msg); }

#define PS_BHIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return bfail(PS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

static void destroy_graphs(ps_batch *b)
{
    for (int l = 0; l < kMaxLanes; ++l) {
        if (b->exec[l]) (void)hipGraphExecDestroy(b->exec[l]);
        b->exec[l] = nullptr;
    }
    b->captured = false;
}

static void free_batch(ps_batch *b)
{
    destroy_graphs(b);
    for (ps_plan *p : b->plans) ps_plan_destroy(p);
    for (int l = 0; l < kMaxLanes; ++l) {
        if (b->lanes[l]) (void)hipStreamDestroy(b->lanes[l]);
        if (b->ev_join[l]) (void)hipEventDestroy(b->ev_join[l]);
    }
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    delete b;
}

// Waits for everything the batch has enqueued on its own streams.
static int sync_lanes(ps_batch *b)
{
    for (int l = 0; l < kMaxLanes; ++l)
        if (b->lanes[l]) PS_BHIP(hipStreamSynchronize(b->lanes[l]));
    return PS_OK;
}

// LPT assignment: problems most points first, each to the lane with the
// fewest points so far (ties: the lower lane).
static void assign_lanes(ps_batch *b)
{
    std::vector<long long> load(b->nlanes, 0);
    b->lane_of.assign(b->count, 0);
    for (int i : b->order) {
        int best = 0;
        for (int l = 1; l < b->nlanes; ++l)
            if (load[l] < load[best]) best = l;
        b->lane_of[i] = best;
        load[best] += b->points[i];
    }
}

extern "C" int ps_batch_create(ps_batch **out, int count, const int *nx, const int *ny,
                               const int *nz, const double *dx, const double *dy,
                               const double *const *dz, const double *const *rho, int precision,
                               void *stream)
{
    if (!out) return bfail(PS_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (count < 1 || !nx || !ny || !nz || !dx || !dy || !dz || !rho)
        return bfail(PS_EINVAL, "count >= 1 and all arrays required");
    if (precision < PS_FP64 || precision > PS_FP32_R1)
        return bfail(PS_EUNSUPPORTED, "unknown precision");
    for (int i = 0; i < count; ++i)
        if (!dz[i] || !rho[i]) return bfail(PS_EINVAL, "dz[i] and rho[i] required");
    ps_batch *b = new ps_batch();
    b->count = count;
    b->precision = precision;
    b->stream = reinterpret_cast<hipStream_t>(stream);
    auto bail = [&](int rc) {
        free_batch(b);
        return rc;
    };
    for (int l = 0; l < kMaxLanes; ++l)
        if (hipStreamCreateWithFlags(&b->lanes[l], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->ev_join[l], ps::kStreamEventFlags) != hipSuccess)
            return bail(bfail(PS_EHIP, "stream or event creation failed"));
    if (hipEventCreateWithFlags(&b->ev_in, ps::kStreamEventFlags) != hipSuccess)
        return bail(bfail(PS_EHIP, "event creation failed"));
    b->plans.assign(count, nullptr);
    b->points.assign(count, 0);
    for (int i = 0; i < count; ++i) {
        // planned on a lane stream (not the null stream); ps_batch_solve
        // moves each plan to its lane before it is used
        const int rc = ps_plan_create(&b->plans[i], nx[i], ny[i], nz[i], dx[i], dy[i], dz[i],
                                      rho[i], precision, 0.0, b->lanes[0]);
        if (rc != PS_OK) {
            ps::set_error(rc, std::string("problem ") + std::to_string(i) + ": " + ps_last_error());
            return bail(rc);
        }
        b->points[i] = (long long)nx[i] * ny[i] * nz[i];
        b->tuned_side.push_back(b->plans[i]->geom.special_side);
    }

    b->order.resize(count);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int a, int c) { return b->points[a] > b->points[c]; });
    assign_lanes(b);
    *out = b;
    return PS_OK;
}

// Captures one graph per lane (see the file comment).  On error no graph is
// kept and every capture that was begun has been ended.
static int capture_lanes(ps_batch *b, const void *const *rhs, void *const *p)
{
    destroy_graphs(b);
    assign_lanes(b);
    for (int i = 0; i < b->count; ++i)
        b->plans[i]->geom.special_side = b->fp64_in_order ? 0 : b->tuned_side[i];
    // eager pass: each plan's kernels run once, outside any capture, on the
    // stream the plan is captured on
    for (int i : b->order) {
        int rc = ps_plan_set_stream(b->plans[i], b->lanes[b->lane_of[i]]);
        if (rc == PS_OK) rc = ps_solve(b->plans[i], rhs[i], p[i]);
        if (rc != PS_OK)
            return ps::set_error(rc, std::string("problem ") + std::to_string(i) + ": " +
                                         ps_last_error());
    }
    {
        const int rc = sync_lanes(b);
        if (rc != PS_OK) return rc;
    }
    for (int l = 0; l < b->nlanes; ++l) {
        bool any = false;
        for (int i : b->order) any = any || b->lane_of[i] == l;
        if (!any) continue;
        PS_BHIP(hipStreamBeginCapture(b->lanes[l], hipStreamCaptureModeThreadLocal));
        int rc = PS_OK;
        for (int i : b->order) {
            if (b->lane_of[i] != l || rc != PS_OK) continue;
            rc = ps_solve(b->plans[i], rhs[i], p[i]);
            if (rc != PS_OK)
                ps::set_error(rc, std::string("problem ") + std::to_string(i) + ": " +
                                      ps_last_error());
        }
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(b->lanes[l], &g);
        if (rc != PS_OK || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            destroy_graphs(b);
            if (rc != PS_OK) return rc;
            return bfail(PS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
        }
        const hipError_t ie = hipGraphInstantiate(&b->exec[l], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            b->exec[l] = nullptr;
            destroy_graphs(b);
            return bfail(PS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        }
    }
    b->cap_rhs.assign(rhs, rhs + b->count);
    b->cap_out.assign(p, p + b->count);
    b->captured = true;
    return PS_OK;
}

extern "C" int ps_batch_solve(ps_batch *b, const void *const *rhs, void *const *p)
{
    if (!b || !rhs || !p) return bfail(PS_EINVAL, "batch, rhs and p must not be NULL");
    for (int i = 0; i < b->count; ++i) {
        if (!rhs[i] || !p[i]) return bfail(PS_EINVAL, "rhs[i] and p[i] must not be NULL");
        if (b->precision == PS_FP32_R1 && rhs[i] == p[i])
            return bfail(PS_EINVAL, "rhs[i] and p[i] must not alias in the PS_FP32_R1 form");
    }
    bool same = b->captured;
    for (int i = 0; same && i < b->count; ++i)
        same = b->cap_rhs[i] == rhs[i] && b->cap_out[i] == p[i];
    if (!same) {
        // the caller's earlier work (which may produce rhs) and any replay
        // still using the old graphs must be complete before the eager pass
        PS_BHIP(hipStreamSynchronize(b->stream));
        int rc = sync_lanes(b);
        if (rc == PS_OK) rc = capture_lanes(b, rhs, p);
        if (rc != PS_OK) return rc;
    }
    // fork the lanes from the caller's stream, replay, join back
    PS_BHIP(hipEventRecord(b->ev_in, b->stream));
    for (int l = 0; l < b->nlanes; ++l) {
        if (!b->exec[l]) continue;
        PS_BHIP(hipStreamWaitEvent(b->lanes[l], b->ev_in, 0));
        PS_BHIP(hipGraphLaunch(b->exec[l], b->lanes[l]));
        PS_BHIP(hipEventRecord(b->ev_join[l], b->lanes[l]));
        PS_BHIP(hipStreamWaitEvent(b->stream, b->ev_join[l], 0));
    }
    return PS_OK;
}

extern "C" int ps_batch_set_mode(ps_batch *b, int mode)
{
    if (!b) return bfail(PS_EINVAL, "batch is NULL");
    switch (mode) {
    case PS_BATCH_LANES: return PS_OK;
    case PS_BATCH_PERSISTENT:
        return bfail(PS_EUNSUPPORTED, "the single persistent launch is withdrawn: it did not "
                                      "complete on the GPU and its cause was not found");
    case PS_BATCH_PHASES:
        return bfail(PS_EUNSUPPORTED, "the per-phase tile launches are withdrawn with the "
                                      "persistent launch whose work list they shared");
    case PS_BATCH_PLANS:
        return bfail(PS_EUNSUPPORTED, "the single-graph capture over forked plan streams is "
                                      "withdrawn after a host fault during its capture; use "
                                      "PS_BATCH_LANES");
    default: return bfail(PS_EINVAL, "unknown batch mode");
    }
}

extern "C" int ps_batch_set_lanes(ps_batch *b, int lanes)
{
    if (!b) return bfail(PS_EINVAL, "batch is NULL");
    if (lanes < 1 || lanes > kMaxLanes) return bfail(PS_EINVAL, "lanes must be in [1, 8]");
    if (lanes == b->nlanes) return PS_OK;
    // a replay may still run the old graphs
    PS_BHIP(hipStreamSynchronize(b->stream));
    const int rc = sync_lanes(b);
    if (rc != PS_OK) return rc;
    destroy_graphs(b);
    b->nlanes = lanes;
    assign_lanes(b);
    return PS_OK;
}

extern "C" int ps_batch_set_fp64_order(ps_batch *b, int in_order)
{
    if (!b) return bfail(PS_EINVAL, "batch is NULL");
    if (in_order != 0 && in_order != 1) return bfail(PS_EINVAL, "in_order must be 0 or 1");
    if (in_order == b->fp64_in_order) return PS_OK;
    // a replay may still run the old graphs
    PS_BHIP(hipStreamSynchronize(b->stream));
    const int rc = sync_lanes(b);
    if (rc != PS_OK) return rc;
    destroy_graphs(b);
    b->fp64_in_order = in_order;
    return PS_OK;
}

extern "C" int ps_batch_set_stream(ps_batch *b, void *stream)
{
    if (!b) return bfail(PS_EINVAL, "batch is NULL");
    b->stream = reinterpret_cast<hipStream_t>(stream);
    return PS_OK;
}

// Each problem's plan times its own kernel variants (ps_plan_autotune;
// equal shapes share the choice through the tune cache), then every lane
// count 1, 2, 4, 8 with the FP64 columns in order on the lanes and with each
// plan's own placement is timed over reps replays on the given fields, and
// the fastest pair is kept.  The graphs are captured again on the next solve.
extern "C" int ps_batch_autotune(ps_batch *b, const void *const *rhs, void *const *p, int reps)
{
    if (!b || !rhs || !p) return bfail(PS_EINVAL, "batch, rhs and p must not be NULL");
    if (reps < 1) reps = 1;
    if (reps > 100) reps = 100;
    PS_BHIP(hipStreamSynchronize(b->stream));
    int rc = sync_lanes(b);
    if (rc != PS_OK) return rc;
    destroy_graphs(b);
    for (int i : b->order) {
        rc = ps_plan_set_stream(b->plans[i], b->lanes[0]);
        if (rc == PS_OK) rc = ps_plan_autotune(b->plans[i], reps);
        if (rc == PS_OK) b->tuned_side[i] = b->plans[i]->geom.special_side;
        if (rc != PS_OK)
            return ps::set_error(rc, std::string("problem ") + std::to_string(i) + ": " +
                                         ps_last_error());
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PS_BHIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(PS_EHIP, "event creation failed");
    }
    int best = b->nlanes, best_order = b->fp64_in_order;
    float best_ms = 1e30f;
    for (int order : {1, 0}) {
        for (int lanes : {1, 2, 4, 8}) {
            if (lanes > b->count && lanes > 1) break;
            rc = ps_batch_set_fp64_order(b, order);
            if (rc == PS_OK) rc = ps_batch_set_lanes(b, lanes);
            if (rc == PS_OK) rc = ps_batch_solve(b, rhs, p); // capture + one replay
            if (rc != PS_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e0, b->stream) != hipSuccess)
                rc = bfail(PS_EHIP, "autotune timing");
            for (int r = 0; r < reps && rc == PS_OK; ++r) rc = ps_batch_solve(b, rhs, p);
            if (rc == PS_OK && (hipEventRecord(e1, b->stream) != hipSuccess ||
                                hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = bfail(PS_EHIP, "autotune timing");
            if (rc != PS_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = lanes;
                best_order = order;
            }
        }
        if (rc != PS_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PS_OK) return rc;
    rc = ps_batch_set_fp64_order(b, best_order);
    if (rc != PS_OK) return rc;
    return ps_batch_set_lanes(b, best);
}

extern "C" int ps_batch_query(const ps_batch *b, int *count, int *lanes, int *fp64_in_order)
{
    if (!b) return bfail(PS_EINVAL, "batch is NULL");
    if (count) *count = b->count;
    if (lanes) *lanes = b->nlanes;
    if (fp64_in_order) *fp64_in_order = b->fp64_in_order;
    return PS_OK;
}

// Synchronises the caller's stream (which the replay joins) and the lanes.
extern "C" int ps_batch_status(ps_batch *b)
{
    if (!b) return bfail(PS_EINVAL, "batch is NULL");
    PS_BHIP(hipStreamSynchronize(b->stream));
    return sync_lanes(b);
}

extern "C" int ps_batch_destroy(ps_batch *b)
{
    if (!b) return PS_OK;
    (void)hipStreamSynchronize(b->stream);
    (void)sync_lanes(b);
    free_batch(b);
    return PS_OK;
}
