// Host runtime of libtpasym: argument validation, launch plans, per-stream
// workspaces, HIP-graph capture and replay, the autotuner, and the host-only
// reductions (asymmetries of eq. (5)-(6) and the T-odd quantities; S_CP of eq. (1)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/tpasym.h"
#include "tp_kernel.h"
#include "tp_noalloc.h"

namespace tpk {
hipError_t launch_pass(int dtype, int prec, int mode, int epl, int k0, int k1, bool ord, const KParams &kp, int grid,
                       int block, size_t lds, hipStream_t st);
hipError_t launch_exact(int dtype, int mode, const KParams &kp, int grid, hipStream_t st);
hipError_t launch_probe(const KSample &k, float *det32, float *bound32, double *det64, double *scale64,
                        hipStream_t st);
}  // namespace tpk

using namespace tpk;

#include "tp_energy.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define TP_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(TP_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

// The exact-tier list holds one entry per event of a launch (the plan's
// virtual events, at most 2^31), so it cannot overflow: every event the pass
// defers is decided by the later tiers.
constexpr uint64_t XCAP_MIN = 1u << 16;
constexpr uint64_t XCAP_MAX = 1ull << 31;
constexpr int EXACT_GRID = 128;

// Workgroups of the exact-tier launch (64 threads each, one listed event per
// thread and pass over the list): more for larger launches, whose lists are
// longer.
int exact_grid(int64_t vtotal)
{
    return (int)std::min<int64_t>(EXACT_GRID, std::max<int64_t>(16, vtotal >> 16));
}
constexpr size_t MAX_PLANS = 256;        // launch plans kept per device
constexpr size_t LDS_LIMIT = 64 * 1024;

uint64_t fnv(const void *p, size_t n, uint64_t h = 1469598103934665603ull)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct Workspace {
    void *buf = nullptr;   // xlist | xcount | xdone
    uint64_t *xlist = nullptr;
    uint32_t *xcount = nullptr;
    uint32_t *xdone = nullptr;
    uint64_t cap = 0;      // list entries
};

// List capacity for a launch over ``vtotal`` virtual events.
uint64_t list_capacity(int64_t vtotal)
{
    return std::min<uint64_t>(std::max<uint64_t>((uint64_t)vtotal, XCAP_MIN), XCAP_MAX);
}

// Samples of one binning scheme (and of one kind as to identical-particle
// ordering): contiguous in the plan's sample table and in the virtual event
// space; one pass launch each.
struct Group {
    int k0 = AX_NONE, k1 = AX_NONE;
    bool ord = false;
    int sbeg = 0, send = 0;
    int64_t vbeg = 0, vend = 0;
    int hist_stride = 0;
    int edge_doubles = 0;
};

struct Plan {
    std::vector<KSample> hs;
    std::vector<double> hedges;
    std::vector<Group> groups;
    int64_t vtotal = 0;
    int dtype = 0;
    void *dbuf = nullptr;        // device: samples | edges
    void *pinned = nullptr;      // host copy source
    hipEvent_t ready = nullptr;
    hipStream_t made_on = nullptr;
    KSample *dsamples = nullptr;
    double *dedges = nullptr;
    // the latest enqueued work that reads the plan (a use on another stream
    // first waits for it, so this event covers every earlier use)
    hipEvent_t last_use = nullptr;
    hipStream_t last_stream = nullptr;
    bool used = false;
    std::list<uint64_t>::iterator lru_pos;
    std::vector<uint64_t> graph_keys;   // graphs captured with this plan's tables
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    Workspace ws;
};

struct TimingState {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ring;
    size_t next = 0, used = 0;
};

struct Device {
    int cus = 256;
    std::map<hipStream_t, Workspace> ws;
    std::unordered_map<uint64_t, Plan *> plans;
    std::list<uint64_t> lru;
    std::unordered_map<uint64_t, GraphEntry> graphs;
    std::map<std::string, tp_tuning> tuned;
    bool tune_loaded = false;             // TP_TUNE_CACHE read into ``tuned``
    uint64_t *scratch_counts = nullptr;   // autotune sink
    size_t scratch_words = 0;
    std::map<hipStream_t, uint32_t *> eflag;   // pair sums per stream: range flag, workgroup count
    // scheme groups of one launch run on parallel branches: the caller's
    // stream and up to NSIDE side streams (default priority), forked from and
    // joined back into the caller's stream by events
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
};

constexpr int NSIDE = 3;
// Workgroups per CU, at most, of a scheme group running beside the largest
// (batched 64-sample workload: 1.284 against 1.299 ms per step uncapped, 1.286
// with 2; same box, three rounds each).
constexpr int SIDE_WG_PER_CU = 4;
// Workgroups per CU of the largest scheme group when others run beside it.
// Each pass kernel holds 4 waves per SIMD, so a CU runs 4 of the launches'
// workgroups at a time; the largest group's workgroups that find a free CU only
// when a side launch drains still have their whole range to process, and the
// step ends with them.  Finer ranges shorten that tail (batched 64-sample
// workload: 16 against the tuned 8, 1.268 against 1.295 ms per step on one box
// and 1.295 against 1.307 on another, three rounds each; 24 or 32 no better).
constexpr int LARGEST_WG_PER_CU = 16;

std::mutex g_mu;
std::map<int, Device> g_dev;
TimingState g_timing;

Device &device(int id)
{
    auto it = g_dev.find(id);
    if (it != g_dev.end()) return it->second;
    Device &d = g_dev[id];
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, id) == hipSuccess && v > 0)
        d.cus = v;
    return d;
}

// A deferral workspace of ``cap`` list entries; its counters are cleared on ``st``.
int new_workspace(uint64_t cap, hipStream_t st, Workspace &w)
{
    const size_t bytes = cap * sizeof(uint64_t) + 64;
    if (hipMalloc(&w.buf, bytes) != hipSuccess) return fail(TP_ENOMEM, "workspace allocation failed");
    w.cap = cap;
    w.xlist = static_cast<uint64_t *>(w.buf);
    w.xcount = reinterpret_cast<uint32_t *>(static_cast<char *>(w.buf) + cap * sizeof(uint64_t));
    w.xdone = w.xcount + 1;
    TP_HIP(hipMemsetAsync(w.xcount, 0, 64, st));
    return TP_OK;
}

// The stream's workspace, grown (after the stream's earlier work) to ``cap`` entries.
int get_workspace(Device &d, hipStream_t st, uint64_t cap, Workspace &out)
{
    auto it = d.ws.find(st);
    if (it != d.ws.end() && it->second.cap >= cap) {
        out = it->second;
        return TP_OK;
    }
    if (it != d.ws.end()) {
        TP_HIP(hipStreamSynchronize(st));
        hipFree(it->second.buf);
        d.ws.erase(it);
    }
    Workspace w;
    const int rc = new_workspace(cap, st, w);
    if (rc) return rc;
    d.ws[st] = w;
    out = w;
    return TP_OK;
}

// ------------------------------------------------------------------ validation
int perm_sign(const int *p, int n)
{
    int s = 1;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (p[i] > p[j]) s = -s;
    return s;
}

int check_events(const tp_events *ev, int precision)
{
    if (!ev) return fail(TP_EINVAL, "events is NULL");
    if (ev->n < 0) return fail(TP_EINVAL, "n < 0");
    if (ev->n >= (int64_t(1) << 40)) return fail(TP_ERANGE, "n >= 2^40 events in one sample");
    if (ev->dtype != TP_F32 && ev->dtype != TP_F64) return fail(TP_EINVAL, "dtype must be TP_F32 or TP_F64");
    if (precision != TP_PREC_F64 && precision != TP_PREC_F32_RECHECK)
        return fail(TP_EINVAL, "unknown precision");
    if (precision == TP_PREC_F32_RECHECK && ev->dtype != TP_F32)
        return fail(TP_EUNSUPPORTED, "TP_PREC_F32_RECHECK needs float32 storage");
    if (ev->n > 0) {
        for (int s = 0; s < 4; ++s)
            for (int c = 0; c < 4; ++c)
                if (!ev->p[s][c]) return fail(TP_EINVAL, "component pointer is NULL");
        if (!ev->tag) return fail(TP_EINVAL, "tag pointer is NULL");
    }
    return TP_OK;
}

int check_channel(const tp_channel *ch)
{
    if (!ch) return fail(TP_EINVAL, "channel is NULL");
    for (int k = 0; k < 3; ++k)
        if (ch->triple[k] < 0 || ch->triple[k] > 3) return fail(TP_EINVAL, "triple slot out of 0..3");
    if (ch->triple[0] == ch->triple[1] || ch->triple[0] == ch->triple[2] || ch->triple[1] == ch->triple[2])
        return fail(TP_EINVAL, "triple slots must be distinct");
    int seen = 0;
    for (int k = 0; k < 4; ++k) {
        if (ch->planes[k] < 0 || ch->planes[k] > 3) return fail(TP_EINVAL, "plane slot out of 0..3");
        seen |= 1 << ch->planes[k];
    }
    if (seen != 15) return fail(TP_EINVAL, "planes must be a permutation of 0..3");
    const int f = ch->identical[0], sl = ch->identical[1];
    if (!(f == -1 && sl == -1)) {
        if (f < 0 || f > 3 || sl < 0 || sl > 3 || f == sl)
            return fail(TP_EINVAL, "identical slots must be two distinct slots of 0..3, or both -1");
    }
    return TP_OK;
}

bool has_axis(const tp_binning *bn, int kind)
{
    if (bn)
        for (int a = 0; a < bn->naxes; ++a)
            if (bn->axis[a].kind == kind) return true;
    return false;
}

// Identical particles need kernel slots {0, 2} or {1, 3} (positions of planes
// up to the XOR relabelling).  With a plane angle binned the planes fix the
// order; without one any order serves, and the pair is placed at positions 1, 3.
int check_identical(const tp_channel *ch, const tp_binning *bn)
{
    const int f = ch->identical[0], sl = ch->identical[1];
    if (f < 0 || !has_axis(bn, TP_AXIS_ABSPHI)) return TP_OK;
    int pf = 0, ps = 0;
    for (int t = 0; t < 4; ++t) {
        if (ch->planes[t] == f) pf = t;
        if (ch->planes[t] == sl) ps = t;
    }
    if ((pf ^ ps) != 2)
        return fail(TP_EUNSUPPORTED, "with a plane angle binned, the identical slots must sit at positions "
                                     "(0, 2) or (1, 3) of planes");
    return TP_OK;
}

int check_binning(const tp_binning *bn)
{
    if (!bn) return fail(TP_EINVAL, "binning is NULL");
    if (bn->naxes < 0 || bn->naxes > 2) return fail(TP_EINVAL, "naxes must be 0, 1 or 2");
    int64_t tot = 1;
    int nphi = 0;
    for (int a = 0; a < bn->naxes; ++a) {
        const tp_axis &ax = bn->axis[a];
        if (ax.nbins < 1 || ax.nbins > MAXBINS) return fail(TP_EINVAL, "nbins must be in 1..1024");
        if (!ax.edges) return fail(TP_EINVAL, "edges pointer is NULL");
        tot *= ax.nbins;
        for (int k = 0; k <= ax.nbins; ++k)
            if (!std::isfinite(ax.edges[k])) return fail(TP_EINVAL, "edges must be finite");
        if (ax.kind == TP_AXIS_ABSPHI) {
            ++nphi;
            if (ax.edges[0] != 1.0 || ax.edges[ax.nbins] != -1.0)
                return fail(TP_EINVAL, "ABSPHI edges must run from cos 0 = 1 down to cos pi = -1");
            for (int k = 0; k < ax.nbins; ++k)
                if (!(ax.edges[k] > ax.edges[k + 1])) return fail(TP_EINVAL, "ABSPHI edges must decrease");
        } else if (ax.kind == TP_AXIS_MASS) {
            if (__builtin_popcount((unsigned)ax.slots & 15u) < 2 || (ax.slots & ~15))
                return fail(TP_EINVAL, "MASS slots must be a bit mask of at least two of slots 0..3");
            if (!(ax.edges[0] >= 0.0)) return fail(TP_EINVAL, "MASS edges must be >= 0");
            for (int k = 0; k < ax.nbins; ++k)
                if (!(ax.edges[k] < ax.edges[k + 1])) return fail(TP_EINVAL, "MASS edges must increase");
            if (ax.edges[ax.nbins] > 1e150) return fail(TP_EINVAL, "MASS edges too large");
        } else if (ax.kind == TP_AXIS_ABSCOS) {
            if (ax.slots < 0 || ax.slots > 3) return fail(TP_EINVAL, "ABSCOS slot out of 0..3");
            if (ax.edges[0] != 0.0 || ax.edges[ax.nbins] != 1.0)
                return fail(TP_EINVAL, "ABSCOS edges must run from 0 to 1");
            for (int k = 0; k < ax.nbins; ++k)
                if (!(ax.edges[k] < ax.edges[k + 1])) return fail(TP_EINVAL, "ABSCOS edges must increase");
        } else {
            return fail(TP_EINVAL, "unknown axis kind");
        }
    }
    if (nphi > 1) return fail(TP_EINVAL, "at most one ABSPHI axis");
    if (tot > MAXBINS) return fail(TP_ERANGE, "more than 1024 bins in total");
    return TP_OK;
}

// e^2 bracketed by two doubles: lo <= e^2 <= hi (exact: the FMA residual tells the side)
void square_bounds(double e, double &lo, double &hi)
{
    const double p = e * e;
    if (p < 0x1p-969) {
        // below 2^-969 the residual e*e - p need not be representable; the
        // rounded square is within half an ulp, so its two neighbours bracket e^2
        lo = std::fmax(std::nextafter(p, -INFINITY), 0.0);
        hi = std::nextafter(p, INFINITY);
        return;
    }
    const double r = std::fma(e, e, -p);
    if (r > 0) {
        lo = p;
        hi = std::nextafter(p, INFINITY);
    } else if (r < 0) {
        lo = std::nextafter(p, -INFINITY);
        hi = p;
    } else {
        lo = hi = p;
    }
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Edge data of one launch in a fixed host array (no heap allocation).
struct FixedEdges {
    double v[NA_EDGES];
    int n = 0;
    bool overflow = false;
    size_t size() const { return (size_t)n; }
    void push_back(double x)
    {
        if (n < NA_EDGES) v[n++] = x;
        else overflow = true;
    }
};

// Fill one KSample (kernel order = channel planes); its edge data is appended
// to ``edges`` (std::vector<double> or FixedEdges).
template <class Edges>
void fill_sample(KSample &k, const tp_events &ev, const tp_channel &ch, const tp_binning *bn,
                 uint64_t *counts, tp_stats *stats, int8_t *cls_out, double *ct_out, Edges &edges)
{
    std::memset(&k, 0, sizeof k);
    // Identical particles without a binned plane angle: any kernel order is
    // valid (sigma follows it), so the planes are replaced by an order that
    // puts the pair at positions 1 and 3.
    int planes[4] = { ch.planes[0], ch.planes[1], ch.planes[2], ch.planes[3] };
    const int idf = ch.identical[0], ids = ch.identical[1];
    if (idf >= 0 && !has_axis(bn, TP_AXIS_ABSPHI)) {
        int o[2], no = 0;
        for (int s = 0; s < 4; ++s)
            if (s != idf && s != ids) o[no++] = s;
        planes[0] = o[0];
        planes[1] = idf;
        planes[2] = o[1];
        planes[3] = ids;
    }
    // Kernel order: kernel slot t holds channel slot planes[t ^ r].  The XOR
    // relabelling t -> t ^ r is the identity or a product of two transpositions
    // ((01)(23), (02)(13), (03)(12)): an even permutation that maps the plane
    // pair {(0,1), (2,3)} onto itself with the orientation of both normals
    // reversed together or swapped, so the triple-product sign and cos Phi are
    // unchanged.  r moves the slot of the first |cos theta| axis to kernel
    // slot 0, which the kernel then reads at a fixed position.
    int r = 0;
    if (bn)
        for (int a = 0; a < bn->naxes; ++a)
            if (bn->axis[a].kind == TP_AXIS_ABSCOS) {
                for (int t = 0; t < 4; ++t)
                    if (planes[t] == bn->axis[a].slots) r = t;
                break;
            }
    int inv[4];
    for (int t = 0; t < 4; ++t) inv[planes[t ^ r]] = t;   // channel slot -> kernel slot
    bool vec = true;
    for (int t = 0; t < 4; ++t)
        for (int c = 0; c < 4; ++c) {
            k.p[t * 4 + c] = ev.p[planes[t ^ r]][c];
            vec = vec && aligned16(ev.p[planes[t ^ r]][c]);
        }
    k.tag = ev.tag;
    vec = vec && ((reinterpret_cast<uintptr_t>(ev.tag) & 3u) == 0);
    k.vec = vec ? 1 : 0;
    k.n = ev.n;
    k.counts = counts;
    k.stats = reinterpret_cast<uint64_t *>(stats);
    k.cls_out = cls_out;
    k.ct_out = ct_out;
    // sigma: C_T^inv = det[p_D; p_A; p_B; p_C] = sgn(D,A,B,C) det[p0..p3]
    //        det[kernel rows] = sgn(planes) det[p0..p3] (the relabelling is even)
    int D = 0 + 1 + 2 + 3 - ch.triple[0] - ch.triple[1] - ch.triple[2];
    int dabc[4] = { D, ch.triple[0], ch.triple[1], ch.triple[2] };
    k.sigma = perm_sign(dabc, 4) * perm_sign(planes, 4);
    // identical pair: kernel slots inv[f], inv[s] are {0, 2} or {1, 3}
    k.olo = -1;
    k.odir = 1;
    if (idf >= 0) {
        const int kf = inv[idf], ks = inv[ids];
        k.olo = kf < ks ? kf : ks;
        k.odir = kf == k.olo ? 1 : -1;
    }
    k.naxes = bn ? bn->naxes : 0;
    k.kind[0] = k.kind[1] = AX_NONE;
    k.nbtot = 0;
    if (bn && bn->naxes > 0) {
        k.nbtot = 1;
        for (int a = 0; a < bn->naxes; ++a) {
            const tp_axis &ax = bn->axis[a];
            k.kind[a] = ax.kind;
            k.nbins[a] = ax.nbins;
            k.nbtot *= ax.nbins;
            k.eoff[a] = (int32_t)edges.size();
            if (ax.kind == TP_AXIS_MASS) {
                int m = 0;
                for (int s = 0; s < 4; ++s)
                    if (ax.slots & (1 << s)) m |= 1 << inv[s];
                k.slots[a] = m;
                // lower bounds of e_k^2, then upper bounds, then the edges
                for (int side = 0; side < 2; ++side)
                    for (int e = 0; e <= ax.nbins; ++e) {
                        double lo, hi;
                        square_bounds(ax.edges[e], lo, hi);
                        edges.push_back(side == 0 ? lo : hi);
                    }
                for (int e = 0; e <= ax.nbins; ++e) edges.push_back(ax.edges[e]);
                k.guess_lo[a] = ax.edges[0];
                k.guess_inv[a] = ax.nbins / (ax.edges[ax.nbins] - ax.edges[0]);
            } else {
                k.slots[a] = ax.kind == TP_AXIS_ABSCOS ? inv[ax.slots] : 0;
                for (int e = 0; e <= ax.nbins; ++e) edges.push_back(ax.edges[e]);
            }
        }
    }
}

struct Req {
    const tp_events *ev;
    const tp_channel *ch;
    const tp_binning *bn;
    uint64_t *counts;
    tp_stats *stats;
    int8_t *cls_out;
    double *ct_out;
};

uint64_t plan_key(const std::vector<Req> &rq, int mode)
{
    uint64_t h = fnv(&mode, sizeof mode);
    for (const Req &r : rq) {
        h = fnv(r.ev, sizeof(tp_events), h);
        h = fnv(r.ch, sizeof(tp_channel), h);
        int na = r.bn ? r.bn->naxes : 0;
        h = fnv(&na, sizeof na, h);
        for (int a = 0; a < na; ++a) {
            const tp_axis &ax = r.bn->axis[a];
            h = fnv(&ax.kind, sizeof(int32_t) * 3, h);
            h = fnv(ax.edges, sizeof(double) * (ax.nbins + 1), h);
        }
        h = fnv(&r.counts, sizeof(void *), h);
        h = fnv(&r.stats, sizeof(void *), h);
        h = fnv(&r.cls_out, sizeof(void *), h);
        h = fnv(&r.ct_out, sizeof(void *), h);
    }
    return h;
}

// Release a plan and the graphs captured with it, once the work that reads
// them has finished.
void free_plan(Device &d, Plan *q)
{
    hipEventSynchronize(q->ready);
    if (q->used) hipEventSynchronize(q->last_use);
    for (uint64_t gk : q->graph_keys) {
        auto g = d.graphs.find(gk);
        if (g == d.graphs.end()) continue;
        hipGraphExecDestroy(g->second.exec);
        hipGraphDestroy(g->second.graph);
        hipFree(g->second.ws.buf);
        d.graphs.erase(g);
    }
    hipFree(q->dbuf);
    hipHostFree(q->pinned);
    hipEventDestroy(q->ready);
    hipEventDestroy(q->last_use);
    delete q;
}

// Order a use of plan p on stream st after its previous use on another stream
// (the plan's tables, graphs and their workspaces are shared by all uses).
int begin_use(Plan &p, hipStream_t st)
{
    if (p.made_on != st) TP_HIP(hipStreamWaitEvent(st, p.ready, 0));
    if (p.used && p.last_stream != st) TP_HIP(hipStreamWaitEvent(st, p.last_use, 0));
    return TP_OK;
}

int end_use(Plan &p, hipStream_t st)
{
    TP_HIP(hipEventRecord(p.last_use, st));
    p.last_stream = st;
    p.used = true;
    return TP_OK;
}

int build_plan(Device &d, const std::vector<Req> &rq, int mode, hipStream_t st, Plan *&out)
{
    const uint64_t key = plan_key(rq, mode);
    auto it = d.plans.find(key);
    if (it != d.plans.end()) {
        out = it->second;
        d.lru.splice(d.lru.end(), d.lru, out->lru_pos);   // most recently used last
        return TP_OK;
    }
    Plan *p = new Plan();
    p->dtype = rq.empty() ? 0 : rq[0].ev->dtype;
    std::vector<KSample> ks(rq.size());
    for (size_t r = 0; r < rq.size(); ++r)
        fill_sample(ks[r], *rq[r].ev, *rq[r].ch, mode == 0 ? rq[r].bn : nullptr, rq[r].counts, rq[r].stats,
                    rq[r].cls_out, rq[r].ct_out, p->hedges);
    // order the samples by binning scheme (stable), one group per scheme
    std::vector<size_t> order(rq.size());
    for (size_t r = 0; r < order.size(); ++r) order[r] = r;
    auto scheme = [&](size_t r) { return (ks[r].kind[0] * 4 + ks[r].kind[1]) * 2 + (ks[r].olo >= 0 ? 1 : 0); };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return scheme(a) < scheme(b); });
    // the pass kernels index each array with 32-bit offsets from its base: a
    // sample whose arrays reach 2^32 bytes becomes several descriptors of at
    // most ``cap`` events each (same counters; their events add up)
    const int64_t cap = p->dtype == TP_F32 ? (int64_t(1) << 30) : (int64_t(1) << 29);
    const size_t esize = p->dtype == TP_F32 ? 4 : 8;
    int64_t v = 0;
    for (size_t r : order)
        for (int64_t e0 = 0; e0 == 0 || e0 < ks[r].n; e0 += cap) {
            KSample k = ks[r];
            if (e0 > 0 || k.n > cap) {
                for (int c = 0; c < 16; ++c) k.p[c] = static_cast<const char *>(k.p[c]) + e0 * esize;
                k.tag += e0;
                if (k.cls_out) k.cls_out += e0;
                if (k.ct_out) k.ct_out += e0;
                k.n = std::min(cap, ks[r].n - e0);
            }
            // samples start on multiples of 256 virtual events: workgroup ranges
            // and tiles are multiples of 256 too, so every wave reads whole
            // 128-byte lines of each component array (arrays 256-byte aligned)
            k.vstart = v;
            v += (k.n + 255) & ~int64_t(255);
            const int sidx = (int)p->hs.size();
            p->hs.push_back(k);
            const bool ord = k.olo >= 0;
            if (p->groups.empty() || p->groups.back().k0 != k.kind[0] || p->groups.back().k1 != k.kind[1] ||
                p->groups.back().ord != ord) {
                Group g;
                g.k0 = k.kind[0];
                g.k1 = k.kind[1];
                g.ord = ord;
                g.sbeg = sidx;
                g.vbeg = k.vstart;
                p->groups.push_back(g);
            }
            Group &g = p->groups.back();
            g.send = sidx + 1;
            g.vend = v;
            // LDS histogram copy: class-total row, bin rows, overflow row, statistics
            const int stride = (k.nbtot + 2) * 4 + NSTAT;
            g.hist_stride = std::max(g.hist_stride, stride);
            int ed = 0;
            for (int a = 0; a < k.naxes; ++a) ed += edge_doubles(k.kind[a], k.nbins[a]);
            g.edge_doubles = std::max(g.edge_doubles, ed);
        }
    p->vtotal = v;
    if (p->hs.size() > (size_t(1) << 20)) {   // the deferral list holds 20 bits of descriptor index
        delete p;
        return fail(TP_ERANGE, "too many samples once split at 2^32 bytes per array");
    }
    if (p->hedges.empty()) p->hedges.push_back(0.0);
    const size_t sb = p->hs.size() * sizeof(KSample);
    const size_t eb = p->hedges.size() * sizeof(double);
    const size_t tot = ((sb + 255) & ~size_t(255)) + eb;
    if (hipMalloc(&p->dbuf, tot) != hipSuccess) {
        delete p;
        return fail(TP_ENOMEM, "plan table allocation failed");
    }
    if (hipHostMalloc(&p->pinned, tot, hipHostMallocDefault) != hipSuccess) {
        hipFree(p->dbuf);
        delete p;
        return fail(TP_ENOMEM, "pinned staging allocation failed");
    }
    std::memcpy(p->pinned, p->hs.data(), sb);
    std::memcpy(static_cast<char *>(p->pinned) + ((sb + 255) & ~size_t(255)), p->hedges.data(), eb);
    p->dsamples = static_cast<KSample *>(p->dbuf);
    p->dedges = reinterpret_cast<double *>(static_cast<char *>(p->dbuf) + ((sb + 255) & ~size_t(255)));
    TP_HIP(hipMemcpyAsync(p->dbuf, p->pinned, tot, hipMemcpyHostToDevice, st));
    TP_HIP(hipEventCreateWithFlags(&p->ready, hipEventDisableTiming));
    TP_HIP(hipEventCreateWithFlags(&p->last_use, hipEventDisableTiming));
    TP_HIP(hipEventRecord(p->ready, st));
    p->made_on = st;
    d.plans[key] = p;
    p->lru_pos = d.lru.insert(d.lru.end(), key);
    if (d.lru.size() > MAX_PLANS) {
        // least recently used: freed (with its graphs) after its last use
        const uint64_t old = d.lru.front();
        d.lru.pop_front();
        Plan *q = d.plans[old];
        d.plans.erase(old);
        free_plan(d, q);
    }
    out = p;
    return TP_OK;
}

void defaults(tp_tuning &t)
{
    if (t.block != 256 && t.block != 512) t.block = 256;
    if (t.wg_per_cu < 1 || t.wg_per_cu > 32) t.wg_per_cu = 4;
    const int waves = t.block / 64;
    if (t.lds_copies < 1 || t.lds_copies > waves) t.lds_copies = waves;
    if (t.unroll != 1 && t.unroll != 2 && t.unroll != 4) t.unroll = 1;
}

// The device's side streams and fork/join events, created on first use.
int side_streams(Device &d)
{
    if (d.fork) return TP_OK;
    hipError_t e = hipSuccess;
    for (int l = 0; l < NSIDE && e == hipSuccess; ++l) {
        hipStream_t s2 = nullptr;
        hipEvent_t e2 = nullptr;
        e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
        if (e == hipSuccess) d.side.push_back(s2);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&e2, hipEventDisableTiming);
        if (e == hipSuccess) d.join.push_back(e2);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&d.fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        for (hipStream_t s2 : d.side) hipStreamDestroy(s2);
        for (hipEvent_t e2 : d.join) hipEventDestroy(e2);
        d.side.clear();
        d.join.clear();
        d.fork = nullptr;
        return fail(TP_EHIP, std::string("side streams: ") + hipGetErrorString(e));
    }
    return TP_OK;
}

// One pass launch over the samples of group g with launch shape ``tu``;
// ``kp`` carries the plan's tables and the deferral workspace.
int launch_group(int cus, const Group &g, tp_tuning tu, int dtype, int prec, int mode, KParams kp, hipStream_t st)
{
    const int64_t nv = g.vend - g.vbeg;
    defaults(tu);
    const int epl = dtype == TP_F32 ? tu.unroll : std::min(tu.unroll, 2);
    const int64_t tile = (int64_t)epl * tu.block;
    int copies = tu.lds_copies;
    size_t hist_bytes = 0;
    for (;;) {
        hist_bytes = ((size_t)(8 + copies * g.hist_stride) * 4 + 15) & ~size_t(15);
        if (hist_bytes + (size_t)g.edge_doubles * 8 <= LDS_LIMIT || copies == 1) break;
        --copies;
    }
    const size_t lds = hist_bytes + (size_t)g.edge_doubles * 8;
    if (lds > LDS_LIMIT) return fail(TP_ERANGE, "histogram does not fit in LDS");
    int64_t grid = (int64_t)cus * tu.wg_per_cu;
    const int64_t need = (nv + tile - 1) / tile;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    int64_t range = (nv + grid - 1) / grid;
    range = (range + tile - 1) / tile * tile;
    // the kernel forms in-segment offsets in 32 bits: at most 2^26 events a workgroup
    range = std::min<int64_t>(range, int64_t(1) << 26);
    grid = (nv + range - 1) / range;
    kp.sbeg = g.sbeg;
    kp.send = g.send;
    kp.vbeg = g.vbeg;
    kp.vend = g.vend;
    kp.lds_copies = copies;
    kp.hist_stride = g.hist_stride;
    kp.edge_doubles = g.edge_doubles;
    kp.range = range;
    TP_HIP(launch_pass(dtype, prec, mode, epl, g.k0, g.k1, g.ord, kp, (int)grid, tu.block, lds, st));
    return TP_OK;
}

// Launch the plan's pass kernels (one per scheme group, each with its own
// launch shape gtu[g]; only the group ``only`` when it is >= 0), then the
// exact tier over the shared deferral list.
int launch_plan(Device &d, const Plan &p, const std::vector<tp_tuning> &gtu, int prec, int mode,
                const Workspace &ws, hipStream_t st, int only = -1)
{
    if (p.vtotal == 0) return TP_OK;
    const bool timed = g_timing.on && !g_timing.ring.empty();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        auto &pr = g_timing.ring[g_timing.next];
        e0 = pr.first;
        e1 = pr.second;
        TP_HIP(hipEventRecord(e0, st));
    }
    KParams kp;
    std::memset(&kp, 0, sizeof kp);
    kp.samples = p.dsamples;
    kp.edges = p.dedges;
    kp.xlist = ws.xlist;
    kp.xcount = ws.xcount;
    kp.xdone = ws.xdone;
    kp.xcap = (uint32_t)ws.cap;
    kp.mode = mode;
    // Several scheme groups run as parallel branches (the caller's stream and
    // NSIDE side streams, in turn): their launches overlap,
    // so one kernel's last workgroups share the chip with the next kernel's
    // first, and memory-bound and issue-bound schemes share the compute units.
    // The exact tier waits for all of them.  (Under graph capture the side
    // streams join the capture through the fork event and leave it through
    // the joins.)
    int ngroups = 0;
    size_t largest = 0;
    for (size_t gi = 0; gi < p.groups.size(); ++gi) {
        const Group &g = p.groups[gi];
        ngroups += g.vend > g.vbeg;
        if (g.vend - g.vbeg > p.groups[largest].vend - p.groups[largest].vbeg) largest = gi;
    }
    const bool fork = only < 0 && ngroups > 1;
    bool joined[NSIDE] = {};
    if (fork) {
        int rc = side_streams(d);
        if (rc) return rc;
        TP_HIP(hipEventRecord(d.fork, st));
    }
    // the largest group (usually the last to finish) on the caller's stream,
    // so that the exact tier follows it without a wait on another stream
    int k = 1;
    for (size_t gi = 0; gi < p.groups.size(); ++gi) {
        if (only >= 0 && (size_t)only != gi) continue;
        const Group &g = p.groups[gi];
        const int64_t nv = g.vend - g.vbeg;
        if (nv <= 0) continue;
        const int lane = !fork || gi == largest ? 0 : k++ % (NSIDE + 1);
        hipStream_t gs = st;
        if (lane > 0) {
            gs = d.side[lane - 1];
            if (!joined[lane - 1]) TP_HIP(hipStreamWaitEvent(gs, d.fork, 0));
            joined[lane - 1] = true;
        }
        // beside the largest group, a group takes at most SIDE_WG_PER_CU
        // workgroups per CU, leaving the largest (the critical path) more of
        // the chip from the start; the largest runs in finer ranges
        // (LARGEST_WG_PER_CU)
        tp_tuning tu = gtu[gi];
        if (fork && gi != largest && tu.wg_per_cu > SIDE_WG_PER_CU) tu.wg_per_cu = SIDE_WG_PER_CU;
        if (fork && gi == largest) tu.wg_per_cu = LARGEST_WG_PER_CU;
        const int rc = launch_group(d.cus, g, tu, p.dtype, prec, mode, kp, gs);
        if (rc) return rc;
    }
    for (int l = 0; l < NSIDE; ++l) {
        if (!joined[l]) continue;
        TP_HIP(hipEventRecord(d.join[l], d.side[l]));
        TP_HIP(hipStreamWaitEvent(st, d.join[l], 0));
    }
    if (timed) {
        TP_HIP(hipEventRecord(e1, st));
        g_timing.next = (g_timing.next + 1) % g_timing.ring.size();
        g_timing.used = std::min(g_timing.used + 1, g_timing.ring.size());
    }
    static const bool debug = std::getenv("TP_DEBUG") != nullptr;
    if (debug) {
        // diagnostics: which events the float64 tier deferred, and at which stage
        uint32_t cnt = 0;
        TP_HIP(hipStreamSynchronize(st));
        TP_HIP(hipMemcpy(&cnt, ws.xcount, sizeof cnt, hipMemcpyDeviceToHost));
        const uint32_t m = std::min<uint32_t>(cnt, 4096);
        std::vector<uint64_t> lst(m);
        if (m) TP_HIP(hipMemcpy(lst.data(), ws.xlist, m * sizeof(uint64_t), hipMemcpyDeviceToHost));
        int why[7] = { 0, 0, 0, 0, 0, 0, 0 };
        for (uint64_t e : lst) why[std::min<int>(6, (int)(e >> 60))]++;
        std::fprintf(stderr, "tp_debug: %u deferred (validity %d, sign %d, axis0 %d, axis1 %d, order %d, "
                     "first pass %d)", cnt, why[1], why[2], why[3], why[4], why[5], why[6]);
        for (uint32_t k = 0; k < std::min<uint32_t>(m, 8); ++k)
            std::fprintf(stderr, " [s%d e%lld w%d]", (int)((lst[k] >> 40) & 0xfffff),
                         (long long)(lst[k] & ((1ull << 40) - 1)), (int)(lst[k] >> 60));
        std::fprintf(stderr, "\n");
    }
    TP_HIP(launch_exact(p.dtype, mode, kp, exact_grid(p.vtotal), st));
    return TP_OK;
}

std::string tune_key(const std::vector<Req> &rq, int prec)
{
    int64_t n = 0;
    int maxbins = 0, phi = 0, mass = 0, cosv = 0;
    for (const Req &r : rq) {
        n += r.ev->n;
        if (r.bn) {
            int tot = 1;
            for (int a = 0; a < r.bn->naxes; ++a) {
                tot *= r.bn->axis[a].nbins;
                phi |= r.bn->axis[a].kind == TP_AXIS_ABSPHI;
                mass |= r.bn->axis[a].kind == TP_AXIS_MASS;
                cosv |= r.bn->axis[a].kind == TP_AXIS_ABSCOS;
            }
            maxbins = std::max(maxbins, r.bn->naxes ? tot : 0);
        }
    }
    int nb = 0;
    while ((int64_t(1) << nb) < n) ++nb;
    char buf[160];
    std::snprintf(buf, sizeof buf, "d%d_p%d_n2^%d_b%d_ax%d%d%d_s%zu", rq.empty() ? 0 : rq[0].ev->dtype, prec,
                  nb, maxbins, phi, mass, cosv, rq.size() > 1 ? (size_t)2 : (size_t)1);
    return buf;
}

void load_tune_file(Device &d)
{
    if (d.tune_loaded) return;
    d.tune_loaded = true;
    const char *fn = std::getenv("TP_TUNE_CACHE");
    if (!fn) return;
    FILE *f = std::fopen(fn, "r");
    if (!f) return;
    char key[200];
    tp_tuning t;
    // {"key": [block, wg_per_cu, lds_copies, unroll], ...}: the opening brace,
    // then one entry per line
    if (std::fscanf(f, " {") == 0) {
        while (std::fscanf(f, " \"%199[^\"]\": [%d, %d, %d, %d]%*[,}\n ]", key, &t.block, &t.wg_per_cu,
                           &t.lds_copies, &t.unroll) == 5)
            d.tuned[key] = t;
    }
    std::fclose(f);
}

void save_tune_file(const Device &d)
{
    const char *fn = std::getenv("TP_TUNE_CACHE");
    if (!fn) return;
    FILE *f = std::fopen(fn, "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (auto &kv : d.tuned) {
        std::fprintf(f, " \"%s\": [%d, %d, %d, %d]%s\n", kv.first.c_str(), kv.second.block, kv.second.wg_per_cu,
                     kv.second.lds_copies, kv.second.unroll, ++i < d.tuned.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
}

// Tuning-cache key of one scheme group: storage, precision, binning kinds,
// size class and histogram size.
std::string group_key(const Plan &p, const Group &g, int prec)
{
    int nb = 0;
    while ((int64_t(1) << nb) < g.vend - g.vbeg) ++nb;
    char buf[160];
    std::snprintf(buf, sizeof buf, "g_d%d_p%d_k%d%d%s_n2^%d_h%d", p.dtype, prec, g.k0, g.k1, g.ord ? "o" : "", nb,
                  g.hist_stride);
    return buf;
}

// Launch shape of every group: the explicit tuning, else the group's tuned
// entry, else the whole request's, else defaults.
std::vector<tp_tuning> resolve_tunings(Device &d, const Plan &p, const std::vector<Req> &rq, int prec,
                                       const tp_tuning *tuning)
{
    std::vector<tp_tuning> out(p.groups.size());
    tp_tuning whole;
    std::memset(&whole, 0, sizeof whole);
    if (!tuning) {
        auto it = d.tuned.find(tune_key(rq, prec));
        if (it != d.tuned.end()) whole = it->second;
    }
    for (size_t g = 0; g < p.groups.size(); ++g) {
        tp_tuning t = tuning ? *tuning : whole;
        if (!tuning) {
            auto it = d.tuned.find(group_key(p, p.groups[g], prec));
            if (it != d.tuned.end()) t = it->second;
        }
        defaults(t);
        out[g] = t;
    }
    return out;
}

int current_device(int &id)
{
    TP_HIP(hipGetDevice(&id));
    return TP_OK;
}

int run(const std::vector<Req> &rq, int prec, int mode, const tp_tuning *tuning, int flags, hipStream_t st)
{
    int dev = 0;
    int rc = current_device(dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Device &d = device(dev);
    load_tune_file(d);
    Plan *p = nullptr;
    rc = build_plan(d, rq, mode, st, p);
    if (rc) return rc;
    rc = begin_use(*p, st);
    if (rc) return rc;
    const std::vector<tp_tuning> gtu = resolve_tunings(d, *p, rq, prec, tuning);
    if (flags & TP_BATCH_GRAPH) {
        uint64_t gk = plan_key(rq, mode);
        if (!gtu.empty()) gk = fnv(gtu.data(), gtu.size() * sizeof(tp_tuning), gk);
        gk = fnv(&prec, sizeof prec, gk);
        auto it = d.graphs.find(gk);
        if (it == d.graphs.end()) {
            GraphEntry ge;
            rc = new_workspace(list_capacity(p->vtotal), st, ge.ws);
            if (rc) return rc;
            TP_HIP(hipStreamSynchronize(st));
            hipStream_t cap;
            TP_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            TP_HIP(hipStreamWaitEvent(cap, p->ready, 0));
            TP_HIP(hipStreamSynchronize(cap));
            const bool was_on = g_timing.on;
            g_timing.on = false;
            TP_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            rc = launch_plan(d, *p, gtu, prec, mode, ge.ws, cap);
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(cap, &g);
            g_timing.on = was_on;
            hipStreamDestroy(cap);
            if (rc) return rc;
            if (ee != hipSuccess) return fail(TP_EHIP, std::string("graph capture: ") + hipGetErrorString(ee));
            ge.graph = g;
            TP_HIP(hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0));
            it = d.graphs.emplace(gk, ge).first;
            p->graph_keys.push_back(gk);
        }
        const bool timed = g_timing.on && !g_timing.ring.empty();
        if (timed) TP_HIP(hipEventRecord(g_timing.ring[g_timing.next].first, st));
        TP_HIP(hipGraphLaunch(it->second.exec, st));
        if (timed) {
            TP_HIP(hipEventRecord(g_timing.ring[g_timing.next].second, st));
            g_timing.next = (g_timing.next + 1) % g_timing.ring.size();
            g_timing.used = std::min(g_timing.used + 1, g_timing.ring.size());
        }
        return end_use(*p, st);
    }
    Workspace ws;
    rc = get_workspace(d, st, list_capacity(p->vtotal), ws);
    if (rc) return rc;
    rc = launch_plan(d, *p, gtu, prec, mode, ws, st);
    if (rc) return rc;
    return end_use(*p, st);
}

// exact ratio num/den of integers, rounded (long double division, then to double)
double ratio(__int128 num, __int128 den)
{
    return (double)((long double)num / (long double)den);
}

void two_count(uint64_t a, uint64_t b, double &A, double &sA, bool &empty)
{
    const __int128 n = (__int128)a + b;
    empty = (n == 0);
    if (empty) {
        A = sA = NAN;
        return;
    }
    A = ratio((__int128)a - (__int128)b, n);
    // 1 - A^2 = 4ab / n^2 exactly
    const double one_m = ratio((__int128)4 * a * b, n * n);
    sA = std::sqrt(std::max(0.0, one_m) / (double)n);
}

void half_comb(uint64_t n1, uint64_t n2, uint64_t n3, uint64_t n4, int sgn, double sa, double sb, double &v,
               double &s)
{
    // (A + sgn B)/2 with A = (n1 - n2)/(n1 + n2), B = (n3 - n4)/(n3 + n4)
    const __int128 N = (__int128)n1 + n2, Nb = (__int128)n3 + n4;
    if (N == 0 || Nb == 0) {
        v = s = NAN;
        return;
    }
    const __int128 num = ((__int128)n1 - (__int128)n2) * Nb + sgn * ((__int128)n3 - (__int128)n4) * N;
    v = ratio(num, 2 * N * Nb);
    s = 0.5 * std::sqrt(sa * sa + sb * sb);
}

// Regularised upper incomplete gamma Q(a, x): power series for x < a + 1,
// Lentz's continued fraction otherwise (Press et al., Numerical Recipes, 6.2).
double gamma_q(double a, double x)
{
    if (x <= 0) return 1.0;
    const double lg = std::lgamma(a);
    if (x < a + 1.0) {
        double ap = a, del = 1.0 / a, sum = del;
        for (int n = 0; n < 100000; ++n) {
            ap += 1.0;
            del *= x / ap;
            sum += del;
            if (std::fabs(del) < std::fabs(sum) * 1e-17) break;
        }
        return std::max(0.0, 1.0 - sum * std::exp(-x + a * std::log(x) - lg));
    }
    const double tiny = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / tiny, dd = 1.0 / b, h = dd;
    for (int i = 1; i < 100000; ++i) {
        const double an = -i * (i - a);
        b += 2.0;
        dd = an * dd + b;
        if (std::fabs(dd) < tiny) dd = tiny;
        c = b + an / c;
        if (std::fabs(c) < tiny) c = tiny;
        dd = 1.0 / dd;
        const double del = dd * c;
        h *= del;
        if (std::fabs(del - 1.0) < 1e-16) break;
    }
    return std::exp(-x + a * std::log(x) - lg) * h;
}

}  // namespace

// ====================================================================== C-ABI
extern "C" {

int tp_compute(const tp_events *ev, const tp_channel *ch, int32_t precision, int8_t *cls_out, double *ct_out,
               tp_stats *stats, void *stream)
{
    int rc = check_events(ev, precision);
    if (rc) return rc;
    rc = check_channel(ch);
    if (rc) return rc;
    if (!stats) return fail(TP_EINVAL, "stats is NULL");
    if (ev->n == 0) return TP_OK;   // per-event outputs of no elements may be NULL too
    if (!cls_out && !ct_out) return fail(TP_EINVAL, "tp_compute needs cls_out or ct_out");
    if (!cls_out) return fail(TP_EINVAL, "cls_out is required (the exact tier writes through it)");
    std::vector<Req> rq{ Req{ ev, ch, nullptr, nullptr, stats, cls_out, ct_out } };
    return run(rq, precision, 1, nullptr, 0, static_cast<hipStream_t>(stream));
}

int tp_bin(const tp_events *ev, const tp_channel *ch, const tp_binning *bn, int32_t precision, uint64_t *counts,
           tp_stats *stats, void *stream)
{
    int rc = check_events(ev, precision);
    if (rc) return rc;
    rc = check_channel(ch);
    if (rc) return rc;
    rc = check_binning(bn);
    if (rc) return rc;
    rc = check_identical(ch, bn);
    if (rc) return rc;
    if (!counts || !stats) return fail(TP_EINVAL, "counts and stats are required");
    if (ev->n == 0) return TP_OK;
    std::vector<Req> rq{ Req{ ev, ch, bn, counts, stats, nullptr, nullptr } };
    return run(rq, precision, 0, nullptr, 0, static_cast<hipStream_t>(stream));
}

int tp_bin_noalloc(const tp_events *ev, const tp_channel *ch, const tp_binning *bn, int32_t precision,
                   uint64_t *counts, tp_stats *stats, void *stream)
{
    int rc = check_events(ev, precision);
    if (rc) return rc;
    rc = check_channel(ch);
    if (rc) return rc;
    rc = check_binning(bn);
    if (rc) return rc;
    rc = check_identical(ch, bn);
    if (rc) return rc;
    if (!counts || !stats) return fail(TP_EINVAL, "counts and stats are required");
    if (ev->n > NA_MAX_EVENTS) return fail(TP_ERANGE, "tp_bin_noalloc takes at most 2^22 events per call");
    if (ev->n == 0) return TP_OK;
    KSample k;
    FixedEdges ed;
    fill_sample(k, *ev, *ch, bn, counts, stats, nullptr, nullptr, ed);
    if (ed.overflow) return fail(TP_ERANGE, "tp_bin_noalloc holds at most 384 doubles of edge data per call");
    k.vstart = 0;
    Group g;
    g.k0 = k.kind[0];
    g.k1 = k.kind[1];
    g.ord = k.olo >= 0;
    g.sbeg = 0;
    g.send = 1;
    g.vbeg = 0;
    g.vend = (k.n + 255) & ~int64_t(255);
    g.hist_stride = (k.nbtot + 2) * 4 + NSTAT;
    g.edge_doubles = ed.n;
    int dev = 0, cus = 0;
    TP_HIP(hipGetDevice(&dev));
    TP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    unsigned char *base = nullptr;
    TP_HIP(noalloc_scratch(dev, &base));
    const hipStream_t st = static_cast<hipStream_t>(stream);
    TP_HIP(launch_noalloc_setup(k, ed.v, ed.n, base, st));
    KParams kp;
    std::memset(&kp, 0, sizeof kp);
    kp.samples = reinterpret_cast<const KSample *>(base + NA_SAMPLE_OFF);
    kp.edges = reinterpret_cast<const double *>(base + NA_EDGES_OFF);
    kp.xlist = reinterpret_cast<uint64_t *>(base + NA_LIST_OFF);
    kp.xcount = reinterpret_cast<uint32_t *>(base + NA_COUNT_OFF);
    kp.xdone = kp.xcount + 1;
    kp.xcap = (uint32_t)NA_MAX_EVENTS;
    kp.mode = 0;
    tp_tuning tu;
    tu.block = 256;
    tu.wg_per_cu = 8;
    tu.lds_copies = 4;
    tu.unroll = 1;
    rc = launch_group(cus > 0 ? cus : 256, g, tu, ev->dtype, precision, 0, kp, st);
    if (rc) return rc;
    TP_HIP(launch_exact(ev->dtype, 0, kp, exact_grid(g.vend), st));
    return TP_OK;
}

int tp_probe_f32(const tp_events *ev, const tp_channel *ch, float *det32, float *bound32, double *det64,
                 double *scale64, void *stream)
{
    int rc = check_events(ev, TP_PREC_F32_RECHECK);
    if (rc) return rc;
    rc = check_channel(ch);
    if (rc) return rc;
    if (!det32 || !bound32 || !det64 || !scale64) return fail(TP_EINVAL, "every output is required");
    if (ev->n > (int64_t(1) << 31)) return fail(TP_ERANGE, "at most 2^31 events per call");
    if (ev->n == 0) return TP_OK;
    KSample k;
    FixedEdges ed;
    fill_sample(k, *ev, *ch, nullptr, nullptr, nullptr, nullptr, nullptr, ed);
    TP_HIP(launch_probe(k, det32, bound32, det64, scale64, static_cast<hipStream_t>(stream)));
    return TP_OK;
}

int tp_batch(const tp_sample *samples, int32_t nsamples, int32_t precision, const tp_tuning *tuning,
             int32_t flags, void *stream)
{
    if (nsamples < 0 || (nsamples > 0 && !samples)) return fail(TP_EINVAL, "bad sample list");
    if (nsamples > (1 << 20)) return fail(TP_ERANGE, "too many samples");
    if (flags & ~TP_BATCH_GRAPH) return fail(TP_EINVAL, "unknown flags");
    std::vector<Req> rq;
    int dtype = -1;
    for (int i = 0; i < nsamples; ++i) {
        const tp_sample &s = samples[i];
        int rc = check_events(&s.ev, precision);
        if (rc) return rc;
        rc = check_channel(&s.ch);
        if (rc) return rc;
        rc = check_binning(&s.bn);
        if (rc) return rc;
        rc = check_identical(&s.ch, &s.bn);
        if (rc) return rc;
        if (!s.counts || !s.stats) return fail(TP_EINVAL, "counts and stats are required");
        if (dtype >= 0 && s.ev.dtype != dtype) return fail(TP_EUNSUPPORTED, "all samples of a batch share one dtype");
        dtype = s.ev.dtype;
        if (s.ev.n > 0) rq.push_back(Req{ &s.ev, &s.ch, &s.bn, s.counts, s.stats, nullptr, nullptr });
    }
    if (rq.empty()) return TP_OK;   // nothing to launch (and no empty graph to capture)
    return run(rq, precision, 0, tuning, flags, static_cast<hipStream_t>(stream));
}

int tp_autotune(const tp_sample *samples, int32_t nsamples, int32_t precision, void *stream, tp_tuning *best)
{
    if (!best) return fail(TP_EINVAL, "best is NULL");
    if (nsamples <= 0 || !samples) return fail(TP_EINVAL, "bad sample list");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // validate and size a scratch sink
    size_t words = 0;
    bool any_events = false;
    for (int i = 0; i < nsamples; ++i) {
        int rc = check_events(&samples[i].ev, precision);
        if (rc) return rc;
        rc = check_channel(&samples[i].ch);
        if (rc) return rc;
        rc = check_binning(&samples[i].bn);
        if (rc) return rc;
        rc = check_identical(&samples[i].ch, &samples[i].bn);
        if (rc) return rc;
        int tot = 1;
        for (int a = 0; a < samples[i].bn.naxes; ++a) tot *= samples[i].bn.axis[a].nbins;
        words += (size_t)(tot + 1) * 4 + NSTAT;
        any_events |= samples[i].ev.n > 0;
    }
    if (!any_events) {   // nothing to time: the default shape
        tp_tuning t{};
        defaults(t);
        *best = t;
        return TP_OK;
    }
    int dev = 0;
    int rc = current_device(dev);
    if (rc) return rc;
    std::vector<Req> rq;
    std::vector<tp_sample> sink(samples, samples + nsamples);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        Device &d = device(dev);
        if (d.scratch_words < words) {
            if (d.scratch_counts) hipFree(d.scratch_counts);
            if (hipMalloc(&d.scratch_counts, words * 8) != hipSuccess) {
                d.scratch_counts = nullptr;
                d.scratch_words = 0;
                return fail(TP_ENOMEM, "autotune scratch allocation failed");
            }
            d.scratch_words = words;
        }
        size_t off = 0;
        for (int i = 0; i < nsamples; ++i) {
            int tot = 1;
            for (int a = 0; a < samples[i].bn.naxes; ++a) tot *= samples[i].bn.axis[a].nbins;
            sink[i].counts = d.scratch_counts + off;
            off += (size_t)(tot + 1) * 4;
            sink[i].stats = reinterpret_cast<tp_stats *>(d.scratch_counts + off);
            off += NSTAT;
        }
    }
    for (auto &s : sink)
        if (s.ev.n > 0) rq.push_back(Req{ &s.ev, &s.ch, &s.bn, s.counts, s.stats, nullptr, nullptr });
    // 16 and 32 workgroups per CU (finer ranges: 4 or 8 rounds of the 4
    // resident workgroups) won for the single-scheme 10^8- and 5e8-event
    // samples (16: 1.1 and 3 % faster than 8; 32: another 1.2 % on the latter)
    std::vector<tp_tuning> cand;
    for (int epl : { 1, 2, 4 })
        for (int wpc : { 2, 4, 8, 16, 32 })
            for (int copies : { 1, 4 }) {
                tp_tuning t;
                t.block = 256;
                t.wg_per_cu = wpc;
                t.lds_copies = copies;
                t.unroll = epl;
                cand.push_back(t);
            }
    hipEvent_t a, b;
    TP_HIP(hipEventCreate(&a));
    TP_HIP(hipEventCreate(&b));
    std::lock_guard<std::mutex> lk(g_mu);
    Device &d = device(dev);
    load_tune_file(d);
    const bool was_on = g_timing.on;
    g_timing.on = false;
    Plan *p = nullptr;
    Workspace ws;
    rc = build_plan(d, rq, 0, st, p);
    if (!rc) rc = begin_use(*p, st);
    if (!rc) rc = get_workspace(d, st, list_capacity(p->vtotal), ws);
    // time ``trials`` runs of ``reps`` launches of group g with shape t; best run, ms per launch
    auto measure = [&](size_t g, const tp_tuning &t, int trials, int reps, float &ms) -> int {
        const std::vector<tp_tuning> gtu(p->groups.size(), t);
        int r = launch_plan(d, *p, gtu, precision, 0, ws, st, (int)g);   // warm-up
        ms = 1e30f;
        for (int trial = 0; trial < trials && !r; ++trial) {
            TP_HIP(hipEventRecord(a, st));
            for (int k = 0; k < reps && !r; ++k) r = launch_plan(d, *p, gtu, precision, 0, ws, st, (int)g);
            TP_HIP(hipEventRecord(b, st));
            TP_HIP(hipEventSynchronize(b));
            float m = 0;
            TP_HIP(hipEventElapsedTime(&m, a, b));
            ms = std::min(ms, m / reps);
        }
        return r;
    };
    // bring the clocks up before anything is timed
    if (!rc) {
        const std::vector<tp_tuning> gtu(p->groups.size(), cand[0]);
        for (int k = 0; k < 5 && !rc; ++k) rc = launch_plan(d, *p, gtu, precision, 0, ws, st);
        if (!rc) TP_HIP(hipStreamSynchronize(st));
    }
    // each scheme group is tuned on its own launches: every candidate briefly,
    // then the three fastest again, longer
    tp_tuning overall = cand[0];
    int64_t largest = -1;
    for (size_t g = 0; g < (p ? p->groups.size() : 0) && !rc; ++g) {
        std::vector<std::pair<float, size_t>> first;
        for (size_t c = 0; c < cand.size() && !rc; ++c) {
            float ms = 0;
            rc = measure(g, cand[c], 2, 3, ms);
            first.emplace_back(ms, c);
        }
        if (rc) break;
        std::sort(first.begin(), first.end());
        float best_ms = 1e30f;
        tp_tuning bt = cand[first[0].second];
        for (size_t k = 0; k < std::min<size_t>(3, first.size()) && !rc; ++k) {
            float ms = 0;
            rc = measure(g, cand[first[k].second], 3, 5, ms);
            if (ms < best_ms) {
                best_ms = ms;
                bt = cand[first[k].second];
            }
        }
        d.tuned[group_key(*p, p->groups[g], precision)] = bt;
        static const bool verbose = std::getenv("TP_TUNE_VERBOSE") != nullptr;
        if (verbose)
            std::fprintf(stderr, "tp_tune: group %zu (kinds %d,%d, %lld events): block %d wg/cu %d copies %d "
                         "epl %d, %.4f ms per launch\n", g, p->groups[g].k0, p->groups[g].k1,
                         (long long)(p->groups[g].vend - p->groups[g].vbeg), bt.block, bt.wg_per_cu, bt.lds_copies,
                         bt.unroll, best_ms);
        const int64_t nv = p->groups[g].vend - p->groups[g].vbeg;
        if (nv > largest) {
            largest = nv;
            overall = bt;
        }
    }
    // No whole-plan stage: the groups' launches overlap (parallel branches),
    // and timing the whole plan as eager launches ranked some shapes wrongly
    // for the graphed batch (two workgroups per CU for the largest group
    // looked faster eagerly and ran 10-15 % slower as a graph); each group's
    // own ranking held.
    g_timing.on = was_on;
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (p && !rc) rc = end_use(*p, st);
    if (rc) return rc;
    // the whole request's entry (for callers that pass it explicitly): the
    // largest group's shape
    *best = overall;
    d.tuned[tune_key(rq, precision)] = overall;
    save_tune_file(d);
    return TP_OK;
}

int tp_asym(const uint64_t *counts, int64_t nrows, tp_asym_row *out)
{
    if (!counts || !out) return fail(TP_EINVAL, "null pointer");
    if (nrows < 0) return fail(TP_EINVAL, "nrows < 0");
    for (int64_t r = 0; r < nrows; ++r) {
        const uint64_t *n = counts + r * 4;
        tp_asym_row &o = out[r];
        std::memset(&o, 0, sizeof o);
        for (int k = 0; k < 4; ++k) o.N[k] = n[k];
        bool e0, e1, e2, e3;
        two_count(n[0], n[1], o.A_T, o.s_A_T, e0);
        two_count(n[2], n[3], o.Abar_T, o.s_Abar_T, e1);
        two_count(n[0], n[2], o.A_plus, o.s_A_plus, e2);
        two_count(n[1], n[3], o.A_minus, o.s_A_minus, e3);
        o.flags = (e0 ? 1u : 0u) | (e1 ? 2u : 0u) | (e2 ? 4u : 0u) | (e3 ? 8u : 0u);
        half_comb(n[0], n[1], n[2], n[3], -1, o.s_A_T, o.s_Abar_T, o.a_CP, o.s_a_CP);
        half_comb(n[0], n[1], n[2], n[3], +1, o.s_A_T, o.s_Abar_T, o.a_P, o.s_a_P);
        half_comb(n[0], n[2], n[1], n[3], +1, o.s_A_plus, o.s_A_minus, o.A_even, o.s_A_even);
        half_comb(n[0], n[2], n[1], n[3], -1, o.s_A_plus, o.s_A_minus, o.A_odd, o.s_A_odd);
    }
    return TP_OK;
}

int tp_scp(const uint64_t *counts, int64_t nbins, int32_t mode, double *s_out, double *chi2, int64_t *ndf,
           double *pvalue)
{
    if (!counts || !chi2 || !ndf || !pvalue) return fail(TP_EINVAL, "null pointer");
    if (nbins < 1) return fail(TP_EINVAL, "nbins < 1");
    if (mode != 0 && mode != 1) return fail(TP_EINVAL, "mode must be 0 (P-even) or 1 (P-odd)");
    std::vector<uint64_t> x(nbins), xb(nbins);
    __int128 tx = 0, txb = 0;
    for (int64_t i = 0; i < nbins; ++i) {
        const uint64_t *n = counts + (i + 1) * 4;
        x[i] = mode == 0 ? n[0] + n[1] : n[0] + n[3];
        xb[i] = mode == 0 ? n[2] + n[3] : n[1] + n[2];
        tx += x[i];
        txb += xb[i];
    }
    double c2 = 0.0;
    for (int64_t i = 0; i < nbins; ++i) {
        double s = 0.0;
        if (txb != 0) {
            // S = (x - a xb)/sqrt(x + a^2 xb), a = tx/txb:  numerator (x txb - tx xb)/txb,
            // radicand (x txb^2 + tx^2 xb)/txb^2
            const __int128 num = (__int128)x[i] * txb - tx * (__int128)xb[i];
            const long double rad = (long double)x[i] * (long double)txb * (long double)txb +
                                    (long double)tx * (long double)tx * (long double)xb[i];
            if (rad > 0) s = (double)((long double)num / sqrtl(rad));
        }
        if (s_out) s_out[i] = s;
        c2 += s * s;
    }
    *chi2 = c2;
    *ndf = nbins - 1;
    *pvalue = nbins > 1 ? gamma_q(0.5 * (double)(nbins - 1), 0.5 * c2) : NAN;
    return TP_OK;
}

int tp_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (on && g_timing.ring.empty()) {
        g_timing.ring.resize(4096);
        for (auto &pr : g_timing.ring) {
            TP_HIP(hipEventCreate(&pr.first));
            TP_HIP(hipEventCreate(&pr.second));
        }
    }
    g_timing.on = on != 0;
    g_timing.next = 0;
    g_timing.used = 0;
    return TP_OK;
}

int tp_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_timing.next = 0;
    g_timing.used = 0;
    return TP_OK;
}

int tp_timing_read(double *avg_ms, int64_t *launches)
{
    if (!avg_ms || !launches) return fail(TP_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0;
    const size_t n = g_timing.used;
    for (size_t i = 0; i < n; ++i) {
        auto &pr = g_timing.ring[i];
        TP_HIP(hipEventSynchronize(pr.second));
        float ms = 0.0f;
        TP_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
    }
    *launches = (int64_t)n;
    *avg_ms = n ? tot / (double)n : 0.0;
    return TP_OK;
}

int tp_release(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    hipDeviceSynchronize();
    for (auto &kv : g_dev) {
        Device &d = kv.second;
        for (auto &w : d.ws) hipFree(w.second.buf);
        for (auto &p : d.plans) free_plan(d, p.second);
        for (auto &g : d.graphs) {
            hipGraphExecDestroy(g.second.exec);
            hipGraphDestroy(g.second.graph);
            hipFree(g.second.ws.buf);
        }
        if (d.scratch_counts) hipFree(d.scratch_counts);
        for (auto &f : d.eflag) hipFree(f.second);
        for (hipStream_t s2 : d.side) hipStreamDestroy(s2);
        for (hipEvent_t e2 : d.join) hipEventDestroy(e2);
        if (d.fork) hipEventDestroy(d.fork);
    }
    g_dev.clear();
    return TP_OK;
}

const char *tp_strerror(int status)
{
    if (!g_err.empty() && status != TP_OK) return g_err.c_str();
    switch (status) {
    case TP_OK: return "ok";
    case TP_EINVAL: return "invalid argument";
    case TP_EUNSUPPORTED: return "unsupported";
    case TP_EHIP: return "HIP runtime error";
    case TP_ENOMEM: return "out of device memory";
    case TP_ERANGE: return "size beyond an implementation limit";
    case TP_EUNCERTAIN: return "a decision could not be certified";
    default: return "unknown status";
    }
}

int tp_version(void) { return TPASYM_VERSION; }

// ------------------------------------------------------------ energy test
int tp_coords(const tp_events *ev, const int32_t *masks, int32_t ncoord, double scale, int32_t relabel,
              float *coords, int64_t ld, void *stream)
{
    if (relabel != TP_RELABEL_NONE && relabel != TP_RELABEL_D4PI) return fail(TP_EINVAL, "unknown relabel");
    if (!ev || !masks || !coords) return fail(TP_EINVAL, "null pointer");
    if (ev->n < 0 || ev->n >= (int64_t(1) << 40)) return fail(TP_ERANGE, "n out of range");
    if (ev->dtype != TP_F32 && ev->dtype != TP_F64) return fail(TP_EINVAL, "dtype must be TP_F32 or TP_F64");
    if (ncoord < 1 || ncoord > tpe::MAXD) return fail(TP_ERANGE, "ncoord must be 1..8");
    if (ld < ev->n) return fail(TP_EINVAL, "ld < n");
    if (!(scale > 0.0) || !std::isfinite(scale)) return fail(TP_EINVAL, "scale must be positive and finite");
    tpe::CParams c;
    std::memset(&c, 0, sizeof c);
    for (int k = 0; k < ncoord; ++k) {
        if (masks[k] < 1 || masks[k] > 15) return fail(TP_EINVAL, "mask must be a nonzero 4-bit slot mask");
        c.masks[k] = masks[k];
    }
    if (ev->n == 0) return TP_OK;
    for (int s = 0; s < 4; ++s)
        for (int q = 0; q < 4; ++q) {
            if (!ev->p[s][q]) return fail(TP_EINVAL, "component pointer is NULL");
            c.p[s * 4 + q] = ev->p[s][q];
        }
    c.n = ev->n;
    c.ncoord = ncoord;
    c.scale = scale;
    c.out = coords;
    c.ldo = ld;
    c.relabel = relabel;
    TP_HIP(tpe::launch_coords(c, ev->dtype, static_cast<hipStream_t>(stream)));
    return TP_OK;
}

int tp_pairsums(const float *coords, int32_t dims, int64_t ld, int64_t n, double sigma, const uint8_t *cols,
                int32_t ncols, int32_t nrow, double *sums, void *stream)
{
    if (!coords || !cols || !sums) return fail(TP_EINVAL, "null pointer");
    if (dims < 1 || dims > tpe::MAXD) return fail(TP_ERANGE, "dims must be 1..8");
    if (n < 0 || n >= (int64_t(1) << 40)) return fail(TP_ERANGE, "n out of range");
    if (ld < n) return fail(TP_EINVAL, "ld < n");
    if (ncols != 32 && ncols != 64 && ncols != 128) return fail(TP_EINVAL, "ncols must be 32, 64 or 128");
    if (nrow < 0 || nrow > tpe::MAXR) return fail(TP_ERANGE, "nrow must be 0..3");
    if ((reinterpret_cast<uintptr_t>(cols) & 15u) != 0) return fail(TP_EINVAL, "cols must be 16-byte aligned");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(TP_EINVAL, "sigma must be positive and finite");
    tpe::EParams p;
    std::memset(&p, 0, sizeof p);
    if (n < 2) return TP_OK;
    p.Y = coords;
    p.ldY = ld;
    p.n = n;
    p.D = dims;
    p.C = ncols;
    p.R = nrow;
    // psi = exp(-d^2 / (2 sigma^2)) = 2^-(yscale d)^2
    p.yscale = (float)std::sqrt(1.4426950408889634 / (2.0 * sigma * sigma));
    p.G = cols;
    p.sums = sums;
    {
        int dev = 0;
        TP_HIP(hipGetDevice(&dev));
        std::lock_guard<std::mutex> lk(g_mu);
        Device &d = device(dev);
        const hipStream_t st = static_cast<hipStream_t>(stream);
        uint32_t *&f = d.eflag[st];
        if (!f) {
            // zero once; each launch that sets the flag clears it when done
            if (hipMalloc(&f, 2 * sizeof(uint32_t)) != hipSuccess) {
                d.eflag.erase(st);
                return fail(TP_ENOMEM, "flag allocation failed");
            }
            TP_HIP(hipMemset(f, 0, 2 * sizeof(uint32_t)));
        }
        p.flag = f;
    }
    TP_HIP(tpe::launch_pairsums(p, static_cast<hipStream_t>(stream)));
    return TP_OK;
}

int tp_energy_eq2(const double *sums, int32_t ncols, int32_t nrow, int32_t ones_row, int32_t ones_col,
                  const int64_t *nx, int64_t n, double *T)
{
    if (!sums || !nx || !T) return fail(TP_EINVAL, "null pointer");
    if (ncols < 1 || nrow < 1 || ones_row < 0 || ones_row >= nrow || ones_col < 0 || ones_col >= ncols)
        return fail(TP_EINVAL, "bad column or row index");
    const int w = 1 + nrow;
    const double tot = sums[(int64_t)ones_col * w + 1 + ones_row];     // sum over i != j of psi
    for (int c = 0; c < ncols; ++c) {
        const double q = sums[(int64_t)c * w];                         // both in X, ordered
        const double r = sums[(int64_t)c * w + 1 + ones_row];          // j in X, i anywhere
        const double a = (double)nx[c], b = (double)(n - nx[c]);
        if (nx[c] < 2 || n - nx[c] < 2) {
            T[c] = NAN;
            continue;
        }
        const double sxx = 0.5 * q, sbb = 0.5 * (tot - 2.0 * r + q), sxb = r - q;
        T[c] = sxx / (a * (a - 1.0)) + sbb / (b * (b - 1.0)) - sxb / (a * b);
    }
    return TP_OK;
}

int tp_energy_eq3(const double *sums, int32_t ncols, int32_t nrow, int32_t col_main, int32_t col_bkg,
                  int32_t row_main, int32_t row_bkg, const int32_t *perm_cols, int32_t nperm, int64_t n_main,
                  int64_t n_main_bar, int64_t n_bkg, int64_t n_bkg_bar, double b, double b_bar, double *T)
{
    if (!sums || !perm_cols || !T) return fail(TP_EINVAL, "null pointer");
    if (col_main < 0 || col_main >= ncols || col_bkg < 0 || col_bkg >= ncols || row_main < 0 || row_main >= nrow ||
        row_bkg < 0 || row_bkg >= nrow || nperm < 0)
        return fail(TP_EINVAL, "bad column or row index");
    const int w = 1 + nrow;
    auto at = [&](int c, int q) { return sums[(int64_t)c * w + q]; };
    const double Smm = at(col_main, 1 + row_main), Smk = at(col_bkg, 1 + row_main), Skk = at(col_bkg, 1 + row_bkg);
    const double ws = (double)n_main - b, wsb = (double)n_main_bar - b_bar;
    const double bs = (double)n_bkg, bsb = (double)n_bkg_bar;
    for (int k = 0; k < nperm; ++k) {
        const int ca = perm_cols[3 * k], cb = perm_cols[3 * k + 1], cg = perm_cols[3 * k + 2];
        if (ca < 0 || ca >= ncols || cb < 0 || cb >= ncols || cg < 0 || cg >= ncols)
            return fail(TP_EINVAL, "permutation column out of range");
        // ordered-pair sums (j != i) between the four samples, from the column sums:
        // a = main X, abar = main - a, beta = bkg X, betabar = bkg - beta, gamma = a + beta
        const double Saa = at(ca, 0), Sbb = at(cb, 0);
        const double Sab = 0.5 * (at(cg, 0) - Saa - Sbb);
        const double Sam = at(ca, 1 + row_main), Sak = at(ca, 1 + row_bkg);
        const double Sbm = at(cb, 1 + row_main), Sbk = at(cb, 1 + row_bkg);
        const double main_x = Saa, main_xb = Smm - 2.0 * Sam + Saa;
        const double bkg_x = Sbb, bkg_xb = Skk - 2.0 * Sbk + Sbb;
        const double mx_bx = Sab;                                  // main X with bkg X
        const double mxb_bxb = Smk - Sbm - Sak + Sab;              // main Xbar with bkg Xbar
        const double mx_mxb = Sam - Saa;                           // main X with main Xbar
        const double mx_bxb = Sak - Sab;                           // main X with bkg Xbar
        const double bx_mxb = Sbm - Sab;                           // bkg X with main Xbar
        const double bx_bxb = Sbk - Sbb;                           // bkg X with bkg Xbar
        const double t1 = (main_x - 2.0 * b / bs * mx_bx + b * (b + 1.0) / (bs * (bs - 1.0)) * bkg_x) /
                          (2.0 * ws * (ws - 1.0));
        const double t2 = (main_xb - 2.0 * b_bar / bsb * mxb_bxb + b_bar * (b_bar + 1.0) / (bsb * (bsb - 1.0)) * bkg_xb) /
                          (2.0 * wsb * (wsb - 1.0));
        const double t3 = (mx_mxb - b_bar / bsb * mx_bxb - b / bs * bx_mxb + b * b_bar / (bs * bsb) * bx_bxb) / (ws * wsb);
        T[k] = t1 + t2 - t3;
    }
    return TP_OK;
}

}  // extern "C"
