// capi.hip -- host side of the C ABI declared in include/flipmc.h.
//
// Validates parameters, lays the system out in the caller's device buffer,
// fills the device descriptor (SysDev) and enqueues the kernels of
// kernels.hip on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "engine.h"
#include "flipmc.h"

using namespace flipmc;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

namespace flipmc {

int api_error(int code, const char* msg)
{
    g_err = msg;
    return code;
}

size_t device_lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 163840;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0) {
        (void)hipGetLastError();
        return 163840;
    }
    return (size_t)v;
}

}  // namespace flipmc

namespace {

// A named range on the host timeline of a profiler that records roctx
// markers (rocprofv3 --marker-trace): one per API call that enqueues work,
// one per launch of sweeps or events inside it.
struct TraceRange {
    explicit TraceRange(const char* what) { roctxRangePushA(what); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

#define HIPCHK(x)                                                                       \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) return fail(MC_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

// Side of the rigid triangle: the minimum of WCA + FENE (Eq. 1 + Eq. 2) of a
// sigma_ij = 1 bond, found by Newton's method on the slope.
double bond_star()
{
    auto slope = [](double x) {
        return -48.0 * std::pow(x, -13.0) + 24.0 * std::pow(x, -7.0) +
               30.0 * x / (1.0 - x * x / 2.25);
    };
    auto curvature = [](double x) {
        const double d = 1.0 - x * x / 2.25;
        return 624.0 * std::pow(x, -14.0) - 168.0 * std::pow(x, -8.0) +
               30.0 / d + 30.0 * x * (2.0 * x / 2.25) / (d * d);
    };
    double x = 0.96;
    for (int it = 0; it < 100; ++it) {
        const double nx = x - slope(x) / curvature(x);
        if (nx == x) break;
        x = nx;
    }
    return x;
}

struct Geometry {
    double L, bond, radius, reach;
    uint32_t k, nc, ncell;
    bool resident;
    bool spread;          // standalone sweeps on the multi-workgroup engine
    uint32_t spread_blocks;  // its workgroups (also of an LDS system a batch may move there)
    size_t lds;
    double sweep_cost;    // modelled cycles of one sweep on one workgroup
    double spread_cost;   // the same with the state in HBM (the multi-workgroup engine's unit)
};

// Critical path of one sweep of the resident kernel in cycles (a model fitted
// to measured per-cell and per-trial costs): k^3 colour phases; in each, the
// busiest wave builds the neighbour list of each of its cells and runs the
// cell's trials one after another.
double cost_estimate(uint32_t M, double L, double reach, uint32_t k, uint32_t nc)
{
    const double ncell = (double)nc * nc * nc;
    const double per_cell = (double)M / ncell;
    const double w = L / nc;
    const double na3 = std::pow((double)(nc / k), 3.0);
    const double cells_per_wave = std::ceil(na3 / kWaves);
    const double span = std::min((double)nc, 2.0 * (k - 1) + 1.0);
    const double stencil = std::min((double)M, span * span * span * per_cell);
    const double region = 0.75 * std::pow(w + 2.0 * reach, 3.0) * (double)M / (L * L * L);
    const double listed = std::min(stencil, region);
    const double t_list = 300.0 + 20.0 * stencil;
    const double t_trial = 1800.0 + 12.0 * listed;
    return (double)k * k * k * (cells_per_wave * (t_list + std::max(1.0, per_cell) * t_trial) + 300.0);
}

// Initial milliseconds per modelled cycle of the engine classes (one
// workgroup with the state in LDS, in HBM; the multi-workgroup engine per
// workgroup), relative to the LDS class; a batch then measures its own.
// The multi-workgroup engine moves about 2.9 times fewer molecules per
// workgroup than an LDS workgroup (1728 molecules on 7 workgroups, 8000 on
// 32), 2.2 per modelled cycle of its HBM cost; 2.5 keeps a margin.
constexpr double kCycleRatio[3] = {1.0, 1.3, 2.5};

// Whether the multi-workgroup engine on nb workgroups is modelled at least
// 25 % faster than the system's own engine on one workgroup, with ms_one and
// ms_multi the milliseconds per modelled cycle of the two (always, for a
// system beyond one workgroup's LDS).
bool spread_pays(const Geometry& g, uint32_t nb, double ms_one, double ms_multi)
{
    return !g.resident || (double)nb * g.sweep_cost * ms_one >= 1.25 * g.spread_cost * ms_multi;
}

int geometry(const mc_params* p, Geometry* g)
{
    if (!p) return fail(MC_EINVAL, "null parameters");
    if (p->n_molecules < 1 || p->n_molecules > (uint32_t)kMaxMolecules)
        return fail(MC_EINVAL, "n_molecules must be in [1, %d]", kMaxMolecules);
    if (p->precision != MC_FP64 && p->precision != MC_FP32_DE)
        return fail(MC_EINVAL, "precision must be MC_FP64 or MC_FP32_DE");
    if (!(p->density > 0) || !(p->temperature > 0))
        return fail(MC_EINVAL, "density and temperature must be positive");
    for (int i = 0; i < 3; ++i)
        if (!(p->sigma[i] > 0)) return fail(MC_EINVAL, "sigma must be positive");
    if (!(p->p_flip >= 0) || !(p->p_translate >= 0) || p->p_flip + p->p_translate > 1.0)
        return fail(MC_EINVAL, "move probabilities out of range");
    if (!(p->max_displacement >= 0) || !(p->max_rotation >= 0))
        return fail(MC_EINVAL, "step sizes must be non-negative");
    if (!(p->gofr_dr > 0)) return fail(MC_EINVAL, "gofr_dr must be positive");
    if (!(p->fs_q >= 0) || !(p->fs_q_cm >= 0)) return fail(MC_EINVAL, "fs_q and fs_q_cm must be >= 0");
    g->L = std::cbrt(3.0 * (double)p->n_molecules / p->density);
    g->bond = p->bond_length > 0 ? p->bond_length : bond_star();
    g->radius = g->bond / std::sqrt(3.0);
    const double smax = std::max(p->sigma[0], std::max(p->sigma[1], p->sigma[2]));
    const double rcmax = std::pow(2.0, 1.0 / 6.0) * smax;
    g->reach = rcmax + 2.0 * g->radius;
    // Pair terms are formed from the nearest image of the two centres plus the
    // site offsets.  That is the nearest image of every interacting site pair
    // only when no molecule reaches another through two images: L >= 2 reach.
    if (g->L < 2.0 * (g->reach + 2.0 * p->max_displacement))
        return fail(MC_EGEOM, "box side %.4f below twice the interaction reach %.4f (minimum image)",
                    g->L, g->reach + 2.0 * p->max_displacement);
    uint32_t k = p->colours_per_axis, nc = p->cells_per_side;
    if (k == 0 && nc == 0) {
        double best = std::numeric_limits<double>::infinity();
        for (uint32_t kk = 2; kk <= 3; ++kk) {
            uint32_t n = (uint32_t)std::floor((kk - 1) * g->L / g->reach);
            n -= n % kk;
            while (n >= 2 && std::pow((double)n, 3.0) > 65535.0) n -= kk;
            if (n < 2 || n < kk) continue;
            const double c = cost_estimate(p->n_molecules, g->L, g->reach, kk, n);
            if (c < best) {
                best = c;
                k = kk;
                nc = n;
            }
        }
        if (k == 0) return fail(MC_EGEOM, "no checkerboard fits a box of side %.4f", g->L);
    } else if (k == 0 || nc == 0) {
        return fail(MC_EINVAL, "give both colours_per_axis and cells_per_side, or neither");
    }
    if (k < 2 || k > 3) return fail(MC_EGEOM, "colours_per_axis must be 2 or 3");
    if (nc < 2 || nc % k != 0) return fail(MC_EGEOM, "cells_per_side must be a multiple of k >= 2");
    if ((double)(k - 1) * (g->L / (double)nc) < g->reach)
        return fail(MC_EGEOM, "(k-1) * cell width %.5f is below the interaction reach %.5f",
                    (double)(k - 1) * g->L / nc, g->reach);
    const double ncell = (double)nc * nc * nc;
    if (ncell > 65535.0) return fail(MC_EGEOM, "too many cells (%u per side)", nc);
    g->k = k;
    g->nc = nc;
    g->ncell = nc * nc * nc;
    const bool fp64 = p->precision == MC_FP64;
    const size_t limit = device_lds_limit();
    const LdsLayout res = lds_layout(fp64, true, p->n_molecules, g->ncell);
    g->resident = res.total <= limit && !(p->flags & MC_FLAG_HBM_STATE);
    g->lds = g->resident ? res.total : lds_layout(fp64, false, p->n_molecules, g->ncell).total;
    const bool one_wg = (p->flags & MC_FLAG_SINGLE_WORKGROUP) || p->workgroups == 1;
    g->spread = !g->resident && !one_wg;
    g->spread_blocks = 1;
    // the model is fitted to the LDS state; with the state in HBM a sweep on
    // one workgroup takes about 1.3 times as long (measured 1.1 - 1.4 over
    // 2197 - 27000 molecules)
    const double cost = cost_estimate(p->n_molecules, g->L, g->reach, k, nc);
    g->sweep_cost = cost * (g->resident ? 1.0 : 1.3);
    g->spread_cost = cost * 1.3;
    if (!one_wg) {
        // one wave per cell of a colour, within one cooperative wave of the
        // device.  A system whose state fits one workgroup's LDS runs alone on
        // the multi-workgroup engine too when that is modelled faster (many
        // cells per colour) or when the caller asks for a workgroup count;
        // otherwise it keeps the count for a batch, which may move it there
        // when compute units are idle
        uint32_t maxb = 0;
        const hipError_t e = spread_max_blocks(fp64, &maxb);
        if (e != hipSuccess || maxb == 0) {
            (void)hipGetLastError();
            g->spread = false;
        } else {
            const uint32_t na = nc / k;
            const uint32_t want = (na * na * na + kSpreadWaves - 1) / kSpreadWaves;
            g->spread_blocks = std::max(1u, std::min({want, maxb, (uint32_t)(kMaxParts / kSpreadWaves)}));
            if (p->workgroups >= 2) {
                g->spread_blocks = std::min(g->spread_blocks, p->workgroups);
                if (g->spread_blocks >= 2) g->spread = true;
            } else if (g->resident && g->spread_blocks >= 2 &&
                       spread_pays(*g, g->spread_blocks, kCycleRatio[0], kCycleRatio[2])) {
                g->spread = true;
            }
        }
    }
    return MC_OK;
}

// Modelled cycles of a time slice of max_moves moves of the 1000-molecule
// reference system (k = 2, n_c = 4) on one workgroup.
double slice_time(uint64_t max_moves)
{
    static const double ref = [] {
        const double L = std::cbrt(3.0 * 1000.0 / 1.2);
        const double reach = std::pow(2.0, 1.0 / 6.0) * 1.1 + 2.0 * bond_star() / std::sqrt(3.0);
        return cost_estimate(1000, L, reach, 2, 4);
    }();
    return (double)max_moves / 1000.0 * ref;
}

// Milliseconds per modelled cycle on an idle device: a sweep of the
// 1000-molecule reference (k = 2, n_c = 4) takes about 0.31 ms on one
// workgroup with the state in LDS.
double ms_per_model_cycle()
{
    return 0.31 / slice_time(1000);
}

// Workgroups of the multi-workgroup event kernel for M molecules (one
// molecule per thread of the O(M^2) loops), 1 = single-workgroup events.
uint32_t event_blocks(uint32_t M)
{
    if (M < 2048) return 1;
    return std::min((uint32_t)kMaxParts, (M + kThreads - 1) / kThreads);
}

struct BufLayout {
    size_t sys, stats, com, quat, types, u0, kref, esamp, dsamp, gall, ginter, c2, c2s;
    size_t img, r0, o0, fs, fscm, mom;
    size_t props, gpart, gsite, gcell, gcellid, glist, gcnt, gecell, gbar, total;
};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

BufLayout buf_layout(const mc_params* p, const Geometry& g)
{
    BufLayout b{};
    const size_t M = p->n_molecules;
    size_t o = 0;
    b.sys = o;    o = al(o + sizeof(SysDev));
    b.stats = o;  o = al(o + sizeof(Stats));
    b.com = o;    o = al(o + 3 * M * sizeof(double));
    b.quat = o;   o = al(o + 4 * M * sizeof(double));
    b.types = o;  o = al(o + M * sizeof(uint32_t));
    b.u0 = o;     o = al(o + 3 * M * sizeof(double));
    b.kref = o;   o = al(o + M);
    b.esamp = o;  o = al(o + size_t(p->max_samples) * sizeof(double));
    b.dsamp = o;  o = al(o + size_t(p->max_samples) * sizeof(double));
    b.gall = o;   o = al(o + kGofrBins * sizeof(uint64_t));
    b.ginter = o; o = al(o + kGofrBins * sizeof(uint64_t));
    b.c2 = o;     o = al(o + kC2Max * sizeof(double));
    b.c2s = o;    o = al(o + kC2Max * sizeof(uint64_t));
    b.img = o;    o = al(o + 3 * M * sizeof(int32_t));
    b.r0 = o;     o = al(o + 3 * M * sizeof(double));
    b.o0 = o;     o = al(o + 9 * M * sizeof(double));
    b.fs = o;     o = al(o + kC2Max * sizeof(double));
    b.fscm = o;   o = al(o + kC2Max * sizeof(double));
    b.mom = o;    o = al(o + 4 * kC2Max * sizeof(double));
    b.props = o;  o = al(o + M * 48);
    b.gpart = o;  o = al(o + kMaxParts * sizeof(double));
    if (!g.resident || g.spread_blocks >= 2) {
        const bool fp64 = p->precision == MC_FP64;
        b.gsite = o;   o = al(o + 3 * M * site_bytes(fp64));
        b.gcell = o;   o = al(o + (size_t(g.ncell) + 1) * sizeof(uint32_t));
        b.gcellid = o; o = al(o + M * sizeof(uint16_t));
        b.glist = o;   o = al(o + M * sizeof(uint16_t));
        b.gcnt = o;    o = al(o + 2 * size_t(g.ncell) * sizeof(uint32_t));
        b.gecell = o;  o = al(o + size_t(g.ncell) * sizeof(double));
        b.gbar = o;    o = al(o + sizeof(uint32_t));
    }
    b.total = o;
    return b;
}

}  // namespace

struct mc_system {
    mc_params p;
    Geometry g;
    BufLayout lay;
    SysDev host;
    SysDev* dev;
    uint8_t* buf;
    hipStream_t stream;
    uint64_t sweep;   // host mirror of the device sweep counter
    uint64_t origin;  // host mirror of the observable origin
    mc_batch* batch;
    // launch timing (mc_timing_enable)
    bool timing;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_sweep, ev_event;
};

struct mc_batch {
    uint32_t max_slots;
    uint32_t precision;
    hipStream_t stream;
    std::vector<mc_system*> sys;
    std::vector<uint64_t> remaining;
    Slot* dev_slots[2];   // per parity: [resident | non-resident | events] x max_slots
    Slot* host_slots[2];
    hipEvent_t copied[2];
    bool pending[2];
    int parity;
    // systems on the multi-workgroup engine: one cooperative launch per run on
    // stream2, overlapping the batch stream's launches
    hipStream_t stream2;              // caller's second stream (or the batch stream)
    hipEvent_t go, done;              // stream2 waits for go (stream), stream for done (stream2)
    // systems on one workgroup with the state in HBM: their launch on stream3
    // (a third caller stream) runs beside the LDS class's launch on stream;
    // nullptr = after it on stream
    hipStream_t stream3;
    hipEvent_t go3, done3;            // stream3 waits for go3 (stream), stream for done3 (stream3)
    SpreadSlot* dev_spread[2];        // per parity: [systems | (events as Slot)] x max_slots
    SpreadSlot* host_spread[2];
    Slot* dev_ev2[2];
    Slot* host_ev2[2];
    hipEvent_t copied2[2];
    bool pending2[2];
    uint32_t spread_max;              // co-resident workgroups of the cooperative launch
    uint32_t ncu;                     // compute units of the device
    uint32_t wg_limit;                // compute units the batch's runs use at once
    uint32_t turn;                    // where the next run starts taking systems when
                                      // there are more than wg_limit
    // slice calibration per engine class (one workgroup with the state in LDS,
    // one workgroup with the state in HBM, multi-workgroup): milliseconds per
    // modelled cycle, learnt from the timed launches of earlier runs
    double ms_per_cycle[3];
    double pred[3];                   // modelled cycles of the class's last launch (0: none)
    hipEvent_t t_beg[3], t_end[3];
};

namespace {

// A system inside a batch is advanced on the batch's stream: wait for it
// before reading the system's state on its own stream.
int sync_owner(mc_system* s)
{
    if (s->batch) HIPCHK(hipStreamSynchronize(s->batch->stream));
    return MC_OK;
}

int upload_desc(mc_system* s)
{
    HIPCHK(hipMemcpyAsync(s->dev, &s->host, sizeof(SysDev), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return MC_OK;
}

hipEvent_t take_event(mc_system* s)
{
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Record a start event when timing is on (nullptr otherwise).
hipEvent_t timing_start(mc_system* s)
{
    if (!s->timing) return nullptr;
    hipEvent_t a = take_event(s);
    if (a && hipEventRecord(a, s->stream) != hipSuccess) return nullptr;
    return a;
}

void timing_stop(mc_system* s, hipEvent_t a, bool sweep_kernel)
{
    if (!a) return;
    hipEvent_t b = take_event(s);
    if (!b || hipEventRecord(b, s->stream) != hipSuccess) return;
    (sweep_kernel ? s->ev_sweep : s->ev_event).emplace_back(a, b);
}

int launch_events_one(mc_system* s, uint32_t flags)
{
    TraceRange tr((flags & (kFlagResumSet | kFlagResumReport | kFlagResumPeriodic)) ? "flipmc events: FP64 re-sum"
                                                                                    : "flipmc events");
    Slot one{};
    one.sys = s->dev;
    one.flags = flags;
    hipEvent_t t0 = timing_start(s);
    const uint32_t nb = event_blocks(s->p.n_molecules);
    if (nb > 1 && (flags & (kFlagResumSet | kFlagResumReport | kFlagResumPeriodic | kFlagGofr))) {
        // the O(M^2) re-sum and g(r) frame on many workgroups, then the rest
        PartList pl{};
        pl.s[0] = PartSlot{s->dev, flags, 0u, nb, 0u};
        pl.n = 1;
        HIPCHK(launch_event_parts(pl, nb, s->stream));
        one.flags = flags | kFlagParts;
        one.pad = nb;
    }
    HIPCHK(launch_events(nullptr, one, 1, s->stream));
    timing_stop(s, t0, false);
    return MC_OK;
}

bool is_c2_time(uint64_t t)
{
    if (t == 0) return false;
    while (t % 10 == 0) t /= 10;
    return t == 1 || t == 2 || t == 5;
}

// Event work due right after sweep `sweep` of system s.
uint32_t events_at(const mc_system* s, uint64_t sweep)
{
    uint32_t f = 0;
    const mc_params& p = s->p;
    if (p.resum_interval && sweep % p.resum_interval == 0) f |= kFlagResumPeriodic;
    const uint64_t t = sweep - s->origin;
    if (p.gofr_interval && t >= p.obs_start && t % p.gofr_interval == 0) f |= kFlagGofr;
    if (is_c2_time(t)) f |= kFlagC2;
    return f;
}

// First sweep after s->sweep at which some event work is due (only g(r)
// frames when the sweep kernel takes the re-sums and C_2 samples itself).
uint64_t next_event(const mc_system* s, bool gofr_only = false)
{
    const mc_params& p = s->p;
    const uint64_t now = s->sweep;
    uint64_t best = UINT64_MAX;
    if (p.resum_interval && !gofr_only)
        best = std::min(best, (now / p.resum_interval + 1) * p.resum_interval);
    const uint64_t t = now - s->origin;
    if (p.gofr_interval) {
        uint64_t n = (t / p.gofr_interval + 1) * p.gofr_interval;
        if (n < p.obs_start) n = ((p.obs_start + p.gofr_interval - 1) / p.gofr_interval) * p.gofr_interval;
        best = std::min(best, s->origin + n);
    }
    for (uint64_t dec = 1; !gofr_only && dec <= (uint64_t)1e18; dec *= 10) {
        bool found = false;
        for (uint64_t m : {1ull, 2ull, 5ull}) {
            if (m * dec > t) {
                best = std::min(best, s->origin + m * dec);
                found = true;
                break;
            }
        }
        if (found) break;
    }
    return best;
}

constexpr uint64_t kMaxSweepsPerLaunch = 1u << 16;

// Zero a system's barrier counter with a kernel, not a memset: mc_sweep stays
// free of memset nodes for callers that capture it into a graph.
__global__ void k_zero_counter(uint32_t* c)
{
    if (threadIdx.x == 0) *c = 0u;
}

// Enqueue n sweeps of one system, split at event sweeps.
int advance(mc_system* s, uint64_t n)
{
    Slot one{};
    one.sys = s->dev;
    while (n > 0) {
        // at most kMaxSweepsPerLaunch sweeps per launch (a bounded kernel time)
        const uint64_t chunk = std::min<uint64_t>({n, next_event(s) - s->sweep, kMaxSweepsPerLaunch});
        one.n_sweeps = chunk;
        one.flags = 0;
        TraceRange tr(s->g.spread ? "flipmc sweeps: multi-workgroup launch" : "flipmc sweeps: one-workgroup launch");
        if (s->g.spread) {
            hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s->stream, s->host.g_bar);
            HIPCHK(hipGetLastError());
        }
        hipEvent_t t0 = timing_start(s);
        if (s->g.spread) {
            SpreadSlot sl{};
            sl.sys = s->dev;
            sl.n_sweeps = chunk;
            sl.first_block = 0;
            sl.n_blocks = s->g.spread_blocks;
            HIPCHK(launch_spread(s->p.precision == MC_FP64, nullptr, 1, sl, s->g.spread_blocks,
                                 s->stream));
        }
        else
            HIPCHK(launch_sweeps(s->p.precision == MC_FP64, s->g.resident, nullptr, one, 1,
                                 s->g.lds, s->stream));
        timing_stop(s, t0, true);
        s->sweep += chunk;
        n -= chunk;
        const uint32_t f = events_at(s, s->sweep);
        if (f) {
            const int rc = launch_events_one(s, f);
            if (rc) return rc;
        }
    }
    return MC_OK;
}

int read_stats(mc_system* s, Stats* st)
{
    if (int rc = sync_owner(s)) return rc;
    HIPCHK(hipMemcpyAsync(st, s->host.stats, sizeof(Stats), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (st->fault)
        return fail(MC_EDEVICE, "a workgroup barrier of the multi-workgroup engine timed out: "
                                "the system's state is invalid");
    return MC_OK;
}

int write_stats(mc_system* s, const Stats* st)
{
    HIPCHK(hipMemcpyAsync(s->host.stats, st, sizeof(Stats), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return MC_OK;
}

int upload_state(mc_system* s, const double* com, const double* quat, const uint8_t* types)
{
    const size_t M = s->p.n_molecules;
    std::vector<double> c(3 * M), q(4 * M);
    std::vector<uint32_t> t(M);
    for (size_t m = 0; m < M; ++m) {
        for (int a = 0; a < 3; ++a) c[a * M + m] = com[3 * m + a];
        double nrm = 0;
        for (int a = 0; a < 4; ++a) nrm += quat[4 * m + a] * quat[4 * m + a];
        if (!(std::fabs(nrm - 1.0) < 1e-6))
            return fail(MC_EINVAL, "quaternion of molecule %zu is not a unit quaternion", m);
        for (int a = 0; a < 4; ++a) q[a * M + m] = quat[4 * m + a];
        const uint8_t a0 = types[3 * m], a1 = types[3 * m + 1], a2 = types[3 * m + 2];
        if (a0 > 2 || a1 > 2 || a2 > 2 || a0 == a1 || a0 == a2 || a1 == a2)
            return fail(MC_EINVAL, "types of molecule %zu are not a permutation of A, B, C", m);
        t[m] = (uint32_t)a0 | ((uint32_t)a1 << 8) | ((uint32_t)a2 << 16);
    }
    HIPCHK(hipMemcpyAsync(s->host.com, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->host.quat, q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->host.types, t.data(), t.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return MC_OK;
}

// The event work over many workgroups of several systems: one launch per
// kPartSlots systems, each system on its own event_blocks() workgroups.
hipError_t launch_parts_of(const std::vector<std::pair<mc_system*, uint32_t>>& parts,
                                  hipStream_t stream)
{
    for (size_t i0 = 0; i0 < parts.size(); i0 += kPartSlots) {
        PartList pl{};
        uint32_t blocks = 0;
        for (size_t i = i0; i < std::min(parts.size(), i0 + kPartSlots); ++i) {
            const uint32_t nb = event_blocks(parts[i].first->p.n_molecules);
            pl.s[pl.n++] = PartSlot{parts[i].first->dev, parts[i].second, blocks, nb, 0u};
            blocks += nb;
        }
        const hipError_t e = launch_event_parts(pl, blocks, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

const char* mc_last_error(void) { return g_err.c_str(); }

void mc_params_default(mc_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->n_molecules = 1000;
    p->precision = MC_FP64;
    p->density = 1.2;
    p->temperature = 3.0;
    p->sigma[0] = 0.9;
    p->sigma[1] = 1.0;
    p->sigma[2] = 1.1;
    p->bond_length = 0.0;
    p->p_flip = 0.2;
    p->p_translate = 0.4;
    p->max_displacement = 0.1;
    p->max_rotation = 0.2;
    p->seed = 1;
    p->colours_per_axis = 0;
    p->cells_per_side = 0;
    p->resum_interval = 100;
    p->obs_interval = 10;
    p->gofr_interval = 100;
    p->obs_start = 0;
    p->max_samples = 4096;
    p->gofr_dr = 0.02;
    p->barrier_polls = 0;
    p->fs_q = 7.4;     // first peak of the site structure factor (Sec. III.B)
    p->fs_q_cm = 5.1;  // first peak of the centres' structure factor
    p->workgroups = 0;
}

int mc_geometry(const mc_params* p, double* box, uint32_t* k, uint32_t* nc)
{
    Geometry g;
    const int rc = geometry(p, &g);
    if (rc) return rc;
    if (box) *box = g.L;
    if (k) *k = g.k;
    if (nc) *nc = g.nc;
    return MC_OK;
}

int mc_placement(const mc_params* p, int* resident, size_t* lds_bytes)
{
    Geometry g;
    const int rc = geometry(p, &g);
    if (rc) return rc;
    if (resident) *resident = g.resident ? 1 : 0;
    if (lds_bytes) *lds_bytes = g.lds;
    return MC_OK;
}

int mc_engine(const mc_params* p, int* engine, uint32_t* workgroups)
{
    Geometry g;
    const int rc = geometry(p, &g);
    if (rc) return rc;
    if (engine) *engine = g.spread ? MC_ENGINE_SPREAD : (g.resident ? MC_ENGINE_LDS : MC_ENGINE_HBM);
    if (workgroups) *workgroups = g.spread ? g.spread_blocks : 1u;
    return MC_OK;
}

int mc_required_bytes(const mc_params* p, size_t* bytes)
{
    Geometry g;
    const int rc = geometry(p, &g);
    if (rc) return rc;
    if (!bytes) return fail(MC_EINVAL, "null output");
    *bytes = buf_layout(p, g).total;
    return MC_OK;
}

int mc_init_system(const mc_params* p, const double* com, const double* quat, const uint8_t* types,
                   void* device_buf, size_t buf_bytes, void* hip_stream, mc_system** out)
{
    if (!out) return fail(MC_EINVAL, "null output handle");
    *out = nullptr;
    Geometry g;
    int rc = geometry(p, &g);
    if (rc) return rc;
    const bool lattice = !com && !quat && !types;
    if (!lattice && !(com && quat && types))
        return fail(MC_EINVAL, "give com, quat and types together, or none of them");
    if (lattice) {
        uint32_t n = 1;
        while ((n + 1) * (n + 1) * (n + 1) <= p->n_molecules) ++n;
        if (n * n * n != p->n_molecules)
            return fail(MC_EINVAL, "lattice start needs n_molecules = n^3 (got %u)", p->n_molecules);
    }
    if (!device_buf) return fail(MC_EINVAL, "null device buffer");
    if (((uintptr_t)device_buf & 255u) != 0) return fail(MC_EINVAL, "device buffer must be 256-byte aligned");
    const BufLayout lay = buf_layout(p, g);
    if (buf_bytes < lay.total)
        return fail(MC_ENOMEM, "device buffer of %zu bytes, %zu needed", buf_bytes, lay.total);

    mc_system* s = new mc_system();
    s->p = *p;
    s->g = g;
    s->lay = lay;
    s->buf = (uint8_t*)device_buf;
    s->stream = (hipStream_t)hip_stream;
    s->sweep = 0;
    s->batch = nullptr;
    s->timing = false;
    SysDev& D = s->host;
    std::memset(&D, 0, sizeof D);
    uint8_t* b = s->buf;
    D.M = p->n_molecules;
    D.k = g.k;
    D.nc = g.nc;
    D.ncell = g.ncell;
    D.precision = p->precision;
    D.resident = g.resident ? 1u : 0u;
    D.seed_lo = (uint32_t)p->seed;
    D.seed_hi = (uint32_t)(p->seed >> 32);
    D.L = g.L;
    D.w = g.L / (double)g.nc;
    D.T = p->temperature;
    D.p_flip = p->p_flip;
    D.p_ft = p->p_flip + p->p_translate;
    D.dmax = p->max_displacement;
    D.rot_max = p->max_rotation;
    const double reach = g.reach * (1.0 + 1e-9);
    D.reach2 = reach * reach;
    D.radius = g.radius;
    D.rc2_factor = std::cbrt(2.0);
    const double body[9] = {g.radius, 0.0, 0.0, -0.5 * g.radius, 0.5 * g.bond, 0.0,
                            -0.5 * g.radius, -0.5 * g.bond, 0.0};
    std::memcpy(D.body, body, sizeof body);
    for (int i = 0; i < 3; ++i) D.sigma[i] = p->sigma[i];
    D.resum_interval = p->resum_interval;
    D.obs_interval = p->obs_interval;
    D.gofr_interval = p->gofr_interval;
    D.obs_start = p->obs_start;
    D.max_samples = p->max_samples;
    const double rmax = std::min(0.5 * g.L, 5.0);
    uint32_t nb = (uint32_t)std::floor(rmax / p->gofr_dr + 1e-6);
    if (nb > (uint32_t)kGofrBins) nb = kGofrBins;
    D.gofr_nbins = nb;
    D.gofr_dr = p->gofr_dr;
    D.barrier_polls = p->barrier_polls ? p->barrier_polls : (1u << 23);
    D.gofr_rmax = rmax;
    D.lds_bytes = (uint32_t)g.lds;
    D.com = (double*)(b + lay.com);
    D.quat = (double*)(b + lay.quat);
    D.types = (uint32_t*)(b + lay.types);
    D.u0 = (double*)(b + lay.u0);
    D.kref = (uint8_t*)(b + lay.kref);
    D.stats = (Stats*)(b + lay.stats);
    D.e_samples = (double*)(b + lay.esamp);
    D.drift_samples = (double*)(b + lay.dsamp);
    D.gofr_all = (uint64_t*)(b + lay.gall);
    D.gofr_inter = (uint64_t*)(b + lay.ginter);
    D.c2 = (double*)(b + lay.c2);
    D.c2_sweep = (uint64_t*)(b + lay.c2s);
    D.img = (int32_t*)(b + lay.img);
    D.r0 = (double*)(b + lay.r0);
    D.o0 = (double*)(b + lay.o0);
    D.fs = (double*)(b + lay.fs);
    D.fs_cm = (double*)(b + lay.fscm);
    D.mom = (double*)(b + lay.mom);
    D.fs_q = p->fs_q;
    D.fs_q_cm = p->fs_q_cm;
    D.props = (void*)(b + lay.props);
    D.g_part = (double*)(b + lay.gpart);
    if (!g.resident || g.spread_blocks >= 2) {
        D.g_site = (void*)(b + lay.gsite);
        D.g_cell = (uint32_t*)(b + lay.gcell);
        D.g_cellid = (uint16_t*)(b + lay.gcellid);
        D.g_list = (uint16_t*)(b + lay.glist);
        D.g_cnt = (uint32_t*)(b + lay.gcnt);
        D.g_ecell = (double*)(b + lay.gecell);
        D.g_bar = (uint32_t*)(b + lay.gbar);
    }
    s->dev = (SysDev*)(b + lay.sys);

    auto bail = [&](int code) {
        delete s;
        return code;
    };
    hipError_t e = hipMemsetAsync(device_buf, 0, lay.total, s->stream);
    if (e != hipSuccess) return bail(fail(MC_EDEVICE, "hipMemsetAsync: %s", hipGetErrorString(e)));
    if ((rc = upload_desc(s))) return bail(rc);
    if (lattice) {
        e = launch_init_lattice(s->dev, p->n_molecules, s->stream);
        if (e != hipSuccess) return bail(fail(MC_EDEVICE, "lattice kernel: %s", hipGetErrorString(e)));
    } else if ((rc = upload_state(s, com, quat, types))) {
        return bail(rc);
    }
    s->origin = 0;
    if ((rc = launch_events_one(s, kFlagResumSet | kFlagObsReset))) return bail(rc);
    Stats st;
    if ((rc = read_stats(s, &st))) return bail(rc);
    if (!std::isfinite(st.e_acc))
        return bail(fail(MC_ENONFINITE, "initial energy is not finite (overlapping sites)"));
    *out = s;
    return MC_OK;
}

int mc_sweep(mc_system* s, uint64_t n)
{
    TraceRange tr("mc_sweep");
    if (!s) return fail(MC_EINVAL, "null system");
    if (s->batch) return fail(MC_EBUSY, "system is in a batch");
    return advance(s, n);
}

int mc_energy(mc_system* s, double* e_total, double* e_per_molecule, double* drift)
{
    TraceRange tr("mc_energy");
    if (!s) return fail(MC_EINVAL, "null system");
    if (s->batch) return fail(MC_EBUSY, "system is in a batch");
    int rc = launch_events_one(s, kFlagResumReport);
    if (rc) return rc;
    Stats st;
    if ((rc = read_stats(s, &st))) return rc;
    if (e_total) *e_total = st.e_resum;
    if (e_per_molecule) *e_per_molecule = st.e_resum / (double)s->p.n_molecules;
    if (drift) *drift = st.e_acc - st.e_resum;
    if (!std::isfinite(st.e_resum)) return fail(MC_ENONFINITE, "energy is not finite");
    return MC_OK;
}

namespace {

// Eq. (3): g(r) = counts / (frames N rho (4 pi / 3) (r_{b+1}^3 - r_b^3)) with
// N = 3 M sites, rho = N / L^3 and the exact shell volume of bin b.
void gofr_normalise(const mc_system* s, mc_obs* o)
{
    const double N = 3.0 * (double)s->p.n_molecules;
    const double rho = N / (s->g.L * s->g.L * s->g.L);
    const double frames = (double)o->n_gofr_frames;
    const double dr = o->gofr_dr;
    for (uint32_t b = 0; b < o->gofr_nbins && frames > 0.0; ++b) {
        const double r0 = dr * (double)b, r1 = dr * (double)(b + 1);
        const double shell = 4.0 * M_PI / 3.0 * (r1 * r1 * r1 - r0 * r0 * r0);
        const double ideal = frames * N * rho * shell;
        o->gofr_norm_all[b] = (double)o->gofr_all[b] / ideal;
        o->gofr_norm_inter[b] = (double)o->gofr_inter[b] / ideal;
    }
}

}  // namespace

int mc_observables(mc_system* s, mc_obs* o)
{
    if (!s || !o) return fail(MC_EINVAL, "null argument");
    Stats st;
    int rc = read_stats(s, &st);
    if (rc) return rc;
    std::memset(o, 0, sizeof *o);
    o->sweep = st.sweep;
    for (int i = 0; i < 3; ++i) {
        o->attempts[i] = st.attempts[i];
        o->accepts[i] = st.accepts[i];
    }
    o->exits = st.exits;
    o->pair_terms = st.pair_terms;
    o->pair_tests = st.pair_tests;
    o->near_overflows = st.near_overflows;
    o->e_acc = st.e_acc;
    o->e_resum = st.e_resum;
    o->drift = st.drift;
    o->max_abs_drift = st.max_abs_drift;
    o->resum_sweep = st.resum_sweep;
    o->n_energy_samples = st.n_e;
    o->n_drift_samples = st.n_drift;
    o->energy_sum = st.e_sum;
    o->energy_sumsq = st.e_sumsq;
    o->n_gofr_frames = st.n_gofr;
    o->gofr_nbins = s->host.gofr_nbins;
    o->gofr_dr = s->host.gofr_dr;
    o->gofr_rmax = s->host.gofr_rmax;
    o->n_c2 = st.n_c2;
    HIPCHK(hipMemcpyAsync(o->gofr_all, s->host.gofr_all, sizeof o->gofr_all, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(o->gofr_inter, s->host.gofr_inter, sizeof o->gofr_inter, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(o->c2, s->host.c2, sizeof o->c2, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(o->fs, s->host.fs, sizeof o->fs, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(o->fs_cm, s->host.fs_cm, sizeof o->fs_cm, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(o->c2_sq, s->host.mom, sizeof o->c2_sq, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(o->fs_cm_sq, s->host.mom + kC2Max, sizeof o->fs_cm_sq, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(o->c2_fs_cm, s->host.mom + 2 * kC2Max, sizeof o->c2_fs_cm, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(o->fs_sq, s->host.mom + 3 * kC2Max, sizeof o->fs_sq, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(o->c2_sweep, s->host.c2_sweep, sizeof o->c2_sweep, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    gofr_normalise(s, o);
    return MC_OK;
}

int mc_samples(mc_system* s, double* energy, double* drift, size_t cap, size_t* n_energy,
               size_t* n_drift)
{
    if (!s) return fail(MC_EINVAL, "null system");
    Stats st;
    int rc = read_stats(s, &st);
    if (rc) return rc;
    const size_t ne = std::min<size_t>({(size_t)st.n_e, (size_t)s->p.max_samples, cap});
    const size_t nd = std::min<size_t>({(size_t)st.n_drift, (size_t)s->p.max_samples, cap});
    if (energy && ne)
        HIPCHK(hipMemcpyAsync(energy, s->host.e_samples, ne * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (drift && nd)
        HIPCHK(hipMemcpyAsync(drift, s->host.drift_samples, nd * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (n_energy) *n_energy = ne;
    if (n_drift) *n_drift = nd;
    return MC_OK;
}

int mc_reset_observables(mc_system* s)
{
    if (!s) return fail(MC_EINVAL, "null system");
    if (s->batch) return fail(MC_EBUSY, "system is in a batch");
    s->origin = s->sweep;
    return launch_events_one(s, kFlagObsReset);
}

int mc_get_state(mc_system* s, double* com, double* quat, uint8_t* types, uint64_t* sweep,
                 double* e_acc)
{
    if (!s) return fail(MC_EINVAL, "null system");
    const size_t M = s->p.n_molecules;
    std::vector<double> c(3 * M), q(4 * M);
    std::vector<uint32_t> t(M);
    Stats st;
    if (int rc0 = sync_owner(s)) return rc0;
    HIPCHK(hipMemcpyAsync(c.data(), s->host.com, c.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(q.data(), s->host.quat, q.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(t.data(), s->host.types, t.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    int rc = read_stats(s, &st);
    if (rc) return rc;
    for (size_t m = 0; m < M; ++m) {
        if (com)
            for (int a = 0; a < 3; ++a) com[3 * m + a] = c[a * M + m];
        if (quat)
            for (int a = 0; a < 4; ++a) quat[4 * m + a] = q[a * M + m];
        if (types)
            for (int a = 0; a < 3; ++a) types[3 * m + a] = (uint8_t)((t[m] >> (8 * a)) & 0xFFu);
    }
    if (sweep) *sweep = st.sweep;
    if (e_acc) *e_acc = st.e_acc;
    return MC_OK;
}

int mc_set_state(mc_system* s, const double* com, const double* quat, const uint8_t* types,
                 uint64_t sweep, double e_acc)
{
    if (!s || !com || !quat || !types) return fail(MC_EINVAL, "null argument");
    if (s->batch) return fail(MC_EBUSY, "system is in a batch");
    int rc = upload_state(s, com, quat, types);
    if (rc) return rc;
    // the new state has crossed no periodic images yet
    HIPCHK(hipMemsetAsync(s->host.img, 0, 3 * sizeof(int32_t) * s->p.n_molecules, s->stream));
    Stats st;
    if ((rc = read_stats(s, &st))) return rc;
    st.sweep = sweep;
    st.e_acc = std::isnan(e_acc) ? 0.0 : e_acc;
    if (sweep < s->origin) {
        st.obs_origin = sweep;
        s->origin = sweep;
    }
    if ((rc = write_stats(s, &st))) return rc;
    s->sweep = sweep;
    if (std::isnan(e_acc)) {
        if ((rc = launch_events_one(s, kFlagResumSet))) return rc;
        if ((rc = read_stats(s, &st))) return rc;
        if (!std::isfinite(st.e_acc)) return fail(MC_ENONFINITE, "energy of the new state is not finite");
    }
    return MC_OK;
}

int mc_decision_log(mc_system* s, void* device_records, size_t capacity)
{
    if (!s) return fail(MC_EINVAL, "null system");
    if (s->batch) return fail(MC_EBUSY, "system is in a batch");
    Stats st;
    int rc = read_stats(s, &st);
    if (rc) return rc;
    s->host.log = device_records;
    s->host.log_sweep0 = st.sweep;
    s->host.log_sweeps = device_records ? capacity / s->p.n_molecules : 0;
    return upload_desc(s);
}

int mc_timing_enable(mc_system* s, int enable)
{
    if (!s) return fail(MC_EINVAL, "null system");
    HIPCHK(hipStreamSynchronize(s->stream));
    for (auto& pr : s->ev_sweep) { s->ev_pool.push_back(pr.first); s->ev_pool.push_back(pr.second); }
    for (auto& pr : s->ev_event) { s->ev_pool.push_back(pr.first); s->ev_pool.push_back(pr.second); }
    s->ev_sweep.clear();
    s->ev_event.clear();
    s->timing = enable != 0;
    return MC_OK;
}

int mc_timing_read(mc_system* s, double* sweep_ms, uint64_t* sweep_launches, double* event_ms,
                   uint64_t* event_launches)
{
    if (!s) return fail(MC_EINVAL, "null system");
    HIPCHK(hipStreamSynchronize(s->stream));
    double t[2] = {0.0, 0.0};
    const std::vector<std::pair<hipEvent_t, hipEvent_t>>* v[2] = {&s->ev_sweep, &s->ev_event};
    for (int i = 0; i < 2; ++i)
        for (auto& pr : *v[i]) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
            t[i] += ms;
        }
    if (sweep_ms) *sweep_ms = t[0];
    if (sweep_launches) *sweep_launches = s->ev_sweep.size();
    if (event_ms) *event_ms = t[1];
    if (event_launches) *event_launches = s->ev_event.size();
    return MC_OK;
}

void mc_destroy(mc_system* s)
{
    if (!s) return;
    // no kernel of the system may still run when the caller frees its buffer:
    // wait for its own stream and, inside a batch, for the batch's streams
    (void)hipStreamSynchronize(s->stream);
    if (s->batch) {
        (void)hipStreamSynchronize(s->batch->stream);
        if (s->batch->stream2) (void)hipStreamSynchronize(s->batch->stream2);
        if (s->batch->stream3) (void)hipStreamSynchronize(s->batch->stream3);
    }
    for (auto& pr : s->ev_sweep) { s->ev_pool.push_back(pr.first); s->ev_pool.push_back(pr.second); }
    for (auto& pr : s->ev_event) { s->ev_pool.push_back(pr.first); s->ev_pool.push_back(pr.second); }
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->batch) {
        mc_batch* b = s->batch;
        for (size_t i = 0; i < b->sys.size(); ++i)
            if (b->sys[i] == s) b->sys[i] = nullptr;
    }
    delete s;
}

// ------------------------------------------------- analysis of several runs --

namespace {

// First time the samples c[0..n) fall to `level`: linear in ln t between the
// two samples around the crossing; NaN when they never do.
double crossing_time(const uint64_t* t, const double* c, uint32_t n, double level)
{
    for (uint32_t j = 1; j < n; ++j) {
        if (c[j] <= level && level < c[j - 1]) {
            const double x0 = std::log((double)t[j - 1]), x1 = std::log((double)t[j]);
            return std::exp(x0 + (x1 - x0) * (c[j - 1] - level) / (c[j - 1] - c[j]));
        }
    }
    return std::numeric_limits<double>::quiet_NaN();
}

}  // namespace

namespace {

// mc_dynamics and mcf_dynamics: sites = particles of F_s per molecule (the
// susceptibility of F_s counts n M of them).
int dynamics_of(const mc_obs* runs, size_t n_runs, uint32_t n_molecules, uint32_t sites, mc_dyn* out)
{
    if (!runs || !out || n_runs == 0 || n_molecules == 0 || sites == 0) return fail(MC_EINVAL, "bad arguments");
    std::memset(out, 0, sizeof *out);
    const uint32_t n = runs[0].n_c2;
    if (n > MC_C2_MAX) return fail(MC_EINVAL, "n_c2 above %d", MC_C2_MAX);
    for (size_t r = 1; r < n_runs; ++r) {
        if (runs[r].n_c2 != n) return fail(MC_EINVAL, "run %zu has %u samples, run 0 %u", r, runs[r].n_c2, n);
        for (uint32_t j = 0; j < n; ++j)
            if (runs[r].c2_sweep[j] != runs[0].c2_sweep[j])
                return fail(MC_EINVAL, "run %zu samples other sweeps than run 0", r);
    }
    out->n_times = n;
    out->n_runs = (uint32_t)n_runs;
    const double R = (double)n_runs, M = (double)n_molecules;
    for (uint32_t j = 0; j < n; ++j) {
        out->t[j] = runs[0].c2_sweep[j];
        double m[3] = {0, 0, 0}, m2[3] = {0, 0, 0}, sq[3] = {0, 0, 0}, cross = 0.0;
        for (size_t r = 0; r < n_runs; ++r) {
            const mc_obs& o = runs[r];
            const double v[3] = {o.c2[j], o.fs[j], o.fs_cm[j]};
            const double q[3] = {o.c2_sq[j], o.fs_sq[j], o.fs_cm_sq[j]};
            for (int a = 0; a < 3; ++a) {
                m[a] += v[a];
                m2[a] += v[a] * v[a];
                sq[a] += q[a];
            }
            cross += o.c2_fs_cm[j];
        }
        double chi[3], self[3];
        const double npart[3] = {M, (double)sites * M, M};
        for (int a = 0; a < 3; ++a) {
            m[a] /= R;
            chi[a] = npart[a] * (m2[a] / R - m[a] * m[a]);
            self[a] = sq[a] / R - m[a] * m[a];
        }
        out->c2[j] = m[0]; out->fs[j] = m[1]; out->fs_cm[j] = m[2];
        out->chi4_c2[j] = chi[0]; out->chi4_fs[j] = chi[1]; out->chi4_fs_cm[j] = chi[2];
        out->chi4s_c2[j] = self[0]; out->chi4s_fs[j] = self[1]; out->chi4s_fs_cm[j] = self[2];
        out->rho[j] = (cross / R - m[0] * m[2]) / std::sqrt(self[0] * self[2]);
    }
    const double e1 = std::exp(-1.0);
    out->tau_c2 = crossing_time(out->t, out->c2, n, e1);
    out->tau_fs = crossing_time(out->t, out->fs, n, e1);
    out->tau_fs_cm = crossing_time(out->t, out->fs_cm, n, e1);
    return MC_OK;
}

}  // namespace

int mc_dynamics(const mc_obs* runs, size_t n_runs, uint32_t n_molecules, mc_dyn* out)
{
    return dynamics_of(runs, n_runs, n_molecules, 3u, out);
}

int mcf_dynamics(const mc_obs* runs, size_t n_runs, uint32_t n_molecules, uint32_t atoms_per_molecule,
                 mc_dyn* out)
{
    if (atoms_per_molecule < 3 || atoms_per_molecule > 4) return fail(MC_EINVAL, "atoms_per_molecule must be 3 or 4");
    return dynamics_of(runs, n_runs, n_molecules, atoms_per_molecule, out);
}

// ------------------------------------------------------------------ batches --

namespace {

// The batch's device slot tables in the caller's buffer, double-buffered:
// per parity [resident | non-resident | events] x max_slots Slots, max_slots
// SpreadSlots, max_slots Slots of the multi-workgroup engine's events.
struct BatchLayout {
    size_t slots[2], spread[2], ev2[2], total;
};

BatchLayout batch_layout(uint32_t max_slots)
{
    BatchLayout l{};
    size_t o = 0;
    for (int i = 0; i < 2; ++i) {
        l.slots[i] = o;  o = al(o + 3 * sizeof(Slot) * max_slots);
        l.spread[i] = o; o = al(o + sizeof(SpreadSlot) * max_slots);
        l.ev2[i] = o;    o = al(o + sizeof(Slot) * max_slots);
    }
    l.total = o;
    return l;
}

constexpr uint32_t kMaxBatchSlots = 1u << 16;

}  // namespace

int mc_batch_required_bytes(uint32_t max_slots, size_t* bytes)
{
    if (!bytes || max_slots == 0 || max_slots > kMaxBatchSlots)
        return fail(MC_EINVAL, "max_slots must be in [1, %u] and bytes non-null", kMaxBatchSlots);
    *bytes = batch_layout(max_slots).total;
    return MC_OK;
}

int mc_batch_create(uint32_t max_slots, uint32_t precision, void* device_buf, size_t buf_bytes,
                    void* hip_stream, void* hip_stream_aux, mc_batch** out)
{
    if (!out) return fail(MC_EINVAL, "null output handle");
    *out = nullptr;
    if (max_slots == 0 || max_slots > kMaxBatchSlots)
        return fail(MC_EINVAL, "max_slots must be in [1, %u]", kMaxBatchSlots);
    if (precision != MC_FP64 && precision != MC_FP32_DE) return fail(MC_EINVAL, "bad precision");
    if (!device_buf) return fail(MC_EINVAL, "null device buffer");
    if (((uintptr_t)device_buf & 255u) != 0) return fail(MC_EINVAL, "device buffer must be 256-byte aligned");
    const BatchLayout lay = batch_layout(max_slots);
    if (buf_bytes < lay.total)
        return fail(MC_ENOMEM, "device buffer of %zu bytes, %zu needed", buf_bytes, lay.total);
    mc_batch* b = new mc_batch();
    b->max_slots = max_slots;
    b->precision = precision;
    b->stream = (hipStream_t)hip_stream;
    b->sys.assign(max_slots, nullptr);
    b->remaining.assign(max_slots, 0);
    b->parity = 0;
    b->stream2 = nullptr;
    b->go = b->done = nullptr;
    b->stream3 = nullptr;
    b->go3 = b->done3 = nullptr;
    b->spread_max = 0;
    b->ncu = 1;
    b->wg_limit = 0;
    b->turn = 0;
    for (int c = 0; c < 3; ++c) {
        b->ms_per_cycle[c] = ms_per_model_cycle() * kCycleRatio[c];
        b->pred[c] = 0.0;
        b->t_beg[c] = b->t_end[c] = nullptr;
    }
    for (int i = 0; i < 2; ++i) {
        b->dev_slots[i] = nullptr;
        b->host_slots[i] = nullptr;
        b->pending[i] = false;
        b->copied[i] = nullptr;
        b->dev_spread[i] = nullptr;
        b->host_spread[i] = nullptr;
        b->dev_ev2[i] = nullptr;
        b->host_ev2[i] = nullptr;
        b->copied2[i] = nullptr;
        b->pending2[i] = false;
    }
    uint8_t* dbuf = (uint8_t*)device_buf;
    for (int i = 0; i < 2; ++i) {
        // slot tables: one per residency class, double-buffered; the device
        // copies in the caller's buffer, their pinned host staging owned here
        b->dev_slots[i] = (Slot*)(dbuf + lay.slots[i]);
        b->dev_spread[i] = (SpreadSlot*)(dbuf + lay.spread[i]);
        b->dev_ev2[i] = (Slot*)(dbuf + lay.ev2[i]);
        if (hipHostMalloc((void**)&b->host_slots[i], 3 * sizeof(Slot) * max_slots, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&b->copied[i], hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&b->host_spread[i], sizeof(SpreadSlot) * max_slots, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&b->host_ev2[i], sizeof(Slot) * max_slots, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&b->copied2[i], hipEventDisableTiming) != hipSuccess) {
            mc_batch_destroy(b);
            return fail(MC_EDEVICE, "could not allocate the host staging of the slot tables");
        }
    }
    for (int c = 0; c < 3; ++c)
        if (hipEventCreate(&b->t_beg[c]) != hipSuccess || hipEventCreate(&b->t_end[c]) != hipSuccess) {
            mc_batch_destroy(b);
            return fail(MC_EDEVICE, "could not create the timing events");
        }
    b->stream2 = hip_stream_aux ? (hipStream_t)hip_stream_aux : b->stream;
    if (hipEventCreateWithFlags(&b->go, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->go3, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->done3, hipEventDisableTiming) != hipSuccess) {
        mc_batch_destroy(b);
        return fail(MC_EDEVICE, "could not create the stream events");
    }
    if (spread_max_blocks(precision == MC_FP64, &b->spread_max) != hipSuccess) {
        (void)hipGetLastError();
        b->spread_max = 0;
    }
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        mc_batch_destroy(b);
        return fail(MC_EDEVICE, "could not query the device");
    }
    b->ncu = (uint32_t)ncu;
    b->wg_limit = (uint32_t)ncu;
    {
        // the first launch of a kernel carries one-time set-up costs: run the
        // sweep kernels once here with no system, so the batch's timing of its
        // own launches (its engine calibration) does not see them
        const bool fp64 = precision == MC_FP64;
        Slot none{};
        SpreadSlot snone{};
        hipError_t e = launch_sweeps(fp64, true, nullptr, none, 1, 0, b->stream, true);
        if (e == hipSuccess) e = launch_sweeps(fp64, false, nullptr, none, 1, 0, b->stream, true);
        if (e == hipSuccess && b->spread_max >= 2) e = launch_spread(fp64, nullptr, 0, snone, 1, b->stream);
        if (e != hipSuccess) {
            mc_batch_destroy(b);
            return fail(MC_EDEVICE, "warm-up launch: %s", hipGetErrorString(e));
        }
    }
    *out = b;
    return MC_OK;
}

int mc_batch_add(mc_batch* b, mc_system* s, uint64_t n_sweeps, uint32_t* slot)
{
    if (!b || !s) return fail(MC_EINVAL, "null argument");
    if (s->batch) return fail(MC_EINVAL, "system is already in a batch");
    if (s->p.precision != b->precision) return fail(MC_EINVAL, "precision differs from the batch's");
    for (uint32_t i = 0; i < b->max_slots; ++i) {
        if (!b->sys[i]) {
            b->sys[i] = s;
            b->remaining[i] = n_sweeps;
            s->batch = b;
            if (slot) *slot = i;
            return MC_OK;
        }
    }
    return fail(MC_EBUSY, "no free slot");
}

int mc_batch_set_workgroups(mc_batch* b, uint32_t max_workgroups)
{
    if (!b) return fail(MC_EINVAL, "null batch");
    b->wg_limit = max_workgroups ? max_workgroups : b->ncu;
    return MC_OK;
}

int mc_batch_set_hbm_stream(mc_batch* b, void* hip_stream)
{
    if (!b) return fail(MC_EINVAL, "null batch");
    // the previous run's launch on the old stream was joined into the batch
    // stream, so later work there already follows it
    b->stream3 = (hipStream_t)hip_stream == b->stream ? nullptr : (hipStream_t)hip_stream;
    return MC_OK;
}

int mc_batch_run(mc_batch* b, uint64_t max_moves_per_slot, uint32_t* n_launched)
{
    TraceRange tr("mc_batch_run");
    if (!b) return fail(MC_EINVAL, "null batch");
    const int par = b->parity;
    b->parity ^= 1;
    if (b->pending[par]) {
        HIPCHK(hipEventSynchronize(b->copied[par]));
        b->pending[par] = false;
    }
    if (b->pending2[par]) {
        HIPCHK(hipEventSynchronize(b->copied2[par]));
        b->pending2[par] = false;
    }
    Slot* hs = b->host_slots[par];
    const uint32_t S = b->max_slots;
    const bool fp64 = b->precision == MC_FP64;

    // calibration from the launches of the last run that have finished
    for (int c = 0; c < 3; ++c) {
        if (b->pred[c] <= 0.0) continue;
        if (hipEventQuery(b->t_end[c]) != hipSuccess) {
            (void)hipGetLastError();  // not finished: no sample
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b->t_beg[c], b->t_end[c]) == hipSuccess && ms > 0.f) {
            const double f = b->ms_per_cycle[c];
            const double r = std::min(4.0 * f, std::max(0.25 * f, (double)ms / b->pred[c]));
            b->ms_per_cycle[c] = 0.5 * f + 0.5 * r;
        }
        (void)hipGetLastError();
        b->pred[c] = 0.0;
    }
    // every launch of a run is sized to the time the reference system takes
    // for max_moves_per_slot moves
    const double t_slice = slice_time(max_moves_per_slot) * ms_per_model_cycle();
    double pred[3] = {0.0, 0.0, 0.0};

    // Engine of every system for this run.  Each system needs one workgroup;
    // the workgroups left over (up to the batch's limit) go to the systems
    // that can run on the multi-workgroup engine, most remaining work first,
    // each up to its own workgroup count; a system whose state fits in LDS
    // moves there only with enough workgroups to be modelled 25 % faster than
    // on its own one.  The engines make the same decisions, so a system may
    // change engine from run to run.
    std::vector<uint32_t> active;
    for (uint32_t i = 0; i < S; ++i)
        if (b->sys[i] && b->remaining[i] != 0) active.push_back(i);
    // More systems than workgroups at once: a run takes whole rounds of them
    // (the largest multiple of the limit), the systems in turn from run to
    // run, so that no run ends with a partly filled round of workgroups
    if (b->wg_limit && active.size() > b->wg_limit) {
        const size_t A = active.size(), m = (A / b->wg_limit) * b->wg_limit;
        std::vector<uint32_t> chosen;
        chosen.reserve(m);
        for (size_t i = 0; i < m; ++i) chosen.push_back(active[(b->turn + i) % A]);
        b->turn = (uint32_t)((b->turn + m) % A);
        std::sort(chosen.begin(), chosen.end());
        active.swap(chosen);
    }
    std::vector<std::pair<double, uint32_t>> cand;  // (-remaining moves, slot)
    for (uint32_t i : active) {
        const mc_system* s = b->sys[i];
        if (s->g.spread_blocks >= 2 && b->spread_max >= 2)
            cand.emplace_back(-(double)b->remaining[i] * (double)s->p.n_molecules, i);
    }
    std::sort(cand.begin(), cand.end());
    std::vector<uint32_t> nblk(S, 0);
    {
        // the spare compute units shared in proportion to the remaining work,
        // each system up to its own workgroup count (bpc workgroups of the
        // multi-workgroup engine fit on one compute unit), the cooperative
        // launch up to what the device holds at once; what the caps and the
        // rounding leave goes to the systems with the most work, in order
        const uint32_t spare = b->wg_limit > active.size() ? b->wg_limit - (uint32_t)active.size() : 0u;
        const uint32_t bpc = std::max(1u, b->spread_max / std::max(1u, b->ncu));
        double total = 0.0;
        for (const auto& c : cand) total -= c.first;
        uint32_t left = spare, coop = 0;
        auto cus = [&](uint32_t nb) { return (nb + bpc - 1) / bpc; };
        auto pays = [&](const mc_system* s, uint32_t nb) {
            return spread_pays(s->g, nb, b->ms_per_cycle[0], b->ms_per_cycle[2]);
        };
        for (const auto& c : cand) {
            const mc_system* s = b->sys[c.second];
            const uint32_t share = total > 0.0 ? (uint32_t)((double)spare * (-c.first) / total) : 0u;
            const uint32_t nb = std::min({s->g.spread_blocks, (1u + std::min(share, left)) * bpc,
                                          b->spread_max - coop});
            if (nb < 2 || !pays(s, nb)) continue;
            nblk[c.second] = nb;
            left -= cus(nb) - 1;
            coop += nb;
        }
        for (const auto& c : cand) {
            if (left == 0 || coop >= b->spread_max) break;
            const mc_system* s = b->sys[c.second];
            const uint32_t have = nblk[c.second];
            const uint32_t want = std::min({s->g.spread_blocks, (cus(std::max(have, 1u)) + left) * bpc,
                                            b->spread_max - coop + have});
            if (want <= std::max(have, 1u) || want < 2 || !pays(s, want)) continue;
            left -= cus(want) - (have ? cus(have) : 1u);
            coop += want - have;
            nblk[c.second] = want;
        }
    }
    uint32_t n[3] = {0, 0, 0};
    size_t lds[2] = {0, 0};
    uint32_t ns = 0, ne = 0, blocks = 0;
    SpreadSlot* hsp = b->host_spread[par];
    Slot* hev = b->host_ev2[par];
    // the O(M^2) event work of large systems goes to the event kernel over
    // many workgroups, whatever engine ran the sweeps
    std::vector<std::pair<mc_system*, uint32_t>> parts1, parts2;
    auto event_slot = [&](mc_system* s, uint32_t f, std::vector<std::pair<mc_system*, uint32_t>>& parts) {
        Slot ev{};
        ev.sys = s->dev;
        ev.flags = f;
        const uint32_t nbp = event_blocks(s->p.n_molecules);
        if (nbp > 1 && (f & (kFlagResumSet | kFlagResumReport | kFlagResumPeriodic | kFlagGofr))) {
            parts.emplace_back(s, f);
            ev.flags = f | kFlagParts;
            ev.pad = nbp;
        }
        return ev;
    };
    for (uint32_t i : active) {
        mc_system* s = b->sys[i];
        // a system on one workgroup whose events fit the one-workgroup event
        // kernel takes its scheduled re-sums and C_2 samples inside the sweep
        // kernel: its slice stops only at g(r) frames
        const bool inl = !nblk[i] && event_blocks(s->p.n_molecules) == 1;
        uint64_t k = std::min<uint64_t>(b->remaining[i], next_event(s, inl) - s->sweep);
        if (nblk[i]) {
            // modelled cycles of a sweep: the one-workgroup model over the
            // workgroups (the class calibration absorbs the engine's overheads)
            const double unit = s->g.spread_cost / nblk[i];
            if (max_moves_per_slot) {
                const double q = t_slice / (b->ms_per_cycle[2] * unit);
                k = std::min<uint64_t>(k, std::max<uint64_t>(1, (uint64_t)q));
            }
            pred[2] = std::max(pred[2], (double)k * unit);
            SpreadSlot sl{};
            sl.sys = s->dev;
            sl.n_sweeps = k;
            sl.first_block = blocks;
            sl.n_blocks = nblk[i];
            hsp[ns++] = sl;
            blocks += nblk[i];
        } else {
            const int cls = s->g.resident ? 0 : 1;
            if (max_moves_per_slot) {
                // equal time slices: the time of max_moves_per_slot moves of the
                // 1000-molecule reference, in sweeps of this system
                const double cap = t_slice / (b->ms_per_cycle[cls] * s->g.sweep_cost);
                k = std::min<uint64_t>(k, std::max<uint64_t>(1, (uint64_t)cap));
            }
            pred[cls] = std::max(pred[cls], (double)k * s->g.sweep_cost);
            Slot sl{};
            sl.sys = s->dev;
            sl.n_sweeps = k;
            sl.flags = inl ? kFlagInline : 0u;
            hs[cls * S + n[cls]++] = sl;
            lds[cls] = std::max(lds[cls], s->g.lds);
        }
        b->remaining[i] -= k;
        s->sweep += k;
        const uint32_t f = events_at(s, s->sweep) & (inl ? ~(kFlagResumPeriodic | kFlagC2) : ~0u);
        if (f) {
            if (nblk[i]) hev[ne++] = event_slot(s, f, parts2);
            else hs[2 * S + n[2]++] = event_slot(s, f, parts1);
        }
    }

    if (ns) {
        HIPCHK(hipEventRecord(b->go, b->stream));
        HIPCHK(hipStreamWaitEvent(b->stream2, b->go, 0));
        HIPCHK(hipMemcpyAsync(b->dev_spread[par], hsp, sizeof(SpreadSlot) * ns, hipMemcpyHostToDevice,
                              b->stream2));
        if (ne)
            HIPCHK(hipMemcpyAsync(b->dev_ev2[par], hev, sizeof(Slot) * ne, hipMemcpyHostToDevice,
                                  b->stream2));
        HIPCHK(hipEventRecord(b->copied2[par], b->stream2));
        b->pending2[par] = true;
        SpreadSlot none{};
        HIPCHK(launch_zero_barriers(b->dev_spread[par], ns, b->stream2));
        HIPCHK(hipEventRecord(b->t_beg[2], b->stream2));
        HIPCHK(launch_spread(fp64, b->dev_spread[par], ns, none, blocks, b->stream2));
        HIPCHK(hipEventRecord(b->t_end[2], b->stream2));
        b->pred[2] = pred[2];
        HIPCHK(launch_parts_of(parts2, b->stream2));
        Slot none2{};
        if (ne) HIPCHK(launch_events(b->dev_ev2[par], none2, ne, b->stream2));
        HIPCHK(hipEventRecord(b->done, b->stream2));
    }

    if (n[0] + n[1] + n[2]) {
        HIPCHK(hipMemcpyAsync(b->dev_slots[par], hs, 3 * sizeof(Slot) * S, hipMemcpyHostToDevice,
                              b->stream));
        HIPCHK(hipEventRecord(b->copied[par], b->stream));
        b->pending[par] = true;
        Slot none{};
        // with a third stream the HBM class's launch runs beside the LDS
        // class's (each on its own compute units) instead of after it; the
        // events below follow both
        const bool side = n[0] && n[1] && b->stream3;
        if (side) {
            HIPCHK(hipEventRecord(b->go3, b->stream));
            HIPCHK(hipStreamWaitEvent(b->stream3, b->go3, 0));
        }
        for (int cls = 0; cls < 2; ++cls)
            if (n[cls]) {
                hipStream_t st = cls == 1 && side ? b->stream3 : b->stream;
                HIPCHK(hipEventRecord(b->t_beg[cls], st));
                HIPCHK(launch_sweeps(fp64, cls == 0, b->dev_slots[par] + cls * S, none, n[cls],
                                     lds[cls], st, true));
                HIPCHK(hipEventRecord(b->t_end[cls], st));
                b->pred[cls] = pred[cls];
            }
        if (side) {
            HIPCHK(hipEventRecord(b->done3, b->stream3));
            HIPCHK(hipStreamWaitEvent(b->stream, b->done3, 0));
        }
        HIPCHK(launch_parts_of(parts1, b->stream));
        if (n[2]) HIPCHK(launch_events(b->dev_slots[par] + 2 * S, none, n[2], b->stream));
    }
    // later work on the batch stream (the next run, poll, reads) follows the
    // multi-workgroup launch
    if (ns) HIPCHK(hipStreamWaitEvent(b->stream, b->done, 0));
    if (n_launched) *n_launched = (n[0] ? 1u : 0u) + (n[1] ? 1u : 0u) + (ns ? 1u : 0u);
    return MC_OK;
}

int mc_batch_poll(mc_batch* b, uint32_t* slots, mc_system** systems, size_t cap, size_t* n)
{
    if (!b) return fail(MC_EINVAL, "null batch");
    HIPCHK(hipStreamSynchronize(b->stream));
    size_t k = 0;
    for (uint32_t i = 0; i < b->max_slots && k < cap; ++i) {
        mc_system* s = b->sys[i];
        if (!s || b->remaining[i] != 0) continue;
        if (slots) slots[k] = i;
        if (systems) systems[k] = s;
        s->batch = nullptr;
        b->sys[i] = nullptr;
        ++k;
    }
    if (n) *n = k;
    return MC_OK;
}

int mc_batch_cancel(mc_batch* b, uint32_t slot)
{
    if (!b || slot >= b->max_slots || !b->sys[slot]) return fail(MC_EINVAL, "no such slot");
    HIPCHK(hipStreamSynchronize(b->stream));
    b->sys[slot]->batch = nullptr;
    b->sys[slot] = nullptr;
    b->remaining[slot] = 0;
    return MC_OK;
}

void mc_batch_destroy(mc_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (auto* s : b->sys)
        if (s) s->batch = nullptr;
    if (b->stream2) (void)hipStreamSynchronize(b->stream2);
    if (b->stream3) (void)hipStreamSynchronize(b->stream3);
    for (int i = 0; i < 2; ++i) {
        if (b->host_slots[i]) (void)hipHostFree(b->host_slots[i]);
        if (b->copied[i]) (void)hipEventDestroy(b->copied[i]);
        if (b->host_spread[i]) (void)hipHostFree(b->host_spread[i]);
        if (b->host_ev2[i]) (void)hipHostFree(b->host_ev2[i]);
        if (b->copied2[i]) (void)hipEventDestroy(b->copied2[i]);
    }
    for (int c = 0; c < 3; ++c) {
        if (b->t_beg[c]) (void)hipEventDestroy(b->t_beg[c]);
        if (b->t_end[c]) (void)hipEventDestroy(b->t_end[c]);
    }
    if (b->go) (void)hipEventDestroy(b->go);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->go3) (void)hipEventDestroy(b->go3);
    if (b->done3) (void)hipEventDestroy(b->done3);
    delete b;
}

}  // extern "C"
