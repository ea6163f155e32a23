// engine.h -- device-side data layout of the flip Monte Carlo engine.
//
// One system = one workgroup of 512 threads (8 wave64s).  A system whose
// state fits in the workgroup's LDS ("resident") keeps centres of mass, site
// offsets and cell lists there for the whole launch; larger systems keep them
// in HBM and the same code reads them through global pointers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace flipmc {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxSeg = 64;        // stencil row segments per cell (k <= 3: <= 50)
constexpr int kGofrBins = 256;
constexpr int kGofrQueue = 128;  // per-wave queue of molecule pairs of a g(r) frame
constexpr int kC2Max = 32;
constexpr int kMaxMolecules = 65535;  // indices are stored as u16 in cell lists
constexpr int kCellListCap = 192;     // per-wave list of molecules near the current cell
// The single-workgroup event kernel copies centres, quaternions and types of
// systems up to this size into LDS for its O(M^2) loops (larger systems use
// the multi-workgroup event kernel).
constexpr uint32_t kEventStage = 2047;
constexpr size_t kEventStageBytes = size_t(kEventStage) * (7 * sizeof(double) + sizeof(uint32_t));

// Work of the event kernel (Slot::flags).
enum : uint32_t {
    kFlagResumSet = 1u,       // re-sum E and take it as the accumulated energy
    kFlagResumReport = 2u,    // re-sum E and store it as e_resum / drift
    kFlagObsReset = 4u,       // take the current state as the C_2 reference / time origin
    kFlagResumPeriodic = 8u,  // scheduled re-sum: also record the drift sample
    kFlagGofr = 16u,          // accumulate one g(r) frame
    kFlagC2 = 32u,            // record one C_2 sample
    kFlagParts = 64u,         // the re-sum and the g(r) frame were done by the
                              // multi-workgroup event kernel: sum its partial
                              // energies (Slot::pad of them), count the frame
    kFlagInline = 128u,       // (a sweep slot) the scheduled re-sums and C_2
                              // samples of its sweeps are taken by the sweep
                              // kernel itself, as the event kernel takes them
};

// Device accumulators of one system.
struct Stats {
    uint64_t sweep;          // sweeps done (keys the random numbers)
    uint64_t obs_origin;     // sweep at the last observable reset
    double e_acc;            // E_0 + sum of accepted dE
    double e_resum;          // last FP64 re-sum
    double drift;            // e_acc - e_resum at that re-sum
    double max_abs_drift;    // over re-sums after the first window
    uint64_t resum_sweep;
    uint64_t n_resum;
    uint64_t attempts[3];
    uint64_t accepts[3];
    uint64_t exits;
    uint64_t pair_terms;
    uint64_t pair_tests;
    uint64_t near_overflows;  // cells whose near list overflowed (every stencil molecule evaluated)
    double e_sum;
    double e_sumsq;
    uint32_t n_e;
    uint32_t n_drift;
    uint32_t n_gofr;
    uint32_t n_c2;
    uint32_t fault;          // nonzero: a workgroup barrier of the multi-workgroup engine timed out
    uint32_t pad;
};

// Everything a workgroup needs about its system; lives in the system's device
// buffer and is written by the host.
struct SysDev {
    uint32_t M, k, nc, ncell;
    uint32_t precision, resident, seed_lo, seed_hi;
    double L, w, T, p_flip, p_ft, dmax, rot_max, reach2, radius, rc2_factor;
    double body[9];      // body-frame site offsets, row s = site s
    double sigma[3];     // diameters of types A, B, C
    uint32_t resum_interval, obs_interval, gofr_interval, obs_start;
    uint32_t max_samples, gofr_nbins, lds_bytes, barrier_polls;
    double gofr_dr, gofr_rmax;
    double fs_q, fs_q_cm;  // wavenumbers of F_s (sites) and F_s^cm (centres)
    // state
    double* com;         // SoA [3][M]
    double* quat;        // SoA [4][M], (w, x, y, z)
    uint32_t* types;     // [M]: byte s = type of site s
    double* u0;          // SoA [3][M] C_2 reference orientation
    uint8_t* kref;       // [M] site index followed by C_2
    Stats* stats;
    double* e_samples;
    double* drift_samples;
    uint64_t* gofr_all;
    uint64_t* gofr_inter;
    double* c2;
    uint64_t* c2_sweep;
    int32_t* img;        // SoA [3][M] periodic images crossed by accepted translations
    double* r0;          // SoA [3][M] unwrapped centres at the observable origin
    double* o0;          // SoA [9][M] site offsets at the observable origin
    double* fs;          // [kC2Max] F_s(q, t) at the C_2 sample sweeps
    double* fs_cm;       // [kC2Max] F_s^cm(q, t) at the same sweeps
    double* mom;         // [4][kC2Max] per-particle moments at the same sweeps
    // HBM copies of the work arrays of non-resident systems
    void* g_site;        // Real4 [3M]: offset xyz + sigma of the site's type
    uint32_t* g_cell;    // [ncell + 1] cell starts
    uint16_t* g_cellid;  // [M]
    uint16_t* g_list;    // [M] molecules sorted by cell, ascending inside a cell
    void* props;         // [M] proposals of the current sweep (48 bytes each)
    uint32_t* g_cnt;     // [2 * ncell] cell counts and fill cursors (multi-workgroup engine)
    double* g_part;      // [kMaxParts] per-workgroup partial sums of the event kernel
    double* g_ecell;     // [ncell] accepted dE of each cell in the current sweep (HBM state)
    uint32_t* g_bar;     // barrier counter of the system's workgroups (multi-workgroup engine)
    // decision log
    void* log;
    uint64_t log_sweep0;
    uint64_t log_sweeps;
};

struct Slot {
    SysDev* sys;
    uint64_t n_sweeps;
    uint32_t flags;
    uint32_t pad;
};

struct MoveRecord {   // mirrors mc_move_record
    double delta_e;
    double scale;
    double t_log_u;
    uint64_t sweep;
    uint32_t molecule;
    uint8_t move, accepted, exited, axis;
    uint32_t pair_terms;
    uint32_t pad;
};
static_assert(sizeof(MoveRecord) == 48, "record layout");

// Per-wave LDS work areas: the molecules near the current cell, the
// survivors of a trial's prune, the trial in flight.
__host__ __device__ constexpr size_t site_bytes(bool fp64) { return fp64 ? 32 : 16; }
__host__ __device__ constexpr size_t trial_bytes(bool fp64) { return fp64 ? 272 : 160; }

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// LDS carve-up, shared by the host (launch size) and the kernel (pointers).
struct LdsLayout {
    size_t surv, seglo, segoff, near, misc, trial;
    size_t com, site, cell, cellid, list, ecell, total;
};

__host__ __device__ inline LdsLayout lds_layout(bool fp64, bool resident, uint32_t M,
                                                 uint32_t ncell)
{
    LdsLayout l{};
    size_t o = 0;
    l.surv = o;   o = align16(o + kWaves * kCellListCap * sizeof(uint16_t));
    l.seglo = o;  o = align16(o + kWaves * kMaxSeg * sizeof(uint16_t));
    l.segoff = o; o = align16(o + kWaves * kMaxSeg * sizeof(uint16_t));
    l.near = o;   o = align16(o + kWaves * kCellListCap * 8);
    l.misc = o;   o = align16(o + 16 * sizeof(double));
    l.trial = o;  o = align16(o + kWaves * trial_bytes(fp64));
    if (resident) {
        l.com = o;    o = align16(o + 3 * size_t(M) * sizeof(double));
        l.site = o;   o = align16(o + 3 * size_t(M) * site_bytes(fp64));
        l.cell = o;   o = align16(o + (size_t(ncell) + 1) * sizeof(uint32_t));
        l.cellid = o; o = align16(o + size_t(M) * sizeof(uint16_t));
        l.list = o;   o = align16(o + size_t(M) * sizeof(uint16_t));
        l.ecell = o;  o = align16(o + size_t(ncell) * sizeof(double));
    }
    l.total = o;
    return l;
}

// Multi-workgroup ("spread") engine for systems larger than one workgroup's
// LDS: 4 waves per workgroup, every wave takes cells of the current colour and
// stages each cell's neighbourhood (up to kCellListCap molecules, from a
// stencil of up to kSpreadPerLane * 64 molecules) in its LDS.
constexpr int kSpreadThreads = 256;
constexpr int kSpreadWaves = kSpreadThreads / 64;
constexpr int kSpreadPerLane = 8;
constexpr int kMaxParts = 1024;  // workgroups of the event kernel, waves of the spread kernel

__host__ __device__ inline size_t spread_wave_bytes(bool fp64)
{
    size_t o = 0;
    o = align16(o + 3 * size_t(kCellListCap) * sizeof(double));  // staged centres
    o = align16(o + 3 * size_t(kCellListCap) * site_bytes(fp64));  // staged sites
    o = align16(o + size_t(kCellListCap) * sizeof(uint16_t));      // molecule of each slot
    o = align16(o + size_t(kCellListCap) * sizeof(uint16_t));      // slot of each cell molecule
    o = align16(o + size_t(kCellListCap) * 8);                     // near list
    o = align16(o + size_t(kCellListCap) * sizeof(uint16_t));      // survivors
    o = align16(o + 2 * size_t(kMaxSeg) * sizeof(uint16_t));       // stencil segments
    o = align16(o + trial_bytes(fp64));
    return o;
}
__host__ __device__ inline size_t spread_lds_bytes(bool fp64)
{
    return kSpreadWaves * spread_wave_bytes(fp64) + 16 * sizeof(double);
}

// Kernel launchers (kernels.hip).  inline_events: the sweep kernel takes the
// scheduled re-sums and C_2 samples of slots flagged kFlagInline.
hipError_t launch_sweeps(bool fp64, bool resident, const Slot* dev_slots, const Slot& one,
                         uint32_t n_blocks, size_t lds_bytes, hipStream_t stream,
                         bool inline_events = false);
hipError_t launch_events(const Slot* dev_slots, const Slot& one, uint32_t n_blocks,
                         hipStream_t stream);
hipError_t launch_init_lattice(SysDev* dev_sys, uint32_t M, hipStream_t stream);
// One system of a multi-workgroup launch: its workgroups and sweeps.
struct SpreadSlot {
    SysDev* sys;
    uint64_t n_sweeps;
    uint32_t first_block, n_blocks;
};

// Cooperative launch of the multi-workgroup engine over n_blocks workgroups:
// the systems of dev_slots[0 .. n_slots) (device array), or `one` when
// dev_slots is null.  The workgroups of each system synchronise among
// themselves only (each system's g_bar must be zero at launch).
hipError_t launch_spread(bool fp64, const SpreadSlot* dev_slots, uint32_t n_slots,
                         const SpreadSlot& one, uint32_t n_blocks, hipStream_t stream);
// Zero the barrier counters of the systems of dev_slots[0 .. n_slots).
hipError_t launch_zero_barriers(const SpreadSlot* dev_slots, uint32_t n_slots, hipStream_t stream);
// Largest cooperative grid of the spread kernel on the current device.
hipError_t spread_max_blocks(bool fp64, uint32_t* n_blocks);
// The systems of one launch of the event work over many workgroups, passed by
// value (no table in memory): system i owns workgroups [first, first + count)
// and splits its work over them as a launch of count workgroups of its own
// would, so its partial sums do not depend on the systems beside it.
struct PartSlot {
    SysDev* sys;
    uint32_t flags, first, count, pad;
};
constexpr uint32_t kPartSlots = 128;
struct PartList {
    PartSlot s[kPartSlots];
    uint32_t n;
};
// The O(M^2) part of the events of list.s[0 .. n) (re-sum partial energies
// into g_part, g(r) frame into the histograms), n_blocks = the sum of their
// counts; follow with launch_events(flags | kFlagParts, pad = count).
hipError_t launch_event_parts(const PartList& list, uint32_t n_blocks, hipStream_t stream);

// Record msg as the calling thread's last error (mc_last_error) and return code.
int api_error(int code, const char* msg);

}  // namespace flipmc
