// flex_sweep.h -- the sweep kernel of the flexible-molecule engine (the
// paper's own model, Sec. II.A: atoms joined by FENE bonds, Eq. 2, with the
// WCA potential of Eq. 1 between every pair of atoms, intramolecular pairs
// included; and the squares and tetrahedra of Sec. VII), with the descriptor
// it reads.  Included by flex.hip, which holds the event kernels and the host
// code.
//
// A sweep attempts every atom once (a Monte Carlo timestep of N attempts,
// Sec. II.B): with probability p_flip a flip of the atom's molecule -- a
// permutation of the types of its atoms at fixed positions, one of the 180
// degree rotations of the ideal body -- otherwise a translation of the atom,
// uniform in [-d, d)^3 and confined to its cell.
//
// Execution: one workgroup of 8 wave64s per system (several systems per
// launch, a workgroup each), the positions, types and cell lists in LDS when
// they fit.  Per sweep a random shift of a cubic cell grid over the atoms, a
// counting sort into cells (ascending atom index inside each cell), then the
// k^3 colours in order; the waves take the cells of a colour, and a wave runs
// its cell's attempts one after another.  Same-colour cells are at least
// (k - 1) w >= 2 D + r_c apart (D the largest distance two atoms of one
// molecule can reach, r_c the largest cut-off), so no two attempts of a
// colour touch the same pair term.  Per cell the wave lists the atoms of the
// 27 cells around it and draws the proposals of the cell's atoms, a lane
// each; per attempt the lanes take the intramolecular pairs and the listed
// atoms, and a DPP reduction in FP64 gives dE in a fixed order.  A bond
// stretched to 1.5 sigma_ij or beyond makes dE infinite: the move is
// rejected.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "engine.h"
#include "flipmc.h"
#include "wave.h"

namespace flipmc {
namespace {
constexpr int kFxThreads = 512;
constexpr int kFxWaves = kFxThreads / 64;
constexpr int kFxSeg = 64;          // stencil row segments per attempt (radius <= 2: <= 50)
constexpr int kFxCand = 384;        // atoms of a cell's 27-cell stencil listed per wave
// static LDS of the sweep kernel: segments and candidate lists per wave, scan
// scratch and the energy accumulator (with room to spare)
constexpr size_t kFxStaticLds = (size_t)kFxWaves * (2 * kFxSeg + kFxCand) * 4 + 256;
constexpr uint32_t kFxParts = 1024;  // workgroups of the event kernel
constexpr uint32_t kFxMany = 256;    // systems of one sweep launch (a workgroup each)

// Everything a workgroup needs about one system; in the system's buffer.
struct FxDev {
    uint32_t geometry, n, M, N;
    uint32_t k, nc, ncell, nflip;
    uint32_t seed_lo, seed_hi, pad2, pad3;
    uint32_t bonded;  // bit 4 i + j: atoms i, j of a molecule are bonded
    uint32_t resum_interval, obs_interval, gofr_interval, obs_start, max_samples, gofr_nbins;
    uint32_t pad;
    double L, invL, w, T, p_flip, dmax, rc2f;
    double sigma[4];
    double gofr_dr, gofr_rmax, fs_q, fs_q_cm;
    // a colour's cells run side by side when sep = (k - 1) w >= 2 D + dyn_base
    // (dyn_base = r_c + 4 sqrt(3) d), D the largest atom distance inside a
    // molecule with an atom in those cells at the colour's start; always
    // when `together` is 1 (the gap covers the worst case), never when it is
    // 2 (forced one cell at a time)
    double sep, dyn_base;
    uint32_t together, pad4;
    uint8_t flips[4][4];  // new type of atom s = old type of atom flips[q][s]
    double* pos;          // SoA [3][N], wrapped into [0, L)
    uint8_t* type;        // [N]
    int32_t* img;         // SoA [3][N] periodic images crossed by accepted translations
    Stats* stats;
    double* e_samples;
    double* drift_samples;
    uint64_t* gofr_all;
    uint64_t* gofr_inter;
    double* c2;
    uint64_t* c2_sweep;
    double* fs;
    double* fs_cm;
    double* mom;          // [4][kC2Max] per-particle moments at the C_2 samples
    double* u0;           // [3][M] orientation at the observable origin
    uint8_t* kref;        // [M] atom the orientation follows
    double* r0;           // [3][N] unwrapped atoms at the origin
    double* rcm0;         // [3][M] unwrapped centres at the origin
    uint32_t* cell_start; // [ncell + 1]
    uint32_t* cell_list;  // [N] atoms sorted by cell, ascending inside a cell
    uint32_t* cell_id;    // [N]
    double* ecell;        // [ncell] accepted dE of each cell in the current sweep
    double* part;         // [kFxParts] partial energies of the event kernel
    MoveRecord* log;
    uint64_t log_sweep0, log_sweeps;
};

// The systems of one sweep launch, passed by value (2 KiB of kernel
// arguments): workgroup b runs d[b].
struct FxList {
    FxDev* d[kFxMany];
};

// The constants of the sweep kernel, copied from the system's descriptor into
// registers at the start of a launch (read through the descriptor, every
// store to LDS or memory could alias them and force a reload).
struct FxK {
    uint32_t n, N, nc, nflip, bonded, seed_lo, seed_hi, together;
    uint32_t flipw[4];  // byte s of word q: flips[q][s]
    double L, invL, w, T, p_flip, dmax, rc2f, sep, dyn_base;
    double sigma[4];
    int32_t* img;
    MoveRecord* log;
    uint64_t log_sweep0;
};

__device__ __forceinline__ FxK fx_const(const FxDev& D)
{
    FxK K;
    K.n = D.n; K.N = D.N; K.nc = D.nc; K.nflip = D.nflip; K.bonded = D.bonded;
    K.seed_lo = D.seed_lo; K.seed_hi = D.seed_hi;
    for (int q = 0; q < 4; ++q)
        K.flipw[q] = (uint32_t)D.flips[q][0] | ((uint32_t)D.flips[q][1] << 8) | ((uint32_t)D.flips[q][2] << 16) |
                     ((uint32_t)D.flips[q][3] << 24);
    K.L = D.L; K.invL = D.invL; K.w = D.w; K.T = D.T; K.p_flip = D.p_flip; K.dmax = D.dmax; K.rc2f = D.rc2f;
    K.sep = D.sep; K.dyn_base = D.dyn_base; K.together = D.together;
    for (int t = 0; t < 4; ++t) K.sigma[t] = D.sigma[t];
    K.img = D.img;
    K.log = D.log;
    K.log_sweep0 = D.log_sweep0;
    return K;
}

__device__ __forceinline__ double fx_wrap(double x, double L) { return x - L * floor(x / L); }
__device__ __forceinline__ double fx_mi(double d, double L, double invL) { return d - L * rint(d * invL); }

__device__ __forceinline__ int fx_axis(double x, double h, const FxK& D)
{
    int c = (int)floor(fx_wrap(x - h, D.L) / D.w);
    c = c < 0 ? 0 : c;
    return c >= (int)D.nc ? (int)D.nc - 1 : c;
}

__device__ __forceinline__ uint32_t fx_cell(double x, double y, double z, const double h[3], const FxK& D)
{
    const uint32_t nc = D.nc;
    return (uint32_t)fx_axis(x, h[0], D) +
           nc * ((uint32_t)fx_axis(y, h[1], D) + nc * (uint32_t)fx_axis(z, h[2], D));
}

// Whether every atom within distance m of coordinate x (one axis, grid shift
// h) was sorted into the three cells c - 1, c, c + 1 of that axis: x lies at
// least m inside the outer faces of the three
__device__ __forceinline__ bool fx_in_stencil(double x, double h, uint32_t c, const FxK& D, double m)
{
    if (D.nc <= 3u) return true;  // the three cells are the whole axis
    const double t = fx_mi(fx_wrap(x - h, D.L) - (double)c * D.w, D.L, D.invL);
    return t >= m - D.w && t <= 2.0 * D.w - m;
}

// Eq. (1) as (2 (s/r)^6 - 1)^2 below the cut-off, FP64.  1 / r^2 is the
// hardware estimate refined by two Newton steps (within an ulp or two of the
// quotient; r^2 is a normal number for every pair inside the cut-off).
__device__ __forceinline__ double fx_wca(double s2, double r2, double rc2f)
{
    if (!(r2 < rc2f * s2)) return 0.0;
    double y = __builtin_amdgcn_rcp(r2);
    y = fma(fma(-r2, y, 1.0), y, y);
    y = fma(fma(-r2, y, 1.0), y, y);
    const double x = s2 * y;
    const double t = fma(2.0, x * x * x, -1.0);
    return t * t;
}

// Eq. (2), infinite at or beyond 1.5 sigma_ij.
__device__ __forceinline__ double fx_fene(double sig, double r2)
{
    const double lim2 = 2.25 * sig * sig;
    if (!(r2 < lim2)) return __builtin_inf();
    return -33.75 * log(1.0 - r2 / lim2);
}

struct FxCount {
    uint32_t att_t, att_f, acc_t, acc_f, exits;
    uint64_t terms;
    double e;  // accepted dE of the current cell, in attempt order
};

// Per-wave LDS: the stencil's row segments.
struct FxWaveLds {
    uint32_t* seglo;
    uint32_t* segoff;
    uint32_t* cand;  // [kFxCand] atoms of the current cell's stencil
};

// Where the sweep kernel reads and writes the state and the cell lists: the
// workgroup's LDS for systems that fit there, the system's buffer otherwise.
struct FxView {
    double* pos;          // SoA [3][N]
    uint8_t* type;        // [N]
    uint32_t* cell_start; // [ncell + 1]
    uint32_t* cell_list;  // [N]
    uint32_t* cell_id;    // [N]
    double* ecell;        // [ncell]
};

struct FxLds {
    size_t pos, type, cstart, clist, cid, ecell, total;
};

__host__ __device__ inline FxLds fx_lds_layout(uint32_t N, uint32_t ncell)
{
    FxLds l{};
    size_t o = 0;
    auto a16 = [](size_t x) { return (x + 15) & ~size_t(15); };
    l.pos = o;    o = a16(o + 3 * size_t(N) * sizeof(double));
    l.ecell = o;  o = a16(o + size_t(ncell) * sizeof(double));
    l.type = o;   o = a16(o + size_t(N));
    l.cstart = o; o = a16(o + (size_t(ncell) + 1) * sizeof(uint32_t));
    l.clist = o;  o = a16(o + size_t(N) * sizeof(uint32_t));
    l.cid = o;    o = a16(o + size_t(N) * sizeof(uint32_t));
    l.total = o;
    return l;
}

// Row segments of the cells within radius r of cell (cx, cy, cz): rows along
// x of one or two contiguous cell ranges (every cell once when the stencil
// covers the whole axis).  Returns the number of segments; *total = atoms.
__device__ __forceinline__ int fx_segments(const FxK& D, const FxView& V, int cx, int cy, int cz, int r,
                                           const FxWaveLds& W,
                           uint32_t* total)
{
    const int lane = __lane_id();
    const int nc = (int)D.nc;
    const bool full = 2 * r + 1 >= nc;
    const int nrow = full ? nc : 2 * r + 1;
    int xa0, xb0, xa1 = 0, xb1 = -1;
    if (full) {
        xa0 = 0; xb0 = nc - 1;
    } else if (cx - r < 0) {
        xa0 = cx - r + nc; xb0 = nc - 1; xa1 = 0; xb1 = cx + r;
    } else if (cx + r >= nc) {
        xa0 = cx - r; xb0 = nc - 1; xa1 = 0; xb1 = cx + r - nc;
    } else {
        xa0 = cx - r; xb0 = cx + r;
    }
    const int nxr = xb1 >= xa1 ? 2 : 1;
    const int nseg = nrow * nrow * nxr;
    uint32_t cnt = 0, lo = 0;
    if (lane < nseg) {
        const int ixr = lane % nxr, iy = (lane / nxr) % nrow, iz = lane / (nxr * nrow);
        const int y = full ? iy : (cy - r + iy + nc) % nc;
        const int z = full ? iz : (cz - r + iz + nc) % nc;
        const int xa = ixr ? xa1 : xa0, xb = ixr ? xb1 : xb0;
        const uint32_t row = (uint32_t)(nc * (y + nc * z));
        lo = V.cell_start[row + xa];
        cnt = V.cell_start[row + xb + 1] - lo;
    }
    const uint32_t off = wave_excl_scan(cnt, total);
    if (lane < nseg) {
        W.seglo[lane] = lo;
        W.segoff[lane] = off;
    }
    wave_lds_sync();
    return nseg;
}

__device__ __forceinline__ uint32_t fx_stencil_atom(const FxView& V, const FxWaveLds& W, int nseg, uint32_t idx)
{
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (W.segoff[mid] <= idx) lo = mid; else hi = mid;
    }
    return V.cell_list[W.seglo[lo] + (idx - W.segoff[lo])];
}

template <typename T>
__device__ __forceinline__ T fx_pick(const T v[4], uint32_t i)
{
    return i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
}

// The proposal of the attempt on atom a (Sec. II.B): move kind, flip
// rotation or translation target, the cell-exit test and T ln u.  Drawn for
// the atoms of a cell by one lane each before the cell's attempts (an atom's
// position changes only in its own attempt, so the draws do not depend on
// the attempts before it).
struct FxProp {
    double thr;         // T ln u
    double tx, ty, tz;  // translation target before the wrap
    uint32_t kind;      // flip: rotation index; translation: 255
    uint32_t flip, exited;
};

__device__ __forceinline__ FxProp fx_propose(const FxK& D, const FxView& V, uint32_t a, uint64_t sweep,
                                             const double h[3], uint32_t cell)
{
    const uint32_t N = D.N;
    const uint32_t slo = (uint32_t)sweep, shi = (uint32_t)(sweep >> 32);
    const U4 b0 = philox10(a, slo, shi, 0u, D.seed_lo, D.seed_hi);
    const U4 b1 = philox10(a, slo, shi, 1u, D.seed_lo, D.seed_hi);
    const double uacc = unit_53(b0.x, b0.y), ut = unit_open(b0.z);
    const double p0 = unit_open(b1.x), p1 = unit_open(b1.y), p2 = unit_open(b1.z);
    FxProp pr;
    pr.thr = D.T * log(uacc);
    pr.flip = ut < D.p_flip ? 1u : 0u;
    pr.kind = 255;
    pr.exited = 0;
    pr.tx = pr.ty = pr.tz = 0.0;
    if (pr.flip) {
        uint32_t q = (uint32_t)((double)D.nflip * p0);
        pr.kind = q >= D.nflip ? D.nflip - 1 : q;
    } else {
        pr.tx = V.pos[a] + D.dmax * (2.0 * p0 - 1.0);
        pr.ty = V.pos[N + a] + D.dmax * (2.0 * p1 - 1.0);
        pr.tz = V.pos[2 * N + a] + D.dmax * (2.0 * p2 - 1.0);
        pr.exited = fx_cell(fx_wrap(pr.tx, D.L), fx_wrap(pr.ty, D.L), fx_wrap(pr.tz, D.L), h, D) != cell;
    }
    return pr;
}

__device__ __forceinline__ double rl_dbl(double v, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ FxProp fx_prop_of_lane(const FxProp& p, int l)
{
    FxProp r;
    r.thr = rl_dbl(p.thr, l);
    r.tx = rl_dbl(p.tx, l);
    r.ty = rl_dbl(p.ty, l);
    r.tz = rl_dbl(p.tz, l);
    r.kind = (uint32_t)__builtin_amdgcn_readlane((int)p.kind, l);
    r.flip = (uint32_t)__builtin_amdgcn_readlane((int)p.flip, l);
    r.exited = (uint32_t)__builtin_amdgcn_readlane((int)p.exited, l);
    return r;
}

// The atoms of the 27-cell stencil around `cell` into the wave's candidate
// list, in the order fx_stencil_atom gives them.  Returns their count, or
// 0xFFFFFFFF when they exceed the list (attempts then walk the stencil).
__device__ __forceinline__ uint32_t fx_gather_candidates(const FxK& D, const FxView& V, uint32_t cell,
                                                         const FxWaveLds& W)
{
    const uint32_t nc = D.nc;
    uint32_t total;
    const int nseg = fx_segments(D, V, (int)(cell % nc), (int)((cell / nc) % nc), (int)(cell / (nc * nc)), 1,
                                 W, &total);
    if (total > (uint32_t)kFxCand) return 0xFFFFFFFFu;
    for (uint32_t b = 0; b < total; b += 64u) {
        const uint32_t idx = b + (uint32_t)__lane_id();
        if (idx < total) W.cand[idx] = fx_stencil_atom(V, W, nseg, idx);
    }
    wave_lds_sync();
    return total;
}

// One attempt on atom a (Sec. II.B) by a whole wave, with its proposal pr
// (wave-uniform).  `cell` is the atom's cell for the sweep's shift h: a
// translation that leaves it is rejected.  ncand: the size of the wave's
// candidate list of this cell's stencil (0xFFFFFFFF: no list).
__device__ __forceinline__ void fx_attempt(const FxK& D, const FxView& V, uint32_t a, const FxProp& pr,
                                           uint64_t sweep, const double h[3], uint32_t cell, uint32_t ncand,
                                           bool logging, const FxWaveLds& W, FxCount& wc)
{
    const int lane = __lane_id();
    const uint32_t n = D.n, N = D.N;
    const bool flip = pr.flip != 0u;
    const uint32_t base = n * (a / n), sa = a - base;
    const double sig[4] = {D.sigma[0], D.sigma[1], D.sigma[2], D.sigma[3]};

    // the molecule's atoms before and after (wave-uniform)
    double ox[4], oy[4], oz[4], nx[4], ny[4], nz[4];
    uint32_t ot[4], nt[4];
#pragma unroll
    for (uint32_t s = 0; s < 4; ++s) {
        const uint32_t at = base + (s < n ? s : 0u);
        ox[s] = nx[s] = V.pos[at];
        oy[s] = ny[s] = V.pos[N + at];
        oz[s] = nz[s] = V.pos[2 * N + at];
        ot[s] = nt[s] = V.type[at];
    }
    uint32_t changed = 0;  // bit s: atom base + s moves or changes type
    double wx = 0.0, wy = 0.0, wz = 0.0;
    if (flip) {
#pragma unroll
        for (uint32_t s = 0; s < 4; ++s) {
            if (s >= n) continue;
            nt[s] = fx_pick(ot, (fx_pick(D.flipw, pr.kind) >> (8 * s)) & 0xFFu);
            if (nt[s] != ot[s]) changed |= 1u << s;
        }
    } else {
        wx = fx_wrap(pr.tx, D.L);
        wy = fx_wrap(pr.ty, D.L);
        wz = fx_wrap(pr.tz, D.L);
#pragma unroll
        for (uint32_t s = 0; s < 4; ++s)
            if (s == sa) {
                nx[s] = wx;
                ny[s] = wy;
                nz[s] = wz;
            }
        changed = 1u << sa;
    }
    if (flip) wc.att_f += 1; else wc.att_t += 1;
    if (pr.exited) {
        wc.exits += 1;
        if (logging && lane == 0) {
            MoveRecord rec;
            rec.delta_e = 0.0; rec.scale = 0.0; rec.t_log_u = pr.thr; rec.sweep = sweep;
            rec.molecule = a; rec.move = MC_TRANSLATE; rec.accepted = 0; rec.exited = 1;
            rec.axis = 255; rec.pair_terms = 0; rec.pad = 0;
            D.log[(sweep - D.log_sweep0) * N + a] = rec;
        }
        return;
    }

    double de = 0.0, sc = 0.0;
    uint32_t terms = 0;  // wave totals (popcounts of ballots)
    // intramolecular pairs touching a changed atom: pair (i, j), i < j, on
    // lane 0 .. 5 in the order (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
    {
        const uint32_t i = lane < 3 ? 0u : (lane < 5 ? 1u : 2u);
        const uint32_t j = lane < 3 ? (uint32_t)lane + 1u : (lane < 5 ? (uint32_t)lane - 1u : 3u);
        const bool on = lane < 6 && j < n && (((changed >> i) | (changed >> j)) & 1u);
        bool ino = false, inn = false, fino = false, finn = false;
        if (on) {
            const double xi = fx_pick(ox, i), yi = fx_pick(oy, i), zi = fx_pick(oz, i);
            const double xj = fx_pick(ox, j), yj = fx_pick(oy, j), zj = fx_pick(oz, j);
            const double xin = fx_pick(nx, i), yin = fx_pick(ny, i), zin = fx_pick(nz, i);
            const double xjn = fx_pick(nx, j), yjn = fx_pick(ny, j), zjn = fx_pick(nz, j);
            const double dxo = fx_mi(xi - xj, D.L, D.invL), dyo = fx_mi(yi - yj, D.L, D.invL),
                         dzo = fx_mi(zi - zj, D.L, D.invL);
            const double dxn = fx_mi(xin - xjn, D.L, D.invL), dyn = fx_mi(yin - yjn, D.L, D.invL),
                         dzn = fx_mi(zin - zjn, D.L, D.invL);
            const double r2o = dxo * dxo + dyo * dyo + dzo * dzo;
            const double r2n = dxn * dxn + dyn * dyn + dzn * dzn;
            const double so = 0.5 * (fx_pick(sig, fx_pick(ot, i)) + fx_pick(sig, fx_pick(ot, j)));
            const double sn = 0.5 * (fx_pick(sig, fx_pick(nt, i)) + fx_pick(sig, fx_pick(nt, j)));
            const double uo = fx_wca(so * so, r2o, D.rc2f), un = fx_wca(sn * sn, r2n, D.rc2f);
            ino = r2o < D.rc2f * so * so;
            inn = r2n < D.rc2f * sn * sn;
            de = un - uo;
            sc = un + uo;
            if ((D.bonded >> (4 * i + j)) & 1u) {
                // the change of Eq. (2) in one logarithm: the ratio of the
                // arguments before and after; +inf at or beyond the limit
                const double lo2 = 2.25 * so * so, ln2 = 2.25 * sn * sn;
                fino = r2o < lo2;
                finn = r2n < ln2;
                if (fino && finn)
                    de += -33.75 * log((1.0 - r2n / ln2) / (1.0 - r2o / lo2));
                else
                    de += (finn ? 0.0 : __builtin_inf()) - (fino ? 0.0 : __builtin_inf());
                if (logging) sc += fx_fene(so, r2o) + fx_fene(sn, r2n);
            }
        }
        terms += (uint32_t)__popcll(__ballot(ino)) + (uint32_t)__popcll(__ballot(inn)) +
                 (uint32_t)__popcll(__ballot(fino)) + (uint32_t)__popcll(__ballot(finn));
    }
    // intermolecular pairs: for each changed atom, the atoms of the 27 cells
    // around the cell it was sorted into this sweep, a lane each (cells are at
    // least r_c + 2 sqrt(3) d wide, and either atom has moved at most
    // sqrt(3) d since the sort, so every partner within r_c is there)
#pragma unroll
    for (uint32_t s = 0; s < 4; ++s) {
        if (!((changed >> s) & 1u)) continue;  // wave-uniform
        const uint32_t cy_id = V.cell_id[base + s];
        bool listed = ncand != 0xFFFFFFFFu && cy_id == cell;  // wave-uniform
        if (!listed && ncand != 0xFFFFFFFFu && flip) {
            // an atom of another cell whose type changes (its position does
            // not) is served by the list too when every atom that can reach
            // it was sorted into the list's 27 cells: those within the largest
            // cut-off now were within it plus sqrt(3) d at the sort
            const double m = sqrt(D.rc2f) * fmax(fmax(sig[0], sig[1]), fmax(sig[2], sig[3])) +
                             1.7320508075688772 * D.dmax + 1e-9;
            const uint32_t nc = D.nc;
            listed = fx_in_stencil(ox[s], h[0], cell % nc, D, m) &&
                     fx_in_stencil(oy[s], h[1], (cell / nc) % nc, D, m) &&
                     fx_in_stencil(oz[s], h[2], cell / (nc * nc), D, m);
        }
        uint32_t total = ncand;
        int nseg = 0;
        if (!listed) {
            const uint32_t ux = cy_id % D.nc, uy = (cy_id / D.nc) % D.nc, uz = cy_id / (D.nc * D.nc);
            nseg = fx_segments(D, V, (int)ux, (int)uy, (int)uz, 1, W, &total);
        }
        const double sos = fx_pick(sig, ot[s]), sns = fx_pick(sig, nt[s]);
        for (uint32_t b = 0; b < total; b += 64u) {
            const uint32_t idx = b + (uint32_t)lane;
            uint32_t j = 0xFFFFFFFFu;
            if (idx < total) j = listed ? W.cand[idx] : fx_stencil_atom(V, W, nseg, idx);
            const bool valid = j != 0xFFFFFFFFu && j - base >= n;  // not an atom of the molecule
            double xj = 0.0, yj = 0.0, zj = 0.0;
            uint32_t tj = 0;
            if (valid) {
                xj = V.pos[j]; yj = V.pos[N + j]; zj = V.pos[2 * N + j];
                tj = V.type[j];
            }
            const double sj = fx_pick(sig, tj);
            const double dxo = fx_mi(ox[s] - xj, D.L, D.invL), dyo = fx_mi(oy[s] - yj, D.L, D.invL),
                         dzo = fx_mi(oz[s] - zj, D.L, D.invL);
            const double r2o = valid ? dxo * dxo + dyo * dyo + dzo * dzo : 1e30;
            double r2n = r2o;
            if (!flip) {
                const double dxn = fx_mi(nx[s] - xj, D.L, D.invL), dyn = fx_mi(ny[s] - yj, D.L, D.invL),
                             dzn = fx_mi(nz[s] - zj, D.L, D.invL);
                r2n = valid ? dxn * dxn + dyn * dyn + dzn * dzn : 1e30;
            }
            const double so = 0.5 * (sos + sj);
            const double sn = 0.5 * (sns + sj);
            const double uo = fx_wca(so * so, r2o, D.rc2f), un = fx_wca(sn * sn, r2n, D.rc2f);
            de += un - uo;
            sc += un + uo;
            terms += (uint32_t)__popcll(__ballot(r2o < D.rc2f * so * so)) +
                     (uint32_t)__popcll(__ballot(r2n < D.rc2f * sn * sn));
        }
    }
    const double dE = wave_sum_dpp(de);
    const double S = logging ? wave_sum_dpp(sc) : 0.0;
    const bool accept = (dE <= 0.0) || (pr.thr < -dE);
    wc.terms += terms;
    if (accept) {
        if (flip) wc.acc_f += 1; else wc.acc_t += 1;
        wc.e += dE;
    }
    if (lane == 0) {
        if (accept) {
            if (flip) {
#pragma unroll
                for (uint32_t s = 0; s < 4; ++s)
                    if ((changed >> s) & 1u) V.type[base + s] = (uint8_t)nt[s];
            } else {
                V.pos[a] = wx;
                V.pos[N + a] = wy;
                V.pos[2 * N + a] = wz;
                // periodic images crossed (the shifts the wrap took off)
                const int ix = (int)floor(pr.tx / D.L), iy = (int)floor(pr.ty / D.L),
                          iz = (int)floor(pr.tz / D.L);
                if (ix) D.img[a] += ix;
                if (iy) D.img[N + a] += iy;
                if (iz) D.img[2 * N + a] += iz;
            }
        }
        if (logging) {
            MoveRecord rec;
            rec.delta_e = dE; rec.scale = S; rec.t_log_u = pr.thr; rec.sweep = sweep;
            rec.molecule = a; rec.move = flip ? MC_FLIP : MC_TRANSLATE; rec.accepted = accept ? 1 : 0;
            rec.exited = 0; rec.axis = (uint8_t)pr.kind; rec.pair_terms = terms; rec.pad = 0;
            D.log[(sweep - D.log_sweep0) * N + a] = rec;
        }
    }
    wave_lds_sync();
}

// Ascending atom index inside every cell of c0, c0 + cstep, ...: one wave per
// cell, a lane per atom whose place is the number of smaller indices (a cell
// of more than 64 atoms is sorted by one lane).
__device__ void fx_sort_cells(uint32_t* list, const uint32_t* start, uint32_t c0, uint32_t cstep,
                              uint32_t ncell)
{
    const uint32_t lane = (uint32_t)__lane_id();
    for (uint32_t c = c0; c < ncell; c += cstep) {
        const uint32_t b = start[c], cnt = start[c + 1] - b;
        if (cnt <= 1u) continue;
        if (cnt <= 64u) {
            const uint32_t v = lane < cnt ? list[b + lane] : 0xFFFFFFFFu;
            uint32_t rank = 0;
            for (uint32_t q = 0; q < cnt; ++q) rank += (uint32_t)__builtin_amdgcn_readlane((int)v, (int)q) < v;
            wave_lds_sync();
            if (lane < cnt) list[b + rank] = v;
        } else if (lane == 0) {
            for (uint32_t i = b + 1; i < b + cnt; ++i) {
                const uint32_t x = list[i];
                uint32_t q = i;
                while (q > b && list[q - 1] > x) {
                    list[q] = list[q - 1];
                    --q;
                }
                list[q] = x;
            }
        }
        wave_lds_sync();
    }
}

// The hot kernel: n sweeps of one system on one workgroup.  With kRes the
// positions, types and cell lists live in LDS for the whole launch (copied in
// at the start, positions and types written back at the end); otherwise the
// same code runs on the arrays in the system's buffer.
template <bool kRes>
__global__ void __launch_bounds__(kFxThreads) k_fx_sweeps(FxList list, uint64_t n_sweeps)
{
    FxDev* __restrict__ Dp = list.d[blockIdx.x];
    __shared__ uint32_t seg[kFxWaves][2][kFxSeg];
    __shared__ uint32_t cand[kFxWaves][kFxCand];
    __shared__ uint32_t scratch[kFxWaves];
    __shared__ double misc[2];
    __shared__ double dmax2[kFxWaves];
    extern __shared__ __align__(16) unsigned char fx_smem[];
    const FxDev& D = *Dp;
    const FxK K = fx_const(D);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    FxWaveLds W{seg[wave][0], seg[wave][1], cand[wave]};
    Stats* st = D.stats;
    const uint32_t N = D.N, ncell = D.ncell, nc = D.nc, k = D.k;
    FxView V{D.pos, D.type, D.cell_start, D.cell_list, D.cell_id, D.ecell};
    if (kRes) {
        const FxLds l = fx_lds_layout(N, ncell);
        V = FxView{(double*)(fx_smem + l.pos), (uint8_t*)(fx_smem + l.type), (uint32_t*)(fx_smem + l.cstart),
                   (uint32_t*)(fx_smem + l.clist), (uint32_t*)(fx_smem + l.cid), (double*)(fx_smem + l.ecell)};
        for (uint32_t i = tid; i < 3 * N; i += kFxThreads) V.pos[i] = D.pos[i];
        for (uint32_t i = tid; i < N; i += kFxThreads) V.type[i] = D.type[i];
        __syncthreads();
    }
    const uint32_t na = nc / k, nact = na * na * na;
    uint64_t sweep = st->sweep;
    const uint64_t origin = st->obs_origin;
    if (tid == 0) misc[0] = st->e_acc;
    FxCount wc{};
    for (uint64_t it = 0; it < n_sweeps; ++it) {
        const U4 g = philox10(0xFFFFFFFFu, (uint32_t)sweep, (uint32_t)(sweep >> 32), 3u, K.seed_lo, K.seed_hi);
        const double h[3] = {K.w * unit_open(g.x), K.w * unit_open(g.y), K.w * unit_open(g.z)};
        // counting sort of the atoms by cell
        for (uint32_t c = tid; c <= ncell; c += kFxThreads) V.cell_start[c] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < N; i += kFxThreads) {
            const uint32_t c = fx_cell(V.pos[i], V.pos[N + i], V.pos[2 * N + i], h, K);
            V.cell_id[i] = c;
            atomicAdd(&V.cell_start[c + 1], 1u);
        }
        __syncthreads();
        block_excl_scan_t<kFxThreads>(V.cell_start + 1, ncell, scratch);
        for (uint32_t i = tid; i < N; i += kFxThreads)
            V.cell_list[atomicAdd(&V.cell_start[V.cell_id[i] + 1], 1u)] = i;
        __syncthreads();
        fx_sort_cells(V.cell_list, V.cell_start, (uint32_t)wave, kFxWaves, ncell);
        __syncthreads();
        const bool logging = D.log != nullptr && sweep - D.log_sweep0 < D.log_sweeps;
        // The cells of a colour are attempted in ascending index; they run
        // side by side when no attempt in one can reach an atom another
        // reads or writes.  Two attempted atoms of different cells are at
        // least the gap (k - 1) w apart, and their attempts can meet only
        // through pairs within r_c of their molecules' atoms: so the cells
        // cannot interact when the gap is at least 2 D_c + r_c, D_c the
        // largest atom distance inside a molecule with an atom in the
        // colour's cells at the colour's start plus 2 sqrt(3) d (each atom
        // moves at most once per sweep).  Otherwise one cell at a time, in
        // that order: the same chain either way.
        auto colour_together = [&](uint32_t kx, uint32_t ky, uint32_t kz) __attribute__((always_inline)) {
            if (K.together != 0u) return K.together == 1u;
            double d2 = 0.0;
            const uint32_t n = K.n;
            for (uint32_t ci = (uint32_t)wave; ci < nact; ci += kFxWaves) {
                const uint32_t cell = (kx + k * (ci % na)) + nc * ((ky + k * ((ci / na) % na)) +
                                                                  nc * (kz + k * (ci / (na * na))));
                const uint32_t b = V.cell_start[cell], e = V.cell_start[cell + 1];
                for (uint32_t q = b + (uint32_t)lane; q < e; q += 64u) {
                    const uint32_t base = n * (V.cell_list[q] / n);
                    for (uint32_t i = 0; i + 1 < n; ++i)
                        for (uint32_t j = i + 1; j < n; ++j) {
                            const double dx = fx_mi(V.pos[base + i] - V.pos[base + j], K.L, K.invL);
                            const double dy = fx_mi(V.pos[N + base + i] - V.pos[N + base + j], K.L, K.invL);
                            const double dz =
                                fx_mi(V.pos[2 * N + base + i] - V.pos[2 * N + base + j], K.L, K.invL);
                            d2 = fmax(d2, dx * dx + dy * dy + dz * dz);
                        }
                }
            }
#pragma unroll
            for (int o = 32; o; o >>= 1) d2 = fmax(d2, __shfl_xor(d2, o));
            if (lane == 0) dmax2[wave] = d2;
            __syncthreads();
            double dm = 0.0;
            for (int w2 = 0; w2 < kFxWaves; ++w2) dm = fmax(dm, dmax2[w2]);
            __syncthreads();
            return K.sep >= 2.0 * sqrt(dm) + K.dyn_base;
        };
        // the attempts of cell `ci` of a colour by this wave
        auto run_cell = [&](uint32_t kx, uint32_t ky, uint32_t kz, uint32_t ci) __attribute__((always_inline)) {
            const uint32_t cell = (kx + k * (ci % na)) + nc * ((ky + k * ((ci / na) % na)) +
                                                              nc * (kz + k * (ci / (na * na))));
            wc.e = 0.0;
            const uint32_t b = V.cell_start[cell], e = V.cell_start[cell + 1];
            if (b < e) {
                const uint32_t ncand = fx_gather_candidates(K, V, cell, W);
                for (uint32_t q0 = b; q0 < e; q0 += 64u) {
                    const uint32_t cnt = min(64u, e - q0);
                    uint32_t at = 0;
                    FxProp pr{};
                    if ((uint32_t)lane < cnt) {
                        at = V.cell_list[q0 + lane];
                        pr = fx_propose(K, V, at, sweep, h, cell);
                    }
                    for (uint32_t q = 0; q < cnt; ++q)
                        fx_attempt(K, V, (uint32_t)__builtin_amdgcn_readlane((int)at, (int)q),
                                   fx_prop_of_lane(pr, (int)q), sweep, h, cell, ncand, logging, W, wc);
                }
            }
            if (lane == 0) V.ecell[cell] = wc.e;
        };
        for (uint32_t col = 0; col < k * k * k; ++col) {
            const uint32_t kx = col % k, ky = (col / k) % k, kz = col / (k * k);
            if (colour_together(kx, ky, kz)) {
                for (uint32_t ci = (uint32_t)wave; ci < nact; ci += kFxWaves) run_cell(kx, ky, kz, ci);
                __syncthreads();
            } else {
                for (uint32_t ci = 0; ci < nact; ++ci) {
                    if (ci % kFxWaves == (uint32_t)wave) run_cell(kx, ky, kz, ci);
                    __syncthreads();
                }
            }
        }
        ++sweep;
        // E_acc += the sweep's dE, the cells in a fixed order; E/M samples
        if (wave == 0) {
            const double e = misc[0] + sweep_energy(V.ecell, ncell);
            if (lane == 0) misc[0] = e;
        }
        if (tid == 0) {
            const uint64_t t = sweep - origin;
            if (t >= D.obs_start && D.obs_interval && t % D.obs_interval == 0) {
                const double em = misc[0] / (double)D.M;
                if (st->n_e < D.max_samples) D.e_samples[st->n_e] = em;
                st->n_e += 1;
                st->e_sum += em;
                st->e_sumsq += em * em;
            }
        }
        __syncthreads();
    }
    if (lane == 0) {
        if (wc.att_t) atomicAdd((unsigned long long*)&st->attempts[MC_TRANSLATE], (unsigned long long)wc.att_t);
        if (wc.att_f) atomicAdd((unsigned long long*)&st->attempts[MC_FLIP], (unsigned long long)wc.att_f);
        if (wc.acc_t) atomicAdd((unsigned long long*)&st->accepts[MC_TRANSLATE], (unsigned long long)wc.acc_t);
        if (wc.acc_f) atomicAdd((unsigned long long*)&st->accepts[MC_FLIP], (unsigned long long)wc.acc_f);
        if (wc.exits) atomicAdd((unsigned long long*)&st->exits, (unsigned long long)wc.exits);
        if (wc.terms) atomicAdd((unsigned long long*)&st->pair_terms, (unsigned long long)wc.terms);
    }
    __syncthreads();
    if (kRes) {
        for (uint32_t i = tid; i < 3 * N; i += kFxThreads) D.pos[i] = V.pos[i];
        for (uint32_t i = tid; i < N; i += kFxThreads) D.type[i] = V.type[i];
    }
    if (tid == 0) {
        st->sweep = sweep;
        st->e_acc = misc[0];
    }
}

}  // namespace
}  // namespace flipmc
