// kernels.hip -- gfx950 kernels of the flip Monte Carlo engine.
//
// Method (Simon, Barrat & Berthier, Sec. II): Metropolis sweeps over rigid
// triangular A/B/C molecules with the site-site WCA potential (Eq. 1), mixing
// translations, rotations and the intramolecular flip of Sec. II.B.
//
// Execution model: one workgroup of 8 wave64s owns one system for the whole
// launch and runs many sweeps back to back.  A sweep is a checkerboard over a
// randomly shifted cubic cell grid: the k^3 colours run one after another, the
// cells of one colour are spread over the 8 waves, and the molecules of a
// cell are tried in ascending index by that wave.  Cells of one colour are at
// least (k-1) cells apart, farther than any two molecules can interact, so the
// waves never race.  Inside a trial the 64 lanes share the energy difference:
// the molecules near the cell (built once per cell) are pruned against the
// trial molecule's centre, the survivors' sites that can reach a moved site are
// compacted into a per-wave LDS buffer, one 64-lane pass evaluates them against
// the moved sites before and after the move, and a DPP reduction in FP64 gives
// dE in a fixed order.  Proposals of all molecules of a sweep are drawn in
// parallel before its first colour; the lane that holds a molecule's proposal
// publishes its moved sites and commits the accepted move.
//
// The random numbers are Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11)
// keyed by the seed and counted by (molecule, sweep low, sweep high, tag), so a
// run is reproducible regardless of how systems are batched.
#include "engine.h"
#include "wave.h"



namespace flipmc {
namespace {

// Sum over the workgroup in a fixed order (identical bits in every thread).
__device__ double block_sum(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kWaves; ++i) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ void block_excl_scan(uint32_t* a, uint32_t n, uint32_t* scratch)
{
    block_excl_scan_t<kThreads>(a, n, scratch);
}

// --------------------------------------------------------------- geometry --

__device__ __forceinline__ double wrap(double x, double L) { return x - L * floor(x / L); }

__device__ __forceinline__ double min_image(double d, double L, double invL)
{
    return d - L * rint(d * invL);
}

__device__ __forceinline__ int cell_axis(double x, double h, double L, double w, int nc)
{
    const double g = wrap(x - h, L);
    int c = (int)floor(g / w);
    c = c < 0 ? 0 : c;
    return c >= nc ? nc - 1 : c;
}

__device__ __forceinline__ void rotation(double qw, double qx, double qy, double qz, double r[9])
{
    r[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
    r[1] = 2.0 * (qx * qy - qw * qz);
    r[2] = 2.0 * (qx * qz + qw * qy);
    r[3] = 2.0 * (qx * qy + qw * qz);
    r[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
    r[5] = 2.0 * (qy * qz - qw * qx);
    r[6] = 2.0 * (qx * qz - qw * qy);
    r[7] = 2.0 * (qy * qz + qw * qx);
    r[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
}

// Shifted WCA of Eq. (1) written as (2 (s/r)^6 - 1)^2, given s^2 and r^2.
__device__ __forceinline__ float pair_u(float s2, float r2)
{
    const float x = s2 * __builtin_amdgcn_rcpf(r2);
    const float x3 = x * x * x;
    const float t = fmaf(2.0f, x3, -1.0f);
    return t * t;
}
__device__ __forceinline__ double pair_u(double s2, double r2)
{
    // 1 / r2: the hardware estimate refined by two Newton steps (within an
    // ulp or two of the quotient; r2 is a normal number here)
    double y = __builtin_amdgcn_rcp(r2);
    y = fma(fma(-r2, y, 1.0), y, y);
    y = fma(fma(-r2, y, 1.0), y, y);
    const double x = s2 * y;
    const double x3 = x * x * x;
    const double t = fma(2.0, x3, -1.0);
    return t * t;
}

// Body-frame coordinate a of site s of the equilateral triangle.
template <class Cx>
__device__ __forceinline__ double body_at(const Cx& C, uint32_t s, int a)
{
    if (a == 0) return s == 0 ? C.bR : -0.5 * C.bR;
    if (a == 1) return s == 0 ? 0.0 : (s == 1 ? C.bH : -C.bH);
    return 0.0;
}

// Diameter of type t, from the 3-entry table in LDS (filled at kernel entry);
// a table lookup keeps the per-system constants out of dynamically indexed
// memory.
template <class Cx>
__device__ __forceinline__ double sigma_of(const Cx& C, uint32_t t)
{
    return C.misc[1 + t];
}

// ------------------------------------------------------------- per system --

// Everything a workgroup needs, copied from the system descriptor at kernel
// entry (before any store, so the copies are scalar loads kept in SGPRs) plus
// the LDS or HBM addresses of the work arrays.
template <typename Real, bool kRes>
struct Ctx {
    uint32_t M, k, nc, ncell, seed_lo, seed_hi;
    uint32_t resum_interval, obs_interval, gofr_interval, obs_start, max_samples, gofr_nbins;
    double L, invL, w, T, p_flip, p_ft, dmax, rot_max, reach2, radius, rc2_factor;
    double bR, bH;            // body frame: site 0 at (bR, 0, 0), sites 1, 2 at (-bR/2, +-bH, 0)
    double sig0, sig1, sig2;  // diameters of types A, B, C
    double gofr_dr, gofr_rmax;
    double fs_q, fs_q_cm;
    double* gcom;
    double* quat;
    uint32_t* types;
    double* u0;
    uint8_t* kref;
    int32_t* img;
    double* r0;
    double* o0;
    double* fs;
    double* fs_cm;
    double* mom;
    Stats* stats;
    double* e_samples;
    double* drift_samples;
    uint64_t* gofr_all;
    uint64_t* gofr_inter;
    double* c2;
    uint64_t* c2_sweep;
    MoveRecord* log;
    uint64_t log_sweep0, log_sweeps;
    double* gpart;
    // work arrays (LDS when resident)
    double* com;
    R4<Real>* site;
    uint32_t* cellb;
    uint16_t* cellid;
    uint16_t* list;
    double* red;
    double* ecell;  // accepted dE of each cell in the current sweep
    const double* off;  // FP64 site offsets [9][M] computed up front (event kernel), or null
    uint32_t* bins;
    double* misc;
};

// Proposal of one molecule for the current sweep.  All proposals of a sweep
// are drawn at its start by the whole workgroup (they depend only on the
// molecule's own state, which no earlier trial of the sweep can change) and
// kept in HBM; a wave loads those of a cell when it reaches the cell.
struct alignas(16) PropRec {
    uint32_t kind;  // move | exited << 4 | axis << 8
    uint32_t pad;
    double thr;     // T ln u_acc
    double a0, a1, a2, a3;  // translation: displacement a0..a2; rotation: new quaternion
};
static_assert(sizeof(PropRec) == 48, "proposal record");

template <typename Real, bool kRes>
__device__ PropRec propose(const Ctx<Real, kRes>& C, uint32_t m, uint64_t sweep, double hx,
                           double hy, double hz, int cx, int cy, int cz)
{
    PropRec p;
    const uint32_t slo = (uint32_t)sweep, shi = (uint32_t)(sweep >> 32);
    const U4 b0 = philox10(m, slo, shi, 0u, C.seed_lo, C.seed_hi);
    const U4 b1 = philox10(m, slo, shi, 1u, C.seed_lo, C.seed_hi);
    const double uacc = unit_53(b0.x, b0.y), ut = unit_open(b0.z);
    const double p0 = unit_open(b1.x), p1 = unit_open(b1.y), p2 = unit_open(b1.z);
    p.thr = C.T * log(uacc);
    const uint32_t move = ut < C.p_flip ? 2u : (ut < C.p_ft ? 0u : 1u);
    uint32_t exited = 0, axis = 255;
    const uint32_t M = C.M;
    p.pad = 0;
    p.a0 = p.a1 = p.a2 = p.a3 = 0.0;
    if (move == 0u) {
        const double c0 = C.com[m], c1 = C.com[M + m], c2 = C.com[2 * M + m];
        p.a0 = C.dmax * (2.0 * p0 - 1.0);
        p.a1 = C.dmax * (2.0 * p1 - 1.0);
        p.a2 = C.dmax * (2.0 * p2 - 1.0);
        const int nc = (int)C.nc;
        exited = (cell_axis(wrap(c0 + p.a0, C.L), hx, C.L, C.w, nc) != cx) ||
                 (cell_axis(wrap(c1 + p.a1, C.L), hy, C.L, C.w, nc) != cy) ||
                 (cell_axis(wrap(c2 + p.a2, C.L), hz, C.L, C.w, nc) != cz);
    } else if (move == 1u) {
        const double z = 2.0 * p0 - 1.0;
        const double phi = kTwoPi * p1;
        const double st = sqrt(1.0 - z * z);
        const double nx = st * cos(phi), ny = st * sin(phi), nz = z;
        const double th = C.rot_max * (2.0 * p2 - 1.0);
        const double ch = cos(0.5 * th), sh = sin(0.5 * th);
        const double dw = ch, dx = nx * sh, dy = ny * sh, dz = nz * sh;
        const double qw = C.quat[m], qx = C.quat[M + m], qy = C.quat[2 * M + m],
                     qz = C.quat[3 * M + m];
        const double rw = dw * qw - dx * qx - dy * qy - dz * qz;
        const double rx = dw * qx + dx * qw + dy * qz - dz * qy;
        const double ry = dw * qy - dx * qz + dy * qw + dz * qx;
        const double rz = dw * qz + dx * qy - dy * qx + dz * qw;
        const double nrm = sqrt(rw * rw + rx * rx + ry * ry + rz * rz);
        p.a0 = rw / nrm; p.a1 = rx / nrm; p.a2 = ry / nrm; p.a3 = rz / nrm;
    } else {
        int a = (int)(3.0 * p0);
        axis = (uint32_t)(a > 2 ? 2 : a);
    }
    p.kind = move | (exited << 4) | (axis << 8);
    return p;
}

// Proposals of every molecule for this sweep (after the cell build).
template <typename Real, bool kRes>
__device__ void propose_all(const Ctx<Real, kRes>& C, PropRec* props, uint64_t sweep, double hx,
                            double hy, double hz)
{
    const int nc = (int)C.nc;
    for (uint32_t m = threadIdx.x; m < C.M; m += kThreads) {
        const int cid = C.cellid[m];
        const int cx = cid % nc, cy = (cid / nc) % nc, cz = cid / (nc * nc);
        props[m] = propose(C, m, sweep, hx, hy, hz, cx, cy, cz);
    }
}

template <typename Real, bool kRes>
__device__ __forceinline__ void store_sites_from_quat(const Ctx<Real, kRes>& C, uint32_t m)
{
    const uint32_t M = C.M;
    double r[9];
    rotation(C.quat[m], C.quat[M + m], C.quat[2 * M + m], C.quat[3 * M + m], r);
    const uint32_t ty = C.types[m];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        R4<Real> v;
        v.x = (Real)(r[0] * body_at(C, s, 0) + r[1] * body_at(C, s, 1) + r[2] * body_at(C, s, 2));
        v.y = (Real)(r[3] * body_at(C, s, 0) + r[4] * body_at(C, s, 1) + r[5] * body_at(C, s, 2));
        v.z = (Real)(r[6] * body_at(C, s, 0) + r[7] * body_at(C, s, 1) + r[8] * body_at(C, s, 2));
        v.w = (Real)sigma_of(C, (ty >> (8 * s)) & 0xFFu);
        C.site[3 * m + s] = v;
    }
}

// FP64 offsets of molecule m straight from its quaternion, plus site sigmas.
template <typename Real, bool kRes>
__device__ __forceinline__ void offsets_f64(const Ctx<Real, kRes>& C, uint32_t m, double o[9],
                                            double sg[3])
{
    const uint32_t M = C.M;
    if (C.off) {
#pragma unroll
        for (int i = 0; i < 9; ++i) o[i] = C.off[i * M + m];
    } else {
        double r[9];
        rotation(C.quat[m], C.quat[M + m], C.quat[2 * M + m], C.quat[3 * M + m], r);
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                o[3 * s + a] = r[3 * a] * body_at(C, s, 0) + r[3 * a + 1] * body_at(C, s, 1) +
                               r[3 * a + 2] * body_at(C, s, 2);
    }
    const uint32_t ty = C.types[m];
#pragma unroll
    for (int s = 0; s < 3; ++s) sg[s] = sigma_of(C, (ty >> (8 * s)) & 0xFFu);
}

// Total inter-molecular energy in FP64 over balanced molecule pairs.
template <typename Real, bool kRes>
__device__ double resum_energy(const Ctx<Real, kRes>& C, uint32_t m0, uint32_t mstep)
{
    const uint32_t M = C.M, half = M / 2;
    double e = 0.0;
    for (uint32_t m = m0; m < M; m += mstep) {
        double om[9], sm[3];
        offsets_f64(C, m, om, sm);
        const double cx = C.com[m], cy = C.com[M + m], cz = C.com[2 * M + m];
        for (uint32_t dj = 1; dj <= half; ++dj) {
            if ((M & 1u) == 0u && dj == half && m >= half) break;
            uint32_t j = m + dj;
            if (j >= M) j -= M;
            const double dx = min_image(C.com[j] - cx, C.L, C.invL);
            const double dy = min_image(C.com[M + j] - cy, C.L, C.invL);
            const double dz = min_image(C.com[2 * M + j] - cz, C.L, C.invL);
            if (dx * dx + dy * dy + dz * dz >= C.reach2) continue;
            double oj[9], sj[3];
            offsets_f64(C, j, oj, sj);
#pragma unroll
            for (int s = 0; s < 3; ++s)
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const double rx = dx + oj[3 * t] - om[3 * s];
                    const double ry = dy + oj[3 * t + 1] - om[3 * s + 1];
                    const double rz = dz + oj[3 * t + 2] - om[3 * s + 2];
                    const double r2 = rx * rx + ry * ry + rz * rz;
                    const double sg = 0.5 * (sm[s] + sj[t]);
                    const double s2 = sg * sg;
                    if (r2 < C.rc2_factor * s2) e += pair_u(s2, r2);
                }
        }
    }
    return block_sum(e, C.red);
}

// The same total from the cell lists of the last sweep (HBM state): a
// molecule has moved at most sqrt(3) d_max since they were built, so every
// pair within reach lies within `span` cells per axis of the cell it was
// sorted into.  Each pair is counted by its lower index, the neighbour cells
// in a fixed order and the molecules of a cell in ascending index.
// Requires 2 span + 1 <= n_c.
template <typename Real, bool kRes>
__device__ double resum_energy_cells(const Ctx<Real, kRes>& C, uint32_t m0, uint32_t mstep, int span)
{
    const uint32_t M = C.M;
    const int nc = (int)C.nc;
    double e = 0.0;
    for (uint32_t m = m0; m < M; m += mstep) {
        double om[9], sm[3];
        offsets_f64(C, m, om, sm);
        const double cx = C.com[m], cy = C.com[M + m], cz = C.com[2 * M + m];
        const int cid = (int)C.cellid[m];
        const int ix = cid % nc, iy = (cid / nc) % nc, iz = cid / (nc * nc);
        for (int oz = -span; oz <= span; ++oz)
            for (int oy = -span; oy <= span; ++oy)
                for (int ox = -span; ox <= span; ++ox) {
                    const int x = (ix + ox + nc) % nc, y = (iy + oy + nc) % nc, z = (iz + oz + nc) % nc;
                    const uint32_t c = (uint32_t)(x + nc * (y + nc * z));
                    const uint32_t pe = C.cellb[c + 1];
                    for (uint32_t p = C.cellb[c]; p < pe; ++p) {
                        const uint32_t j = C.list[p];
                        if (j <= m) continue;
                        const double dx = min_image(C.com[j] - cx, C.L, C.invL);
                        const double dy = min_image(C.com[M + j] - cy, C.L, C.invL);
                        const double dz = min_image(C.com[2 * M + j] - cz, C.L, C.invL);
                        if (dx * dx + dy * dy + dz * dz >= C.reach2) continue;
                        double oj[9], sj[3];
                        offsets_f64(C, j, oj, sj);
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int t = 0; t < 3; ++t) {
                                const double rx = dx + oj[3 * t] - om[3 * a];
                                const double ry = dy + oj[3 * t + 1] - om[3 * a + 1];
                                const double rz = dz + oj[3 * t + 2] - om[3 * a + 2];
                                const double r2 = rx * rx + ry * ry + rz * rz;
                                const double sg = 0.5 * (sm[a] + sj[t]);
                                const double s2 = sg * sg;
                                if (r2 < C.rc2_factor * s2) e += pair_u(s2, r2);
                            }
                    }
                }
    }
    return block_sum(e, C.red);
}

__device__ __forceinline__ bool is_c2_time(uint64_t t)
{
    if (t == 0) return false;
    while (t % 10 == 0) t /= 10;
    return t == 1 || t == 2 || t == 5;
}

// sin(x) / x, with its Taylor value near 0.
__device__ __forceinline__ double sinc(double x)
{
    return x < 1e-4 ? 1.0 - x * x / 6.0 : sin(x) / x;
}

// The time correlations of one sample (Sec. III.B) and the moments of their
// per-particle contributions (Sec. V.A) that the four-point susceptibilities
// and the Pearson coefficient (Sec. V.B and V.C) are built from:
//   C_2^i    = P_2(u_i(t) . u_i(0)), u following the site that held type B
//              at the observable origin (Eq. 7, l = 2),
//   F_s^cm,i = sin(q d)/(q d) at |q| = C.fs_q_cm, d the displacement of the
//              unwrapped centre (Eq. 6 averaged over all directions of q),
//   F_s^i    = the same over each site index at |q| = C.fs_q (Eq. 5); a
//              site keeps its index through a flip, so a flip moves no site.
// Centres are unwrapped with the image counts of the accepted translations.
// d[0..6] = means of C_2^i, (C_2^i)^2, F_s^cm,i, (F_s^cm,i)^2, C_2^i F_s^cm,i
// over molecules and of F_s^i, (F_s^i)^2 over sites.
constexpr int kDyn = 7;

template <typename Real, bool kRes>
__device__ void dyn_values(const Ctx<Real, kRes>& C, double d[kDyn])
{
    const uint32_t M = C.M;
    double a[kDyn];
#pragma unroll
    for (int j = 0; j < kDyn; ++j) a[j] = 0.0;
    for (uint32_t m = threadIdx.x; m < M; m += kThreads) {
        double o[9], sg[3];
        offsets_f64(C, m, o, sg);
        const int k = C.kref[m];
        double dot = 0.0;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const double okx = k == 0 ? o[x] : (k == 1 ? o[3 + x] : o[6 + x]);
            dot += (okx / C.radius) * C.u0[x * M + m];
        }
        const double c2 = 0.5 * (3.0 * dot * dot - 1.0);
        double dc[3];
#pragma unroll
        for (int x = 0; x < 3; ++x)
            dc[x] = (C.com[x * M + m] + C.L * (double)C.img[x * M + m]) - C.r0[x * M + m];
        const double fcm = sinc(C.fs_q_cm * sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]));
        a[0] += c2; a[1] += c2 * c2; a[2] += fcm; a[3] += fcm * fcm; a[4] += c2 * fcm;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const double ex = dc[0] + (o[3 * t] - C.o0[(3 * t) * M + m]);
            const double ey = dc[1] + (o[3 * t + 1] - C.o0[(3 * t + 1) * M + m]);
            const double ez = dc[2] + (o[3 * t + 2] - C.o0[(3 * t + 2) * M + m]);
            const double f = sinc(C.fs_q * sqrt(ex * ex + ey * ey + ez * ez));
            a[5] += f; a[6] += f * f;
        }
    }
#pragma unroll
    for (int j = 0; j < kDyn; ++j) d[j] = block_sum(a[j], C.red) / ((j < 5 ? 1.0 : 3.0) * (double)M);
}

// One sample of the time correlations at the current sweep.
template <typename Real, bool kRes>
__device__ void store_dyn(const Ctx<Real, kRes>& C, Stats* st, uint64_t t)
{
    double d[kDyn];
    dyn_values(C, d);
    if (threadIdx.x == 0 && st->n_c2 < kC2Max) {
        const uint32_t n = st->n_c2;
        C.c2[n] = d[0];
        C.fs_cm[n] = d[2];
        C.fs[n] = d[5];
        C.mom[n] = d[1];
        C.mom[kC2Max + n] = d[3];
        C.mom[2 * kC2Max + n] = d[4];
        C.mom[3 * kC2Max + n] = d[6];
        C.c2_sweep[n] = t;
        st->n_c2 = n + 1;
    }
}

template <typename Real, bool kRes>
__device__ void reset_observables(const Ctx<Real, kRes>& C)
{
    const uint32_t M = C.M;
    for (uint32_t m = threadIdx.x; m < M; m += kThreads) {
        // F_s references: unwrapped centre and site offsets
        double o[9], sg[3];
        offsets_f64(C, m, o, sg);
#pragma unroll
        for (int i = 0; i < 9; ++i) C.o0[i * M + m] = o[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) C.r0[k * M + m] = C.com[k * M + m] + C.L * (double)C.img[k * M + m];
        const uint32_t ty = C.types[m];
        int k = 0;
        for (int s = 0; s < 3; ++s)
            if (((ty >> (8 * s)) & 0xFFu) == 1u) k = s;
        C.kref[m] = (uint8_t)k;
        double r[9];
        rotation(C.quat[m], C.quat[M + m], C.quat[2 * M + m], C.quat[3 * M + m], r);
        for (int a = 0; a < 3; ++a)
            C.u0[a * M + m] = (r[3 * a] * body_at(C, k, 0) + r[3 * a + 1] * body_at(C, k, 1) +
                               r[3 * a + 2] * body_at(C, k, 2)) / C.radius;
    }
    for (uint32_t b = threadIdx.x; b < kGofrBins; b += kThreads) {
        C.gofr_all[b] = 0;
        C.gofr_inter[b] = 0;
    }
    if (threadIdx.x == 0) {
        Stats* st = C.stats;
        st->obs_origin = st->sweep;
        st->n_e = st->n_drift = st->n_gofr = st->n_c2 = 0;
        st->e_sum = st->e_sumsq = 0.0;
        st->max_abs_drift = 0.0;
    }
}

// One g(r) frame (Eq. 3 numerator): every ordered pair of distinct sites.
template <typename Real, bool kRes>
__device__ void gofr_frame(const Ctx<Real, kRes>& C, uint32_t m0, uint32_t mstep, bool shared_out,
                           uint32_t* queue)
{
    const uint32_t M = C.M, half = M / 2, nb = C.gofr_nbins;
    uint32_t* bintra = C.bins;  // intramolecular pairs; all = intra + inter at the end
    uint32_t* binter = C.bins + kGofrBins;
    uint32_t* q = queue + (threadIdx.x >> 6) * kGofrQueue;  // this wave's molecule pairs
    const uint32_t lane = (uint32_t)__lane_id();
    for (uint32_t b = threadIdx.x; b < 2 * kGofrBins; b += kThreads) C.bins[b] = 0;
    __syncthreads();
    const double dr = C.gofr_dr, rmax = C.gofr_rmax;
    const double cut = rmax + 2.0 * C.radius;
    const double cut2 = cut * cut;
    const float inv_dr = (float)(1.0 / dr);
    // bin floor(sqrt(r2) / dr) in FP64; an FP32 estimate decides unless it
    // lies within 2e-4 of a bin edge (its error stays below 1e-4 up to the last bin)
    auto bin = [&](double r2) __attribute__((always_inline)) {
        const float t = sqrtf((float)r2) * inv_dr;
        const float fl = floorf(t);
        int b = (int)fl;
        if (t - fl < 2e-4f || fl + 1.0f - t < 2e-4f) b = (int)floor(sqrt(r2) / dr);
        return b;
    };
    // the nine site pairs of molecules m, j (each with its own nearest image)
    auto site_pairs = [&](uint32_t m, uint32_t j) __attribute__((always_inline)) {
        double om[9], sm[3], oj[9], sj[3];
        offsets_f64(C, m, om, sm);
        offsets_f64(C, j, oj, sj);
        const double dx = min_image(C.com[j] - C.com[m], C.L, C.invL);
        const double dy = min_image(C.com[M + j] - C.com[M + m], C.L, C.invL);
        const double dz = min_image(C.com[2 * M + j] - C.com[2 * M + m], C.L, C.invL);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const double bx = dx + oj[3 * t], by = dy + oj[3 * t + 1], bz = dz + oj[3 * t + 2];
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                // r reaches L / 2
                const double rx = min_image(bx - om[3 * s], C.L, C.invL);
                const double ry = min_image(by - om[3 * s + 1], C.L, C.invL);
                const double rz = min_image(bz - om[3 * s + 2], C.L, C.invL);
                const int b = bin(rx * rx + ry * ry + rz * rz);
                if (b >= 0 && b < (int)nb) atomicAdd(&binter[b], 2u);
            }
        }
    };
    // the pairs within reach of the bins are queued per wave and binned 64 at
    // a time (the counts do not depend on the order)
    uint32_t qn = 0;
    auto drain = [&](uint32_t upto) __attribute__((always_inline)) {
        while (qn >= upto && qn > 0) {
            const uint32_t take = min(qn, 64u);
            const uint32_t base = qn - take;
            if (lane < take) {
                const uint32_t e = q[base + lane];
                site_pairs(e & 0xFFFFu, e >> 16);
            }
            qn = base;
        }
    };
    // rounds of the wave's first lane (the most of any lane): wave-uniform
    const uint32_t nrounds = (M + mstep - 1 - min(m0 - lane, M)) / mstep;
    for (uint32_t r = 0; r < nrounds; ++r) {
        const uint32_t m = m0 + r * mstep;
        const bool mine = m < M;
        if (mine) {
            double om[9], sm[3];
            offsets_f64(C, m, om, sm);
#pragma unroll
            for (int s = 0; s < 3; ++s)
#pragma unroll
                for (int t = s + 1; t < 3; ++t) {
                    const double rx = om[3 * t] - om[3 * s], ry = om[3 * t + 1] - om[3 * s + 1],
                                 rz = om[3 * t + 2] - om[3 * s + 2];
                    const int b = bin(rx * rx + ry * ry + rz * rz);
                    if (b >= 0 && b < (int)nb) atomicAdd(&bintra[b], 2u);
                }
        }
        const double cx = mine ? C.com[m] : 0.0, cy = mine ? C.com[M + m] : 0.0,
                     cz = mine ? C.com[2 * M + m] : 0.0;
        for (uint32_t dj = 1; dj <= half; ++dj) {
            bool keep = mine && !((M & 1u) == 0u && dj == half && m >= half);
            uint32_t j = m + dj;
            if (j >= M) j -= M;
            if (keep) {
                const double dx = min_image(C.com[j] - cx, C.L, C.invL);
                const double dy = min_image(C.com[M + j] - cy, C.L, C.invL);
                const double dz = min_image(C.com[2 * M + j] - cz, C.L, C.invL);
                keep = dx * dx + dy * dy + dz * dz < cut2;
            }
            const uint64_t bm = __ballot(keep);
            if (keep) q[qn + rank_below(bm)] = m | (j << 16);
            qn += (uint32_t)__popcll(bm);
            wave_lds_sync();
            drain(64u);
            wave_lds_sync();
        }
    }
    drain(1u);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        const uint32_t all = bintra[b] + binter[b];
        if (shared_out) {  // several workgroups add into the histograms
            if (all) atomicAdd((unsigned long long*)&C.gofr_all[b], (unsigned long long)all);
            if (binter[b]) atomicAdd((unsigned long long*)&C.gofr_inter[b], (unsigned long long)binter[b]);
        } else {
            C.gofr_all[b] += all;
            C.gofr_inter[b] += binter[b];
        }
    }
    if (threadIdx.x == 0 && !shared_out) C.stats->n_gofr += 1;
}

// Ascending molecule index inside every cell of cells c0, c0 + cstep, ...,
// one wave per cell and a lane per molecule: its new place is the number of
// smaller indices in the cell.  Up to 8 cells of a wave have their loads in
// flight together; a cell of more than 64 molecules is sorted by one lane.
__device__ void sort_cells(uint16_t* list, const uint32_t* cellb, uint32_t c0, uint32_t cstep,
                           uint32_t ncell)
{
    const uint32_t lane = (uint32_t)__lane_id();
    for (uint32_t cg = c0; cg < ncell; cg += 8u * cstep) {
        uint32_t b[8], n[8], v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint32_t c = cg + (uint32_t)r * cstep;
            b[r] = 0;
            n[r] = 0;
            if (c < ncell) {
                b[r] = cellb[c];
                n[r] = cellb[c + 1] - b[r];
            }
            b[r] = (uint32_t)__builtin_amdgcn_readfirstlane((int)b[r]);
            n[r] = (uint32_t)__builtin_amdgcn_readfirstlane((int)n[r]);
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = lane < n[r] && n[r] <= 64u ? list[b[r] + lane] : 0xFFFFu;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (n[r] <= 1u) continue;
            if (n[r] <= 64u) {
                uint32_t rank = 0;
                for (uint32_t q = 0; q < n[r]; ++q) rank += rl_u(v[r], (int)q) < v[r] ? 1u : 0u;
                if (lane < n[r]) list[b[r] + rank] = (uint16_t)v[r];
            } else if (lane == 0) {
                const uint32_t lo = b[r], hi = b[r] + n[r];
                for (uint32_t i = lo + 1; i < hi; ++i) {
                    const uint16_t x = list[i];
                    uint32_t q = i;
                    while (q > lo && list[q - 1] > x) {
                        list[q] = list[q - 1];
                        --q;
                    }
                    list[q] = x;
                }
            }
        }
    }
}

// Cell grid of one sweep: counting sort of molecules by cell.
template <typename Real, bool kRes>
__device__ void build_cells(const Ctx<Real, kRes>& C, double hx, double hy, double hz,
                            uint32_t* scratch)
{
    const uint32_t M = C.M, ncell = C.ncell;
    const int nc = (int)C.nc;
    for (uint32_t i = threadIdx.x; i <= ncell; i += kThreads) C.cellb[i] = 0;
    __syncthreads();
    for (uint32_t m = threadIdx.x; m < M; m += kThreads) {
        const int ix = cell_axis(C.com[m], hx, C.L, C.w, nc);
        const int iy = cell_axis(C.com[M + m], hy, C.L, C.w, nc);
        const int iz = cell_axis(C.com[2 * M + m], hz, C.L, C.w, nc);
        const uint32_t cid = (uint32_t)(ix + nc * (iy + nc * iz));
        C.cellid[m] = (uint16_t)cid;
        atomicAdd(&C.cellb[cid + 1], 1u);
    }
    __syncthreads();
    block_excl_scan(C.cellb + 1, ncell, scratch);
    for (uint32_t m = threadIdx.x; m < M; m += kThreads) {
        const uint32_t pos = atomicAdd(&C.cellb[C.cellid[m] + 1u], 1u);
        C.list[pos] = (uint16_t)m;
    }
    __syncthreads();
    sort_cells(C.list, C.cellb, threadIdx.x >> 6, kWaves, ncell);
    __syncthreads();
}

// Per-wave counters, kept in registers for the whole launch.
struct WaveCount {
    uint32_t att0, att1, att2, acc0, acc1, acc2, exits, overflows;
    uint64_t terms, tests;
    double e;  // accepted dE of the current sweep, in trial order
};

// The trial in flight, written by the lane that holds the molecule's proposal
// and read by the whole wave.
template <typename Real>
struct alignas(16) TrialLds {
    R4<Real> old_site[3];  // moved sites before the move: offset from the old centre + sigma
    R4<Real> new_site[3];  // after the move: offset from the new centre + sigma
    double cm[3];          // centre of mass before the move
    float mr[3];           // the same relative to the cell centre (pruning only)
    Real dl[3];            // displacement of a translation, zero for the other moves
    uint32_t info;         // molecule | move << 16
};
static_assert(sizeof(TrialLds<float>) <= trial_bytes(false), "trial record (FP32)");
static_assert(sizeof(TrialLds<double>) <= trial_bytes(true), "trial record (FP64)");

// A molecule near the current cell: its index and its centre relative to the
// cell centre (nearest image), rounded to FP16.  The coordinates only prune
// candidates (with a margin); the positions used for energies are formed from
// the FP64 centres.
struct alignas(8) NearEntry {
    uint16_t j;
    __fp16 rx, ry, rz;
};
static_assert(sizeof(NearEntry) == 8, "near-list entry");

// Per-wave LDS work areas.
template <typename Real>
struct WaveLds {
    uint16_t* surv;       // molecules that passed the prune of the trial in flight
    uint16_t* seglo;      // neighbour row segments of the current cell
    uint16_t* segoff;
    NearEntry* near;      // molecules near the current cell
    TrialLds<Real>* tr;
};

// Neighbour cells of cell (cx, cy, cz) as row segments along x: (2r+1)^2 rows
// of 1 or 2 x-ranges (r = k - 1).  Writes the segment table, returns the
// number of segments and the number of molecules they hold.
template <typename Real, bool kRes>
__device__ __forceinline__ int stencil_segments(const Ctx<Real, kRes>& C, int cx, int cy, int cz,
                                                uint16_t* seglo, uint16_t* segoff, uint32_t* total)
{
    const int lane = __lane_id();
    const int nc = (int)C.nc;
    const int r = (int)C.k - 1;
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
    uint32_t scnt = 0, slo = 0;
    if (lane < nseg) {
        const int ixr = lane % nxr, iy = (lane / nxr) % nrow, iz = lane / (nxr * nrow);
        const int y = full ? iy : (cy - r + iy + nc) % nc;
        const int z = full ? iz : (cz - r + iz + nc) % nc;
        const int xa = ixr ? xa1 : xa0, xb = ixr ? xb1 : xb0;
        const uint32_t rowbase = (uint32_t)(nc * (y + nc * z));
        slo = C.cellb[rowbase + xa];
        scnt = C.cellb[rowbase + xb + 1] - slo;
    }
    const uint32_t soff = wave_excl_scan(scnt, total);
    if (lane < nseg) {
        seglo[lane] = (uint16_t)slo;
        segoff[lane] = (uint16_t)soff;
    }
    wave_lds_sync();
    return nseg;
}

// idx-th molecule of the stencil (segment table in LDS).
template <typename Real, bool kRes>
__device__ __forceinline__ uint32_t stencil_molecule(const Ctx<Real, kRes>& C, const uint16_t* seglo,
                                                     const uint16_t* segoff, int nseg, uint32_t idx)
{
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((uint32_t)segoff[mid] <= idx) lo = mid; else hi = mid;
    }
    return C.list[(uint32_t)seglo[lo] + (idx - (uint32_t)segoff[lo])];
}

constexpr uint32_t kListCap = kCellListCap;
constexpr uint32_t kNoMolecule = 0xFFFFFFFFu;

// Where a cell's trials read positions: centres as [3][stride] and site
// offsets as [3 * stride], indexed by a local molecule id (the molecule index
// itself, or the slot of a staged copy of the cell's neighbourhood).
template <typename Real>
struct View {
    double* com;
    R4<Real>* site;
    uint32_t stride;
};

// The moved sites of the trial in flight, in registers (wave-uniform).
template <typename Real>
struct Moved {
    R4<Real> o[3], n[3];
    Real dlx, dly, dlz;
    double cx, cy, cz;
    int nmv;
    bool flip;
};

// Pair terms of one candidate item (a site of a survivor, with the survivor's
// centre and the site's offset already loaded) with the moved sites before and
// after a move of kind kMove (0 translation, 1 rotation, 2 flip): Eq. (1)
// within each pair's cut-off.  Returns u_new - u_old (0 for an invalid item);
// sc gets u_new + u_old; terms counts the pairs inside the cut-off over the
// wave (popcounts of the compare masks).
template <int kMove, bool kLog, typename Real>
__device__ __forceinline__ Real item_terms(const Moved<Real>& mv, double L, double invL,
                                           double jx, double jy, double jz, const R4<Real>& sj,
                                           bool valid, Real rc2f, Real& sc, uint32_t& terms)
{
    const double dx = fma(-L, rint((jx - mv.cx) * invL), jx - mv.cx);
    const double dy = fma(-L, rint((jy - mv.cy) * invL), jy - mv.cy);
    const double dz = fma(-L, rint((jz - mv.cz) * invL), jz - mv.cz);
    Real px = (Real)dx + sj.x, py = (Real)dy + sj.y, pz = (Real)dz + sj.z;
    if (!valid) px = Real(1e4);
    Real d = Real(0);
    sc = Real(0);
    constexpr int kNmv = kMove == 2 ? 2 : 3;
#pragma unroll
    for (int v = 0; v < kNmv; ++v) {
        const R4<Real> o = mv.o[v];
        const Real rx = px - o.x, ry = py - o.y, rz = pz - o.z;
        const Real r2 = fma(rx, rx, fma(ry, ry, rz * rz));
        const Real sg = Real(0.5) * (o.w + sj.w);
        const Real s2 = sg * sg, rc2 = rc2f * s2;
        const bool io = r2 < rc2;
        const Real uo = io ? pair_u(s2, r2) : Real(0);
        Real r2n, s2n, rc2n;
        if (kMove == 0) {  // same offsets about the displaced centre
            const Real qx = rx - mv.dlx, qy = ry - mv.dly, qz = rz - mv.dlz;
            r2n = fma(qx, qx, fma(qy, qy, qz * qz));
            s2n = s2; rc2n = rc2;
        } else if (kMove == 1) {  // rotated offsets about the same centre
            const R4<Real> n = mv.n[v];
            const Real qx = px - n.x, qy = py - n.y, qz = pz - n.z;
            r2n = fma(qx, qx, fma(qy, qy, qz * qz));
            s2n = s2; rc2n = rc2;
        } else {  // same position, swapped type
            const Real sgn = Real(0.5) * (mv.n[v].w + sj.w);
            r2n = r2;
            s2n = sgn * sgn; rc2n = rc2f * s2n;
        }
        const bool in = r2n < rc2n;
        const Real un = in ? pair_u(s2n, r2n) : Real(0);
        d += un - uo;
        if (kLog) sc += un + uo;
        terms += (uint32_t)__popcll(__ballot(io)) + (uint32_t)__popcll(__ballot(in));
    }
    return d;
}

template <typename Real>
struct PassSum {
    Real d, s;       // sum of u_new - u_old, of u_new + u_old
    uint32_t terms;  // pairs inside the cut-off (wave total)
};

// One step of the item loop: items base + lane and base + 64 + lane (item
// 3 s + t = site t of survivor s), with the loads of both passes issued
// before any arithmetic.
template <int kMove, bool kLog, typename Real>
__device__ __forceinline__ PassSum<Real> item_pair_pass(const View<Real>& V, double L, double invL,
                                                        const uint16_t* surv, const Moved<Real>& mv,
                                                        uint32_t base, uint32_t nit, Real rc2f)
{
    const uint32_t S = V.stride;
    const bool two = nit - base > 64u;  // wave-uniform: the second pass has items
    const uint32_t itA = base + (uint32_t)__lane_id(), itB = itA + 64u;
    const bool vA = itA < nit, vB = itB < nit;
    const uint32_t cA = vA ? itA : 0u, cB = vB ? itB : 0u;
    const uint32_t sA = cA / 3u, sB = cB / 3u;
    const uint32_t tA = cA - 3u * sA, tB = cB - 3u * sB;
    const uint32_t jA = surv[sA];
    uint32_t jB = 0;
    if (two) jB = surv[sB];
    const double xA = V.com[jA], yA = V.com[S + jA], zA = V.com[2 * S + jA];
    const R4<Real> gA = V.site[3u * jA + tA];
    double xB = 0.0, yB = 0.0, zB = 0.0;
    R4<Real> gB{};
    if (two) {
        xB = V.com[jB]; yB = V.com[S + jB]; zB = V.com[2 * S + jB];
        gB = V.site[3u * jB + tB];
    }
    __builtin_amdgcn_sched_barrier(0);
    Real sa = Real(0), sb = Real(0);
    uint32_t terms = 0;
    Real d = item_terms<kMove, kLog>(mv, L, invL, xA, yA, zA, gA, vA, rc2f, sa, terms);
    if (two) d += item_terms<kMove, kLog>(mv, L, invL, xB, yB, zB, gB, vB, rc2f, sb, terms);
    return PassSum<Real>{d, sa + sb, terms};
}

// Per-phase constants of the trial loop.
struct PhaseConst {
    double half_w, reach_box, step;
    float prune2;        // largest prune radius squared (3e38 when pruning is off)
    float pr_base, pr_step;  // radius = pr_base + pr_step * (own translation + same cell)
    float box_in;        // |relative centre| per axis below which an entry is in the cell
    bool prune_on;
    bool logging;
};

template <typename Real, bool kRes>
__device__ __forceinline__ PhaseConst phase_const(const Ctx<Real, kRes>& C, uint64_t sweep)
{
    PhaseConst P;
    P.logging = C.log != nullptr && sweep - C.log_sweep0 < C.log_sweeps;
    P.half_w = 0.5 * C.w;
    const double reach = sqrt(C.reach2);
    P.reach_box = (reach + 1e-6) * (reach + 1e-6);
    // prune radius on the FP16 relative centres: own move + a neighbour of the
    // same cell that moved earlier in this cell + rounding
    P.step = C.dmax * 1.7320508075688772;
    const float prune_r = (float)(reach + 2.0 * P.step + 0.02);
    // the relative centres are unique images only while the list region stays
    // below half the box; otherwise every listed molecule survives the prune
    // (and FP16 keeps the rounding below the 0.02 margin only up to |r| < 16)
    const bool prune_ok = P.half_w + (double)prune_r + P.step < fmin(0.5 * C.L - 1e-3, 16.0);
    P.prune2 = prune_ok ? prune_r * prune_r : 3.0e38f;
    P.prune_on = prune_ok;
    // the margins a trial needs: its own move when it translates the
    // molecule, and the moves made earlier in this cell by molecules of the
    // cell (no other molecule within reach moves during the colour phase)
    P.pr_base = (float)(reach + 0.02);
    P.pr_step = (float)P.step;
    P.box_in = (float)(P.half_w + 0.05);
    return P;
}

// The near list as the lanes hold it: entries lane, lane + 64, lane + 128
// (local ids and FP16-rounded relative centres).
struct NearRegs {
    uint32_t j[3];
    float x[3], y[3], z[3];
};

__device__ __forceinline__ NearRegs near_regs(const NearEntry* near, uint32_t nnear, bool overflow)
{
    NearRegs r;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const uint32_t idx = (uint32_t)__lane_id() + 64u * c;
        r.j[c] = kNoMolecule;
        r.x[c] = r.y[c] = r.z[c] = 0.f;
        if (!overflow && idx < nnear) {
            const NearEntry e = near[idx];
            r.j[c] = e.j;
            r.x[c] = (float)e.rx; r.y[c] = (float)e.ry; r.z[c] = (float)e.rz;
        }
    }
    return r;
}

// Where the multi-workgroup engine stages a cell's neighbourhood (per-wave
// LDS): centres, sites, the molecule of each slot and the slot of each of the
// cell's own molecules.
template <typename Real>
struct StageLds {
    double* com;     // [3][kCellListCap] centres
    R4<Real>* site;  // [3 * kCellListCap] site offsets + sigma
    uint16_t* gid;   // molecule of each slot
    uint16_t* own;   // slot of the cell's q-th molecule
};

// Molecules whose centre is within reach of the box of a cell centred at
// (bx0, by0, bz0), from the stencil segments of the cell list, into the near
// list (index and FP16 relative centre; returns the count, sets overflow past
// the list capacity).  The lanes are split over the segments in proportion to
// their molecules and take kPer molecules each per step, loads issued before
// arithmetic; the list order (step, then molecule rank within the step, then
// lane) is the same in all engines.  With kStage the molecules are also copied to S (centres, sites) and
// the list holds their slots; the cell's own molecules (list positions
// cbeg .. cbeg + ccnt) get their slots in S.own.
template <typename Real, bool kRes, bool kStage>
__device__ uint32_t gather_near(const Ctx<Real, kRes>& C, const PhaseConst& P, int nseg,
                                uint32_t total, double bx0, double by0, double bz0, uint32_t cbeg,
                                uint32_t ccnt, const WaveLds<Real>& W, const StageLds<Real>& S,
                                bool& overflow)
{
    constexpr int kPer = 4;
    const int lane = __lane_id();
    const uint32_t M = C.M;
    // lanes per segment (nseg <= 50): one each, and the other 64 - nseg in
    // proportion to the segment's molecules.  Segment s starts at lane
    // s + (64 - nseg) * segoff[s] / total; lane l serves the segment whose
    // start is the last one at or below l (the starts are distinct).
    uint64_t starts = 0;
    if (lane < nseg)
        starts = 1ull << ((uint32_t)lane +
                          (uint32_t)(64 - nseg) * (uint32_t)W.segoff[lane] / max(total, 1u));
#pragma unroll
    for (int o = 32; o; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)starts, o), hi = __shfl_xor((uint32_t)(starts >> 32), o);
        starts |= ((uint64_t)hi << 32) | lo;
    }
    const uint64_t upto = starts & ((2ull << lane) - 1ull);  // starts at or below this lane
    const int my_seg = __popcll(upto) - 1;
    const int first = 63 - __clzll(upto);
    const uint64_t above = starts & ~((2ull << lane) - 1ull);
    const uint32_t nl = (uint32_t)((above ? __ffsll((long long)above) - 1 : 64) - first);
    const uint32_t my_sub = (uint32_t)(lane - first);
    const uint32_t my_lo = W.seglo[my_seg];
    const uint32_t end = my_seg + 1 < nseg ? (uint32_t)W.segoff[my_seg + 1] : total;
    const uint32_t my_len = end - (uint32_t)W.segoff[my_seg];
    const uint32_t step = (uint32_t)kPer * nl;  // this lane's segment per step
    uint32_t nstep = (my_len + step - 1) / step;
#pragma unroll
    for (int o = 32; o; o >>= 1) nstep = max(nstep, (uint32_t)__shfl_xor(nstep, o));
    uint32_t nnear = 0;
    overflow = false;
    for (uint32_t k = 0; k < nstep; ++k) {
        uint32_t li[kPer], jj[kPer];
        bool vv[kPer];
        double xx[kPer], yy[kPer], zz[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const uint32_t t = k * step + (uint32_t)u * nl + my_sub;
            vv[u] = t < my_len;
            li[u] = vv[u] ? my_lo + t : 0u;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) jj[u] = C.list[li[u]];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            xx[u] = C.com[jj[u]];
            yy[u] = C.com[M + jj[u]];
            zz[u] = C.com[2 * M + jj[u]];
        }
        __builtin_amdgcn_sched_barrier(0);
        float fx[kPer], fy[kPer], fz[kPer];
        uint64_t bm[kPer];
        uint32_t base[kPer + 1];
        base[0] = nnear;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const double rx = min_image(xx[u] - bx0, C.L, C.invL);
            const double ry = min_image(yy[u] - by0, C.L, C.invL);
            const double rz = min_image(zz[u] - bz0, C.L, C.invL);
            const double ex = fmax(fabs(rx) - P.half_w, 0.0), ey = fmax(fabs(ry) - P.half_w, 0.0),
                         ez = fmax(fabs(rz) - P.half_w, 0.0);
            vv[u] = vv[u] && ex * ex + ey * ey + ez * ez < P.reach_box;
            bm[u] = __ballot(vv[u]);
            base[u + 1] = base[u] + (uint32_t)__popcll(bm[u]);
            fx[u] = (float)rx; fy[u] = (float)ry; fz[u] = (float)rz;
        }
        if (base[kPer] > kListCap) {
            overflow = true;
            break;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            if (vv[u]) {
                const uint32_t slot = base[u] + rank_below(bm[u]);
                NearEntry e;
                e.j = (uint16_t)(kStage ? slot : jj[u]);
                e.rx = (__fp16)fx[u]; e.ry = (__fp16)fy[u]; e.rz = (__fp16)fz[u];
                W.near[slot] = e;
                if (kStage) {
                    S.com[slot] = xx[u];
                    S.com[kListCap + slot] = yy[u];
                    S.com[2 * kListCap + slot] = zz[u];
                    S.gid[slot] = (uint16_t)jj[u];
                    const uint32_t q = li[u] - cbeg;
                    if (q < ccnt && q < kListCap) S.own[q] = (uint16_t)slot;
                }
            }
        }
        nnear = base[kPer];
    }
    wave_lds_sync();
    if (kStage && !overflow) {
        // the staged molecules' sites, a slot per lane at a time with its
        // three loads in flight (nine at once did not fit the registers and
        // went through scratch memory one load at a time)
        // (copied as 16-byte words: copying R4 values made the compiler keep
        // one of them in a scratch slot, a dead store per slot whose line the
        // release of every barrier then wrote back to memory)
        using W4 = uint32_t __attribute__((ext_vector_type(4)));
        constexpr int kW = 3 * (int)(sizeof(R4<Real>) / sizeof(W4));
#pragma unroll 1
        for (uint32_t sl = (uint32_t)lane; sl < nnear; sl += 64u) {
            const uint32_t g = S.gid[sl];
            const W4* src = reinterpret_cast<const W4*>(C.site + 3 * g);
            W4* dst = reinterpret_cast<W4*>(S.site + 3 * sl);
            W4 v[kW];
#pragma unroll
            for (int i = 0; i < kW; ++i) v[i] = src[i];
#pragma unroll
            for (int i = 0; i < kW; ++i) dst[i] = v[i];
        }
        wave_lds_sync();
    }
    return nnear;
}

// The trials of one cell (molecules list[cbeg .. cbeg + ccnt), a cell box
// centred at (bx0, by0, bz0)), in ascending order, by one wave.
//
// The lanes load the proposals, centres and rotated offsets of the cell's
// molecules (one lane each).  Per trial:
//   1. the lane holding the proposal publishes the moved sites;
//   2. the near list is pruned against the molecule's centre (FP32 on the
//      FP16 relative centres, with margins for the trial's own move and for
//      earlier moves of the same cell) and the survivors are compacted;
//   3. every site of every survivor takes a lane: the separation of the
//      centres is formed in FP64 with the nearest image and the site is
//      evaluated against the moved sites before and after the move (two
//      64-lane passes issued together);
//   4. a DPP reduction in FP64 gives dE in a fixed order, Metropolis decides
//      and the owning lane commits the move.
// Positions are read through V (local ids: molecule indices, or slots of a
// staged neighbourhood when kStaged, where own_slot maps the cell's molecules
// to their slots and commits also go to the state in C).  After a near-list
// overflow every stencil molecule is a candidate and V is the state in C.
template <typename Real, bool kRes, bool kStaged>
__device__ void cell_trials(const Ctx<Real, kRes>& C, const View<Real>& Vn, const PropRec* props,
                            uint64_t sweep, const PhaseConst& P, uint32_t cbeg, uint32_t ccnt,
                            double bx0, double by0, double bz0, const NearRegs& nr, bool overflow,
                            int nseg, uint32_t total, const uint16_t* own_slot,
                            const WaveLds<Real>& W, WaveCount& wc)
{
    const int lane = __lane_id();
    const uint32_t M = C.M;
    const Real rc2f = (Real)C.rc2_factor;
    const bool staged = kStaged && !overflow;
    const View<Real> V = (kStaged && overflow) ? View<Real>{C.com, C.site, M} : Vn;
    const uint32_t S = V.stride;
    TrialLds<Real>* tr = W.tr;

    for (uint32_t q0 = 0; q0 < ccnt; q0 += 64u) {
        const uint32_t n = min(64u, ccnt - q0);
        // one lane per molecule: proposal, centre, relative centre, sites and,
        // for a rotation, the rotated offsets
        PropRec pr;
        uint32_t mi = 0, ml = 0;  // molecule index, local id in V
        double cmx = 0.0, cmy = 0.0, cmz = 0.0;
        float mrx = 0.f, mry = 0.f, mrz = 0.f;
        Real no[9];
        R4<Real> os0{}, os1{}, os2{};  // the molecule's sites before its trial
        if ((uint32_t)lane < n) {
            mi = C.list[cbeg + q0 + lane];
            ml = staged ? (uint32_t)own_slot[q0 + lane] : mi;
            pr = props[mi];
            cmx = V.com[ml]; cmy = V.com[S + ml]; cmz = V.com[2 * S + ml];
            os0 = V.site[3 * ml]; os1 = V.site[3 * ml + 1]; os2 = V.site[3 * ml + 2];
            mrx = (float)min_image(cmx - bx0, C.L, C.invL);
            mry = (float)min_image(cmy - by0, C.L, C.invL);
            mrz = (float)min_image(cmz - bz0, C.L, C.invL);
            if ((pr.kind & 15u) == 1u) {
                double rm[9];
                rotation(pr.a0, pr.a1, pr.a2, pr.a3, rm);
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    const double b0 = body_at(C, s, 0), b1 = body_at(C, s, 1), b2 = body_at(C, s, 2);
                    no[3 * s] = (Real)(rm[0] * b0 + rm[1] * b1 + rm[2] * b2);
                    no[3 * s + 1] = (Real)(rm[3] * b0 + rm[4] * b1 + rm[5] * b2);
                    no[3 * s + 2] = (Real)(rm[6] * b0 + rm[7] * b1 + rm[8] * b2);
                }
            }
        }

        for (uint32_t q = 0; q < n; ++q) {
            const int i = (int)q;
            const uint32_t kind = rl_u(pr.kind, i);
            const uint32_t move = kind & 15u, exited = (kind >> 4) & 1u, axis = kind >> 8;
            const uint32_t m = rl_u(mi, i), mloc = rl_u(ml, i);
            wc.att0 += move == 0u;
            wc.att1 += move == 1u;
            wc.att2 += move == 2u;
            if (exited) {
                wc.exits += 1;
                if (P.logging && lane == i) {
                    MoveRecord rec;
                    rec.delta_e = 0.0; rec.scale = 0.0; rec.t_log_u = pr.thr; rec.sweep = sweep;
                    rec.molecule = m; rec.move = (uint8_t)move; rec.accepted = 0;
                    rec.exited = 1; rec.axis = (uint8_t)axis; rec.pair_terms = 0; rec.pad = 0;
                    C.log[(sweep - C.log_sweep0) * M + m] = rec;
                }
                continue;
            }
            // 1. publish the moved sites: all three, or the two swapped ones
            // of a flip
            const bool flip = move == 2u;
            const uint32_t a1 = (axis + 1) % 3, a2 = (axis + 2) % 3;
            if (lane == i) {
                if (flip) {
                    const R4<Real> x1 = a1 == 0u ? os0 : (a1 == 1u ? os1 : os2);
                    const R4<Real> x2 = a2 == 0u ? os0 : (a2 == 1u ? os1 : os2);
                    tr->old_site[0] = x1;
                    tr->old_site[1] = x2;
                    tr->new_site[0] = R4<Real>{x1.x, x1.y, x1.z, x2.w};
                    tr->new_site[1] = R4<Real>{x2.x, x2.y, x2.z, x1.w};
                } else {
                    tr->old_site[0] = os0;
                    tr->old_site[1] = os1;
                    tr->old_site[2] = os2;
                    if (move == 1u) {
                        tr->new_site[0] = R4<Real>{no[0], no[1], no[2], os0.w};
                        tr->new_site[1] = R4<Real>{no[3], no[4], no[5], os1.w};
                        tr->new_site[2] = R4<Real>{no[6], no[7], no[8], os2.w};
                    } else {
                        tr->new_site[0] = os0;
                        tr->new_site[1] = os1;
                        tr->new_site[2] = os2;
                    }
                }
                tr->cm[0] = cmx; tr->cm[1] = cmy; tr->cm[2] = cmz;
                tr->mr[0] = mrx; tr->mr[1] = mry; tr->mr[2] = mrz;
                tr->dl[0] = move == 0u ? (Real)pr.a0 : Real(0);
                tr->dl[1] = move == 0u ? (Real)pr.a1 : Real(0);
                tr->dl[2] = move == 0u ? (Real)pr.a2 : Real(0);
            }
            // the moved sites, read by every lane once the record is written
            Moved<Real> mv;
            auto load_moved = [&]() __attribute__((always_inline)) {
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    mv.o[s] = tr->old_site[s];
                    mv.n[s] = tr->new_site[s];
                }
                mv.cx = tr->cm[0]; mv.cy = tr->cm[1]; mv.cz = tr->cm[2];
                mv.dlx = tr->dl[0]; mv.dly = tr->dl[1]; mv.dlz = tr->dl[2];
                mv.flip = flip;
                mv.nmv = flip ? 2 : 3;
                __builtin_amdgcn_sched_barrier(0);
            };

            Real acc = Real(0), accs = Real(0);
            uint32_t terms = 0, tests = 0;
            // 3. one lane per (survivor, site), two passes at a time
            auto eval_items = [&](uint32_t nit) __attribute__((always_inline)) {
                wave_lds_sync();
                tests += nit * (uint32_t)mv.nmv * 2u;
                for (uint32_t base = 0; base < nit; base += 128u) {
                    PassSum<Real> ps;
                    if (P.logging) {
                        if (move == 0u)
                            ps = item_pair_pass<0, true>(V, C.L, C.invL, W.surv, mv, base, nit, rc2f);
                        else if (move == 1u)
                            ps = item_pair_pass<1, true>(V, C.L, C.invL, W.surv, mv, base, nit, rc2f);
                        else
                            ps = item_pair_pass<2, true>(V, C.L, C.invL, W.surv, mv, base, nit, rc2f);
                    } else {
                        if (move == 0u)
                            ps = item_pair_pass<0, false>(V, C.L, C.invL, W.surv, mv, base, nit, rc2f);
                        else if (move == 1u)
                            ps = item_pair_pass<1, false>(V, C.L, C.invL, W.surv, mv, base, nit, rc2f);
                        else
                            ps = item_pair_pass<2, false>(V, C.L, C.invL, W.surv, mv, base, nit, rc2f);
                    }
                    acc += ps.d;
                    accs += ps.s;
                    terms += ps.terms;
                }
            };

            // 2. prune and compact the survivors (the prune needs only the
            // molecule's relative centre, taken from the lane that holds it
            // while that lane's record is still being written)
            if (!overflow) {
                const float tmx = rl_f(mrx, i), tmy = rl_f(mry, i), tmz = rl_f(mrz, i);
                uint32_t nsurv = 0;
                const float r_far = P.pr_base + (move == 0u ? P.pr_step : 0.f);
                const float r_near = r_far + P.pr_step;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float px = nr.x[c] - tmx, py = nr.y[c] - tmy, pz = nr.z[c] - tmz;
                    const bool in_cell = fabsf(nr.x[c]) <= P.box_in && fabsf(nr.y[c]) <= P.box_in &&
                                         fabsf(nr.z[c]) <= P.box_in;
                    const float rr = in_cell ? r_near : r_far;
                    const float lim = P.prune_on ? rr * rr : P.prune2;
                    const bool keep = nr.j[c] != kNoMolecule && nr.j[c] != mloc &&
                                      px * px + py * py + pz * pz < lim;
                    const uint64_t bm = __ballot(keep);
                    if (keep) W.surv[nsurv + rank_below(bm)] = (uint16_t)nr.j[c];
                    nsurv += (uint32_t)__popcll(bm);
                }
                wave_lds_sync();  // the record and the survivors
                load_moved();
                if (nsurv) eval_items(3u * nsurv);
            } else {
                wave_lds_sync();
                load_moved();
                // list overflow: every stencil molecule, 64 at a time
                for (uint32_t base = 0; base < total; base += 64u) {
                    const uint32_t idx = base + (uint32_t)lane;
                    uint32_t j = kNoMolecule;
                    if (idx < total) j = stencil_molecule(C, W.seglo, W.segoff, nseg, idx);
                    const bool keep = j != kNoMolecule && j != m;
                    const uint64_t bm = __ballot(keep);
                    wave_lds_sync();
                    if (keep) W.surv[rank_below(bm)] = (uint16_t)j;
                    const uint32_t ns = (uint32_t)__popcll(bm);
                    if (ns) eval_items(3u * ns);
                }
            }

            // 4. Metropolis on the FP64 sum
            const double de = wave_sum_dpp((double)acc);
            const double thr = rl_d(pr.thr, i);
            const bool accept = (de <= 0.0) || (thr < -de);
            double sc = 0.0;
            if (P.logging) sc = wave_sum_dpp((double)accs);
            wc.terms += terms;
            wc.tests += tests;
            if (accept) {
                wc.acc0 += move == 0u;
                wc.acc1 += move == 1u;
                wc.acc2 += move == 2u;
                wc.e += de;
            }
            if (lane == i) {
                if (accept) {
                    R4<Real>* sp = V.site + 3 * ml;
                    R4<Real>* gp = C.site + 3 * mi;
                    if (move == 0u) {
                        const double tx = cmx + pr.a0, ty = cmy + pr.a1, tz = cmz + pr.a2;
                        const double nx = wrap(tx, C.L), ny = wrap(ty, C.L), nz = wrap(tz, C.L);
                        // periodic images crossed (the shifts wrap takes off)
                        const int ix = (int)floor(tx / C.L), iy = (int)floor(ty / C.L),
                                  iz = (int)floor(tz / C.L);
                        if (ix) atomicAdd(&C.img[mi], ix);
                        if (iy) atomicAdd(&C.img[M + mi], iy);
                        if (iz) atomicAdd(&C.img[2 * M + mi], iz);
                        V.com[ml] = nx; V.com[S + ml] = ny; V.com[2 * S + ml] = nz;
                        if (staged) {
                            C.com[mi] = nx; C.com[M + mi] = ny; C.com[2 * M + mi] = nz;
                        }
                    } else if (move == 1u) {
#pragma unroll
                        for (int s = 0; s < 3; ++s) {
                            sp[s].x = no[3 * s];
                            sp[s].y = no[3 * s + 1];
                            sp[s].z = no[3 * s + 2];
                            if (staged) {
                                gp[s].x = no[3 * s];
                                gp[s].y = no[3 * s + 1];
                                gp[s].z = no[3 * s + 2];
                            }
                        }
                        C.quat[mi] = pr.a0;
                        C.quat[M + mi] = pr.a1;
                        C.quat[2 * M + mi] = pr.a2;
                        C.quat[3 * M + mi] = pr.a3;
                    } else {
                        const Real w1 = a1 == 0u ? os0.w : (a1 == 1u ? os1.w : os2.w);
                        const Real w2 = a2 == 0u ? os0.w : (a2 == 1u ? os1.w : os2.w);
                        sp[a1].w = w2;
                        sp[a2].w = w1;
                        if (staged) {
                            gp[a1].w = w2;
                            gp[a2].w = w1;
                        }
                        const uint32_t ty = C.types[mi];
                        const uint32_t t1 = (ty >> (8 * a1)) & 0xFFu, t2 = (ty >> (8 * a2)) & 0xFFu;
                        uint32_t nt = ty & ~((0xFFu << (8 * a1)) | (0xFFu << (8 * a2)));
                        nt |= (t2 << (8 * a1)) | (t1 << (8 * a2));
                        C.types[mi] = nt;
                    }
                }
                if (P.logging) {
                    MoveRecord rec;
                    rec.delta_e = de; rec.scale = sc; rec.t_log_u = thr; rec.sweep = sweep;
                    rec.molecule = m; rec.move = (uint8_t)move; rec.accepted = accept ? 1 : 0;
                    rec.exited = 0; rec.axis = (uint8_t)axis; rec.pair_terms = terms; rec.pad = 0;
                    C.log[(sweep - C.log_sweep0) * M + m] = rec;
                }
            }
            wave_lds_sync();
        }
    }
}

// All trials of the cells of colour `col` owned by this wave of the
// single-workgroup engine: per cell, the near list from the system's own
// arrays, then the cell's trials.
template <typename Real, bool kRes>
__device__ void run_phase(const Ctx<Real, kRes>& C, const PropRec* props, int col, uint64_t sweep,
                          double hx, double hy, double hz, const WaveLds<Real>& W, WaveCount& wc)
{
    const int wave = threadIdx.x >> 6;
    const int lane = __lane_id();
    const int k = (int)C.k, nc = (int)C.nc, na = nc / k;
    const int nact = na * na * na;
    const int kx = col % k, ky = (col / k) % k, kz = col / (k * k);
    const PhaseConst P = phase_const(C, sweep);
    const View<Real> V{C.com, C.site, C.M};
    // With at most one cell per wave, the colour's cells go to the waves in
    // order of decreasing molecule count: the lower waves of each SIMD, whose
    // instructions issue first, take the larger cells, so the two waves of a
    // SIMD tend to finish together.  Otherwise wave w takes cells
    // w + kWaves ci.  Cells of a colour do not interact, so any assignment
    // gives the same results.
    const bool ranked = nact <= kWaves;
    uint32_t rank = 0;
    if (ranked) {
        uint32_t cnt = 0;
        if (lane < nact) {
            const int cx = kx + k * (lane % na), cy = ky + k * ((lane / na) % na),
                      cz = kz + k * (lane / (na * na));
            const uint32_t cell = (uint32_t)(cx + nc * (cy + nc * cz));
            cnt = C.cellb[cell + 1] - C.cellb[cell];
        }
        for (int j = 0; j < nact; ++j) {
            const uint32_t cj = rl_u(cnt, j);
            rank += (cj > cnt || (cj == cnt && j < lane)) ? 1u : 0u;
        }
    }
    const int ncw = (nact + kWaves - 1) / kWaves;

    for (int ci = 0; ci < ncw; ++ci) {
        int a = wave + kWaves * ci;
        if (ranked) {
            const uint64_t bm = __ballot(lane < nact && rank == (uint32_t)wave);
            a = bm ? __ffsll((long long)bm) - 1 : nact;
        }
        if (a >= nact) continue;
        const int cx = kx + k * (a % na), cy = ky + k * ((a / na) % na), cz = kz + k * (a / (na * na));
        const uint32_t cell = (uint32_t)(cx + nc * (cy + nc * cz));
        const uint32_t cbeg = C.cellb[cell], ccnt = C.cellb[cell + 1] - cbeg;
        if (ccnt == 0) {
            if (__lane_id() == 0) C.ecell[cell] = 0.0;
            continue;
        }
        const double bx0 = hx + ((double)cx + 0.5) * C.w;
        const double by0 = hy + ((double)cy + 0.5) * C.w;
        const double bz0 = hz + ((double)cz + 0.5) * C.w;
        uint32_t total;
        const int nseg = stencil_segments(C, cx, cy, cz, W.seglo, W.segoff, &total);
        bool overflow;
        const uint32_t nnear = gather_near<Real, kRes, false>(C, P, nseg, total, bx0, by0, bz0, 0u, 0u,
                                                             W, StageLds<Real>{}, overflow);
        const NearRegs nr = near_regs(W.near, nnear, overflow);
        wc.overflows += overflow ? 1u : 0u;
        wc.e = 0.0;
        cell_trials<Real, kRes, false>(C, V, props, sweep, P, cbeg, ccnt, bx0, by0, bz0, nr,
                                       overflow, nseg, total, nullptr, W, wc);
        if (__lane_id() == 0) C.ecell[cell] = wc.e;
    }
}

// Fill the per-system constants of a workgroup (before any store).
template <typename Real, bool kRes>
__device__ __forceinline__ void load_ctx(Ctx<Real, kRes>& C, const SysDev* __restrict__ Dp)
{
    C.M = Dp->M; C.k = Dp->k; C.nc = Dp->nc; C.ncell = Dp->ncell;
    C.seed_lo = Dp->seed_lo; C.seed_hi = Dp->seed_hi;
    C.resum_interval = Dp->resum_interval; C.obs_interval = Dp->obs_interval;
    C.gofr_interval = Dp->gofr_interval; C.obs_start = Dp->obs_start;
    C.max_samples = Dp->max_samples; C.gofr_nbins = Dp->gofr_nbins;
    C.L = Dp->L; C.invL = 1.0 / Dp->L; C.w = Dp->w; C.T = Dp->T;
    C.p_flip = Dp->p_flip; C.p_ft = Dp->p_ft; C.dmax = Dp->dmax; C.rot_max = Dp->rot_max;
    C.reach2 = Dp->reach2; C.radius = Dp->radius; C.rc2_factor = Dp->rc2_factor;
    C.bR = Dp->body[0]; C.bH = Dp->body[4];
    C.sig0 = Dp->sigma[0]; C.sig1 = Dp->sigma[1]; C.sig2 = Dp->sigma[2];
    C.gofr_dr = Dp->gofr_dr; C.gofr_rmax = Dp->gofr_rmax;
    C.gcom = Dp->com; C.quat = Dp->quat; C.types = Dp->types; C.u0 = Dp->u0; C.kref = Dp->kref;
    C.img = Dp->img; C.r0 = Dp->r0; C.o0 = Dp->o0; C.fs = Dp->fs; C.fs_cm = Dp->fs_cm; C.mom = Dp->mom;
    C.fs_q = Dp->fs_q; C.fs_q_cm = Dp->fs_q_cm;
    C.stats = Dp->stats; C.e_samples = Dp->e_samples; C.drift_samples = Dp->drift_samples;
    C.gofr_all = Dp->gofr_all; C.gofr_inter = Dp->gofr_inter; C.c2 = Dp->c2;
    C.c2_sweep = Dp->c2_sweep;
    C.log = (MoveRecord*)Dp->log; C.log_sweep0 = Dp->log_sweep0; C.log_sweeps = Dp->log_sweeps;
    C.gpart = Dp->g_part;
}

// The scheduled re-sum and C_2 sample of a sweep inside the batch's sweep
// kernel (not inlined: its registers stay out of the sweep loop's).  The
// context is rebuilt from the descriptor and the LDS layout the kernel uses.
template <typename Real, bool kRes>
__device__ __attribute__((noinline)) void inline_events(const SysDev* __restrict__ Dp, unsigned char* smem,
                                                       uint64_t sweep, uint64_t origin, bool resum, bool c2)
{
    Ctx<Real, kRes> E;
    load_ctx(E, Dp);
    const int tid = threadIdx.x;
    const bool fp64 = sizeof(Real) == 8;
    const LdsLayout L = lds_layout(fp64, kRes, E.M, E.ncell);
    E.bins = nullptr;
    E.misc = (double*)(smem + L.misc);
    E.red = E.misc + 8;
    if (kRes) {
        E.com = (double*)(smem + L.com);
        E.site = (R4<Real>*)(smem + L.site);
        E.cellb = (uint32_t*)(smem + L.cell);
        E.cellid = (uint16_t*)(smem + L.cellid);
        E.list = (uint16_t*)(smem + L.list);
        E.ecell = (double*)(smem + L.ecell);
    } else {
        E.com = E.gcom;
        E.site = (R4<Real>*)Dp->g_site;
        E.cellb = Dp->g_cell;
        E.cellid = Dp->g_cellid;
        E.list = Dp->g_list;
        E.ecell = Dp->g_ecell;
    }
    E.off = nullptr;
    Stats* st = E.stats;
    __syncthreads();
    if (resum) {
        const double e = resum_energy(E, tid, kThreads);
        if (tid == 0) {
            // re-anchor the accumulated energy: each drift sample is the
            // error of one window
            const double drift = E.misc[0] - e;
            E.misc[0] = e;
            st->e_resum = e;
            st->drift = drift;
            st->resum_sweep = sweep;
            st->n_resum += 1;
            if (st->n_drift < E.max_samples) E.drift_samples[st->n_drift] = drift;
            st->n_drift += 1;
            if (sweep > E.resum_interval && fabs(drift) > st->max_abs_drift) st->max_abs_drift = fabs(drift);
        }
        __syncthreads();
    }
    if (c2) {
        store_dyn(E, st, sweep - origin);
        __syncthreads();
    }
}

// The hot kernel: n checkerboard sweeps of every slot's system, one
// workgroup per system, with the state resident in LDS when it fits.  The
// variant with kInl also takes the scheduled re-sums and C_2 samples of slots
// flagged kFlagInline (a batch's systems); the plain one leaves them to the
// event kernel.
template <typename Real, bool kRes, bool kInl>
__global__ void __launch_bounds__(kThreads) k_sweeps(const Slot* __restrict__ slots, Slot one)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Slot sl = slots ? slots[blockIdx.x] : one;
    if (sl.sys == nullptr || sl.n_sweeps == 0) return;
    const SysDev* __restrict__ Dp = sl.sys;
    Ctx<Real, kRes> C;
    load_ctx(C, Dp);
    void* g_site = Dp->g_site;
    uint32_t* g_cell = Dp->g_cell;
    uint16_t* g_cellid = Dp->g_cellid;
    uint16_t* g_list = Dp->g_list;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool fp64 = sizeof(Real) == 8;
    const LdsLayout L = lds_layout(fp64, kRes, C.M, C.ncell);
    C.red = nullptr;
    C.bins = nullptr;
    C.misc = (double*)(smem + L.misc);
    if (kRes) {
        C.com = (double*)(smem + L.com);
        C.site = (R4<Real>*)(smem + L.site);
        C.cellb = (uint32_t*)(smem + L.cell);
        C.cellid = (uint16_t*)(smem + L.cellid);
        C.list = (uint16_t*)(smem + L.list);
        C.ecell = (double*)(smem + L.ecell);
        C.off = nullptr;
    } else {
        C.com = C.gcom;
        C.site = (R4<Real>*)g_site;
        C.cellb = g_cell;
        C.cellid = g_cellid;
        C.list = g_list;
        C.ecell = Dp->g_ecell;
        C.off = nullptr;
    }
    WaveLds<Real> W;
    W.surv = (uint16_t*)(smem + L.surv) + wave * kCellListCap;
    W.seglo = (uint16_t*)(smem + L.seglo) + wave * kMaxSeg;
    W.segoff = (uint16_t*)(smem + L.segoff) + wave * kMaxSeg;
    W.near = (NearEntry*)(smem + L.near) + wave * kListCap;
    W.tr = (TrialLds<Real>*)(smem + L.trial + (size_t)wave * trial_bytes(fp64));
    PropRec* props = (PropRec*)Dp->props;
    uint32_t* uscratch = (uint32_t*)(C.misc + 8);
    const uint32_t M = C.M;

    Stats* st = C.stats;
    if (tid == 0) {
        C.misc[0] = st->e_acc;
        C.misc[1] = C.sig0;
        C.misc[2] = C.sig1;
        C.misc[3] = C.sig2;
    }
    __syncthreads();
    if (kRes)
        for (uint32_t i = tid; i < 3 * M; i += kThreads) C.com[i] = C.gcom[i];
    for (uint32_t m = tid; m < M; m += kThreads) store_sites_from_quat(C, m);
    WaveCount wc{};
    uint64_t sweep = st->sweep;
    const uint64_t origin = st->obs_origin;
    __syncthreads();

    const int ncol = (int)(C.k * C.k * C.k);
    for (uint64_t it = 0; it < sl.n_sweeps; ++it) {
        const U4 g = philox10(0xFFFFFFFFu, (uint32_t)sweep, (uint32_t)(sweep >> 32), 3u, C.seed_lo,
                              C.seed_hi);
        const double hx = C.w * unit_open(g.x), hy = C.w * unit_open(g.y),
                     hz = C.w * unit_open(g.z);
        build_cells(C, hx, hy, hz, uscratch);
        propose_all(C, props, sweep, hx, hy, hz);
        __syncthreads();
        for (int col = 0; col < ncol; ++col) {
            run_phase(C, props, col, sweep, hx, hy, hz, W, wc);
            __syncthreads();
        }
        // E_acc += the sweep's dE (sweep_energy); E/M samples
        ++sweep;
        if (wave == 0) {
            const double e = C.misc[0] + sweep_energy(C.ecell, C.ncell);
            if (lane == 0) C.misc[0] = e;
        }
        if (tid == 0) {
            const double e = C.misc[0];
            const uint64_t t = sweep - origin;
            if (t >= C.obs_start && C.obs_interval && t % C.obs_interval == 0) {
                const double em = e / (double)M;
                if (st->n_e < C.max_samples) C.e_samples[st->n_e] = em;
                st->n_e += 1;
                st->e_sum += em;
                st->e_sumsq += em * em;
            }
        }
        if (kInl && (sl.flags & kFlagInline)) {
            // this sweep's scheduled re-sum and C_2 sample, taken here with the
            // event kernel's routines and thread mapping (the same sums), so
            // that a slice need not end at them
            const bool resum = C.resum_interval && sweep % C.resum_interval == 0;
            const bool c2 = is_c2_time(sweep - origin);
            if (resum || c2) inline_events<Real, kRes>(Dp, smem, sweep, origin, resum, c2);
        }
    }

    // write back
    if (kRes)
        for (uint32_t i = tid; i < 3 * M; i += kThreads) C.gcom[i] = C.com[i];
    if (lane == 0) {
        const uint64_t att[3] = {wc.att0, wc.att1, wc.att2}, acc[3] = {wc.acc0, wc.acc1, wc.acc2};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (att[i]) atomicAdd((unsigned long long*)&st->attempts[i], (unsigned long long)att[i]);
            if (acc[i]) atomicAdd((unsigned long long*)&st->accepts[i], (unsigned long long)acc[i]);
        }
        if (wc.exits) atomicAdd((unsigned long long*)&st->exits, (unsigned long long)wc.exits);
        if (wc.terms) atomicAdd((unsigned long long*)&st->pair_terms, (unsigned long long)wc.terms);
        if (wc.tests) atomicAdd((unsigned long long*)&st->pair_tests, (unsigned long long)wc.tests);
        if (wc.overflows)
            atomicAdd((unsigned long long*)&st->near_overflows, (unsigned long long)wc.overflows);
    }
    __syncthreads();
    if (tid == 0) {
        st->sweep = sweep;
        st->e_acc = C.misc[0];
    }
}

// Cold work at event sweeps, straight from the HBM state in FP64: re-sum of
// the energy (and drift), a g(r) frame, a C_2 sample, observable reset.
__global__ void __launch_bounds__(kThreads) k_events(const Slot* __restrict__ slots, Slot one)
{
    __shared__ double red[kWaves];
    __shared__ double misc[16];
    __shared__ uint32_t bins[2 * kGofrBins];
    __shared__ uint32_t gqueue[kWaves * kGofrQueue];
    extern __shared__ __align__(16) unsigned char ev_stage[];
    const Slot sl = slots ? slots[blockIdx.x] : one;
    if (sl.sys == nullptr || sl.flags == 0) return;
    Ctx<double, false> C;
    load_ctx(C, sl.sys);
    C.com = C.gcom;
    C.red = red;
    C.misc = misc;
    C.bins = bins;
    C.ecell = nullptr;
    C.off = nullptr;
    C.site = nullptr;
    C.cellb = nullptr;
    C.cellid = nullptr;
    C.list = nullptr;
    const int tid = threadIdx.x;
    Stats* st = C.stats;
    if (tid == 0) {
        misc[1] = C.sig0;
        misc[2] = C.sig1;
        misc[3] = C.sig2;
    }
    const uint64_t sweep = st->sweep;
    const double e_acc = st->e_acc;
    const uint32_t f = sl.flags;
    const uint32_t M = C.M;
    if ((f & (kFlagResumSet | kFlagResumReport | kFlagResumPeriodic | kFlagGofr)) &&
        !(f & kFlagParts) && M <= kEventStage) {
        // the O(M^2) loops read centres, orientations and types from an LDS
        // copy (same values, same order: the same sums)
        // (with the site offsets computed once per molecule when they fit)
        double* scom = (double*)ev_stage;
        double* squat = scom + 3 * M;
        const bool pre = size_t(M) * (12 * sizeof(double) + sizeof(uint32_t)) <= kEventStageBytes;
        uint32_t* stypes = (uint32_t*)(squat + (pre ? 9 : 4) * M);
        for (uint32_t i = tid; i < 3 * M; i += kThreads) scom[i] = C.gcom[i];
        for (uint32_t i = tid; i < M; i += kThreads) stypes[i] = C.types[i];
        if (pre) {
            __syncthreads();  // sigma table (misc) before offsets_f64
            for (uint32_t m = tid; m < M; m += kThreads) {
                double o[9], sg[3];
                offsets_f64(C, m, o, sg);
#pragma unroll
                for (int i = 0; i < 9; ++i) squat[i * M + m] = o[i];
            }
            C.off = squat;
        } else {
            for (uint32_t i = tid; i < 4 * M; i += kThreads) squat[i] = C.quat[i];
            C.quat = squat;
        }
        C.com = scom;
        C.types = stypes;
    }
    __syncthreads();
    if (f & kFlagObsReset) {
        reset_observables(C);
        __syncthreads();
    }
    if (f & (kFlagResumSet | kFlagResumReport | kFlagResumPeriodic)) {
        double e;
        if (f & kFlagParts) {  // partial energies of the multi-workgroup kernel, in order
            e = 0.0;
            for (uint32_t b = 0; b < sl.pad; ++b) e += C.gpart[b];
        } else {
            e = resum_energy(C, threadIdx.x, kThreads);
        }
        if (tid == 0) {
            const double acc = (f & kFlagResumSet) ? e : e_acc;
            // a set or a scheduled re-sum re-anchors the accumulated energy, so
            // each drift sample is the error of one window
            if (f & (kFlagResumSet | kFlagResumPeriodic)) st->e_acc = e;
            const double drift = acc - e;
            st->e_resum = e;
            st->drift = drift;
            st->resum_sweep = sweep;
            if (f & kFlagResumPeriodic) {
                st->n_resum += 1;
                if (st->n_drift < C.max_samples) C.drift_samples[st->n_drift] = drift;
                st->n_drift += 1;
                if (sweep > C.resum_interval && fabs(drift) > st->max_abs_drift)
                    st->max_abs_drift = fabs(drift);
            }
        }
        __syncthreads();
    }
    if (f & kFlagGofr) {
        if (f & kFlagParts) {
            if (tid == 0) st->n_gofr += 1;
        } else {
            gofr_frame(C, threadIdx.x, kThreads, false, gqueue);
        }
        __syncthreads();
    }
    if (f & kFlagC2) store_dyn(C, st, sweep - st->obs_origin);
}

// ----------------------------------------------------- multi-workgroup --
//
// The spread engine advances one large system with many workgroups in one
// cooperative launch.  The state stays in HBM.  A sweep is: cell indices,
// counts and proposals of all molecules (one thread each); an exclusive scan
// of the counts (workgroup 0); the scatter of molecule indices into the cell
// list and a sort of every cell's range; then the k^3 colours, each wave
// taking cells of the colour in turn.  For every cell the wave copies the
// neighbourhood (molecules within reach of the cell's box) into its LDS and
// runs the cell's trials on the copy, writing each accepted move through to
// HBM.  Barriers among the system's workgroups separate the steps; the colours
// keep the waves apart exactly as in the single-workgroup engine, so the
// decisions are the same.

// Barrier of the workgroups of one system inside a cooperative launch (which
// keeps every workgroup resident): a counter in the system's buffer, zero at
// launch, that each workgroup raises once per barrier; a workgroup passes the
// n-th barrier when the counter reaches n x (workgroups of the system).  The
// wait is bounded (SysDev::barrier_polls polls, seconds by default): past the
// bound the system is marked faulted (Stats::fault) and sys_sync returns
// false, and the workgroup must leave the kernel at once.  A workgroup thus
// only goes on past a barrier when every workgroup has finished the work
// before it, and the others, which then miss its increments, time out too.
struct SysBarrier {
    uint32_t* count;
    uint32_t nblk;
    uint32_t epoch;
    uint32_t polls;
};

__device__ bool sys_sync(SysBarrier& B, uint32_t* fault, uint32_t* flag)
{
    __syncthreads();
    ++B.epoch;
    if (threadIdx.x == 0) {
        uint32_t bad = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(B.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the counter may wrap in a long launch: compare the signed distance
        // (the workgroups are never 2^31 increments apart)
        const uint32_t target = B.epoch * B.nblk;
        uint32_t spins = 0;
        while ((int32_t)(__hip_atomic_load(B.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                         target) < 0) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins >= B.polls) {
                bad = 1;
                __hip_atomic_store(fault, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *flag = bad;
    }
    __syncthreads();
    return *flag == 0u;
}

// One launch can advance several systems: slot i owns workgroups
// [first_block, first_block + n_blocks) and runs n_sweeps sweeps; the
// workgroups of a system synchronise among themselves (sys_sync), so systems
// of one launch run at their own pace.
template <typename Real>
__global__ void __launch_bounds__(kSpreadThreads) k_spread(const SpreadSlot* __restrict__ slots,
                                                           uint32_t n_slots, SpreadSlot one)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr bool fp64 = sizeof(Real) == 8;
    constexpr uint32_t kCap = kListCap;
    SpreadSlot sl = one;
    if (slots) {
        for (uint32_t i = 0; i < n_slots; ++i) {
            const SpreadSlot t = slots[i];
            if (blockIdx.x >= t.first_block && blockIdx.x < t.first_block + t.n_blocks) {
                sl = t;
                break;
            }
        }
    }
    if (sl.sys == nullptr || sl.n_blocks == 0) return;  // a workgroup of no system
    SysDev* __restrict__ Dp = sl.sys;
    const uint32_t bid = blockIdx.x - sl.first_block, nblk = sl.n_blocks;
    Ctx<Real, false> C;
    load_ctx(C, Dp);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned char* wb = smem + (size_t)wave * spread_wave_bytes(fp64);
    StageLds<Real> S;
    WaveLds<Real> W;
    size_t o = 0;
    S.com = (double*)(wb + o);    o = align16(o + 3 * size_t(kCap) * sizeof(double));
    S.site = (R4<Real>*)(wb + o); o = align16(o + 3 * size_t(kCap) * site_bytes(fp64));
    S.gid = (uint16_t*)(wb + o);  o = align16(o + size_t(kCap) * sizeof(uint16_t));
    S.own = (uint16_t*)(wb + o);  o = align16(o + size_t(kCap) * sizeof(uint16_t));
    W.near = (NearEntry*)(wb + o); o = align16(o + size_t(kCap) * 8);
    W.surv = (uint16_t*)(wb + o); o = align16(o + size_t(kCap) * sizeof(uint16_t));
    W.seglo = (uint16_t*)(wb + o);
    W.segoff = W.seglo + kMaxSeg; o = align16(o + 2 * size_t(kMaxSeg) * sizeof(uint16_t));
    W.tr = (TrialLds<Real>*)(wb + o);
    C.misc = (double*)(smem + kSpreadWaves * spread_wave_bytes(fp64));
    C.com = C.gcom;
    C.site = (R4<Real>*)Dp->g_site;
    C.cellb = Dp->g_cell;
    C.cellid = Dp->g_cellid;
    C.list = Dp->g_list;
    C.red = nullptr;
    C.bins = nullptr;
    C.ecell = Dp->g_ecell;
    C.off = nullptr;
    uint32_t* cnt = Dp->g_cnt;
    uint32_t* fill = cnt + C.ncell;
    PropRec* props = (PropRec*)Dp->props;
    Stats* st = C.stats;
    const uint32_t M = C.M, ncell = C.ncell;
    const uint32_t gtid = bid * kSpreadThreads + tid, GT = nblk * kSpreadThreads;
    const uint32_t gw = bid * kSpreadWaves + wave, NW = nblk * kSpreadWaves;
    const int k = (int)C.k, nc = (int)C.nc, na = nc / k;
    const uint32_t nact = (uint32_t)(na * na * na);
    const int ncol = k * k * k;

    if (tid == 0) {
        C.misc[1] = C.sig0;
        C.misc[2] = C.sig1;
        C.misc[3] = C.sig2;
    }
    __syncthreads();
    for (uint32_t m = gtid; m < M; m += GT) store_sites_from_quat(C, m);
    for (uint32_t c = gtid; c < 2 * ncell; c += GT) cnt[c] = 0;
    WaveCount wc{};
    double e_acc = st->e_acc;
    uint64_t sweep = st->sweep;
    const uint64_t origin = st->obs_origin;
    SysBarrier B{Dp->g_bar, nblk, 0u, Dp->barrier_polls};
    uint32_t* bflag = (uint32_t*)(C.misc + 15);
    // at every barrier a workgroup that timed out leaves (see sys_sync)
    if (!sys_sync(B, &st->fault, bflag)) return;

    for (uint64_t it = 0; it < sl.n_sweeps; ++it) {
        constexpr bool run = true;
        const U4 g = philox10(0xFFFFFFFFu, (uint32_t)sweep, (uint32_t)(sweep >> 32), 3u, C.seed_lo,
                              C.seed_hi);
        const double hx = C.w * unit_open(g.x), hy = C.w * unit_open(g.y),
                     hz = C.w * unit_open(g.z);
        // cell of every molecule, counts, proposals
        if (run) {
            for (uint32_t m = gtid; m < M; m += GT) {
                const int ix = cell_axis(C.com[m], hx, C.L, C.w, nc);
                const int iy = cell_axis(C.com[M + m], hy, C.L, C.w, nc);
                const int iz = cell_axis(C.com[2 * M + m], hz, C.L, C.w, nc);
                const uint32_t cid = (uint32_t)(ix + nc * (iy + nc * iz));
                C.cellid[m] = (uint16_t)cid;
                atomicAdd(&cnt[cid], 1u);
                props[m] = propose(C, m, sweep, hx, hy, hz, ix, iy, iz);
            }
        }
        if (!sys_sync(B, &st->fault, bflag)) return;
        // cell starts (exclusive scan of the counts); counts cleared for the
        // next sweep
        if (run && bid == 0) {
            for (uint32_t c = tid; c < ncell; c += kSpreadThreads) C.cellb[c] = cnt[c];
            __syncthreads();
            block_excl_scan_t<kSpreadThreads>(C.cellb, ncell, (uint32_t*)(C.misc + 8));
            if (tid == 0) C.cellb[ncell] = M;
            for (uint32_t c = tid; c < ncell; c += kSpreadThreads) cnt[c] = 0;
        }
        if (!sys_sync(B, &st->fault, bflag)) return;
        if (run) {
            for (uint32_t m = gtid; m < M; m += GT) {
                const uint32_t c = C.cellid[m];
                C.list[C.cellb[c] + atomicAdd(&fill[c], 1u)] = (uint16_t)m;
            }
        }
        if (!sys_sync(B, &st->fault, bflag)) return;
        // ascending molecule index inside every cell
        if (run) {
            sort_cells(C.list, C.cellb, gw, NW, ncell);
            for (uint32_t c = gtid; c < ncell; c += GT) fill[c] = 0;
        }
        if (!sys_sync(B, &st->fault, bflag)) return;

        const PhaseConst P = phase_const(C, sweep);
        const View<Real> V{S.com, S.site, kCap};
        for (int col = 0; col < ncol; ++col) {
            if (run) {
                const int kx = col % k, ky = (col / k) % k, kz = col / (k * k);
                for (uint32_t a = gw; a < nact; a += NW) {
                    const int cx = kx + k * (int)(a % na), cy = ky + k * (int)((a / na) % na),
                              cz = kz + k * (int)(a / (na * na));
                    const uint32_t cell = (uint32_t)(cx + nc * (cy + nc * cz));
                    const uint32_t cbeg = C.cellb[cell], ccnt = C.cellb[cell + 1] - cbeg;
                    if (ccnt == 0) {
                        if (lane == 0) C.ecell[cell] = 0.0;
                        continue;
                    }
                    const double bx0 = hx + ((double)cx + 0.5) * C.w;
                    const double by0 = hy + ((double)cy + 0.5) * C.w;
                    const double bz0 = hz + ((double)cz + 0.5) * C.w;
                    uint32_t total;
                    const int nseg = stencil_segments(C, cx, cy, cz, W.seglo, W.segoff, &total);
                    bool overflow;
                    const uint32_t ns = gather_near<Real, false, true>(C, P, nseg, total, bx0, by0, bz0,
                                                                       cbeg, ccnt, W, S, overflow);
                    const NearRegs nr = near_regs(W.near, ns, overflow);
                    wc.overflows += overflow ? 1u : 0u;
                    wc.e = 0.0;
                    cell_trials<Real, false, true>(C, V, props, sweep, P, cbeg, ccnt, bx0, by0, bz0,
                                                   nr, overflow, nseg, total, S.own, W, wc);
                    if (lane == 0) C.ecell[cell] = wc.e;
                }
            }
            if (col == ncol - 1) ++sweep;
            if (!sys_sync(B, &st->fault, bflag)) return;
        }
        // E_acc += the sweep's dE (sweep_energy); E/M samples (the next
        // sweep's steps touch neither)
        if (run && bid == 0 && wave == 0) {
            const double de = sweep_energy(C.ecell, C.ncell);
            e_acc += de;
        }
        if (run && bid == 0 && tid == 0) {
            const uint64_t t = sweep - origin;
            if (t >= C.obs_start && C.obs_interval && t % C.obs_interval == 0) {
                const double em = e_acc / (double)M;
                if (st->n_e < C.max_samples) C.e_samples[st->n_e] = em;
                st->n_e += 1;
                st->e_sum += em;
                st->e_sumsq += em * em;
            }
        }
    }

    if (lane == 0) {
        const uint64_t att[3] = {wc.att0, wc.att1, wc.att2}, acc[3] = {wc.acc0, wc.acc1, wc.acc2};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (att[i]) atomicAdd((unsigned long long*)&st->attempts[i], (unsigned long long)att[i]);
            if (acc[i]) atomicAdd((unsigned long long*)&st->accepts[i], (unsigned long long)acc[i]);
        }
        if (wc.exits) atomicAdd((unsigned long long*)&st->exits, (unsigned long long)wc.exits);
        if (wc.terms) atomicAdd((unsigned long long*)&st->pair_terms, (unsigned long long)wc.terms);
        if (wc.tests) atomicAdd((unsigned long long*)&st->pair_tests, (unsigned long long)wc.tests);
        if (wc.overflows)
            atomicAdd((unsigned long long*)&st->near_overflows, (unsigned long long)wc.overflows);
    }
    if (bid == 0 && tid == 0) {
        st->sweep = sweep;
        st->e_acc = e_acc;
    }
}

// The O(M^2) work of an event on many workgroups: the re-sum's partial energy
// of each workgroup into g_part, the g(r) frame into the histograms.
__global__ void __launch_bounds__(kThreads) k_event_parts(PartList list)
{
    // this workgroup's system: the last slot whose first workgroup is at or
    // below it (the slots are in ascending first)
    uint32_t lo = 0, hi = list.n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (list.s[mid].first <= blockIdx.x) lo = mid; else hi = mid;
    }
    const PartSlot one = list.s[lo];
    const uint32_t bid = blockIdx.x - one.first;
    __shared__ double red[kWaves];
    __shared__ double misc[16];
    __shared__ uint32_t bins[2 * kGofrBins];
    __shared__ uint32_t gqueue[kWaves * kGofrQueue];
    Ctx<double, false> C;
    load_ctx(C, one.sys);
    C.com = C.gcom;
    C.red = red;
    C.misc = misc;
    C.bins = bins;
    C.ecell = nullptr;
    C.off = nullptr;
    C.site = nullptr;
    C.cellb = one.sys->g_cell;
    C.cellid = one.sys->g_cellid;
    C.list = one.sys->g_list;
    if (threadIdx.x == 0) {
        misc[1] = C.sig0;
        misc[2] = C.sig1;
        misc[3] = C.sig2;
    }
    __syncthreads();
    const uint32_t f = one.flags;
    const uint32_t m0 = bid * kThreads + threadIdx.x, step = one.count * kThreads;
    if (f & (kFlagResumSet | kFlagResumReport | kFlagResumPeriodic)) {
        // a scheduled re-sum follows sweeps, whose cell lists are still there
        const int span = (int)ceil((sqrt(C.reach2) + 2.0 * 1.7320508075688772 * C.dmax + 1e-9) / C.w);
        const bool cells = (f & (kFlagResumSet | kFlagResumReport)) == 0 && C.cellb != nullptr &&
                           2 * span + 1 <= (int)C.nc;
        const double e = cells ? resum_energy_cells(C, m0, step, span) : resum_energy(C, m0, step);
        if (threadIdx.x == 0) C.gpart[bid] = e;
        __syncthreads();
    }
    if (f & kFlagGofr) gofr_frame(C, m0, step, true, gqueue);
}

__global__ void k_init_lattice(SysDev* Dp, uint32_t n)
{
    const SysDev& D = *Dp;
    const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t M = D.M;
    if (m >= M) return;
    const double a = D.L / (double)n;
    const uint32_t i = m % n, j = (m / n) % n, l = m / (n * n);
    D.com[m] = ((double)i + 0.5) * a;
    D.com[M + m] = ((double)j + 0.5) * a;
    D.com[2 * M + m] = ((double)l + 0.5) * a;
    const U4 g = philox10(m, 0xFFFFFFFFu, 0xFFFFFFFFu, 2u, D.seed_lo, D.seed_hi);
    const double u1 = unit_open(g.x), u2 = unit_open(g.y), u3 = unit_open(g.z);
    const double r1 = sqrt(1.0 - u1), r2 = sqrt(u1);
    D.quat[m] = r2 * cos(kTwoPi * u3);
    D.quat[M + m] = r1 * sin(kTwoPi * u2);
    D.quat[2 * M + m] = r1 * cos(kTwoPi * u2);
    D.quat[3 * M + m] = r2 * sin(kTwoPi * u3);
    D.types[m] = 0u | (1u << 8) | (2u << 16);
}

template <typename Real, bool kRes, bool kInl>
hipError_t launch_one(const Slot* dev_slots, const Slot& one, uint32_t n_blocks, size_t lds,
                      hipStream_t stream)
{
    static size_t configured = 0;
    if (lds > configured) {
        hipError_t e = hipFuncSetAttribute((const void*)&k_sweeps<Real, kRes, kInl>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        configured = lds;
    }
    hipLaunchKernelGGL((k_sweeps<Real, kRes, kInl>), dim3(n_blocks), dim3(kThreads), lds, stream,
                       dev_slots, one);
    return hipGetLastError();
}

template <typename Real, bool kInl>
hipError_t launch_res(bool resident, const Slot* dev_slots, const Slot& one, uint32_t n_blocks,
                      size_t lds, hipStream_t stream)
{
    return resident ? launch_one<Real, true, kInl>(dev_slots, one, n_blocks, lds, stream)
                    : launch_one<Real, false, kInl>(dev_slots, one, n_blocks, lds, stream);
}

}  // namespace

hipError_t launch_sweeps(bool fp64, bool resident, const Slot* dev_slots, const Slot& one,
                         uint32_t n_blocks, size_t lds_bytes, hipStream_t stream, bool inline_events)
{
    if (fp64)
        return inline_events
                   ? launch_res<double, true>(resident, dev_slots, one, n_blocks, lds_bytes, stream)
                   : launch_res<double, false>(resident, dev_slots, one, n_blocks, lds_bytes, stream);
    return inline_events
               ? launch_res<float, true>(resident, dev_slots, one, n_blocks, lds_bytes, stream)
               : launch_res<float, false>(resident, dev_slots, one, n_blocks, lds_bytes, stream);
}

hipError_t launch_events(const Slot* dev_slots, const Slot& one, uint32_t n_blocks,
                         hipStream_t stream)
{
    static const hipError_t attr = hipFuncSetAttribute(
        (const void*)&k_events, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kEventStageBytes);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k_events, dim3(n_blocks), dim3(kThreads), kEventStageBytes, stream,
                       dev_slots, one);
    return hipGetLastError();
}

namespace {

template <typename Real>
hipError_t spread_configure()
{
    static bool done = false;
    if (done) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute((const void*)&k_spread<Real>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)spread_lds_bytes(sizeof(Real) == 8));
    if (e == hipSuccess) done = true;
    return e;
}

template <typename Real>
hipError_t spread_max_blocks_t(uint32_t* n_blocks)
{
    hipError_t e = spread_configure<Real>();
    if (e != hipSuccess) return e;
    int occ = 0, dev = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)&k_spread<Real>, kSpreadThreads,
                                                     spread_lds_bytes(sizeof(Real) == 8));
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    *n_blocks = (uint32_t)(occ * cus);
    return hipSuccess;
}

template <typename Real>
hipError_t launch_spread_t(const SpreadSlot* dev_slots, uint32_t n_slots, const SpreadSlot& one,
                           uint32_t n_blocks, hipStream_t stream)
{
    hipError_t e = spread_configure<Real>();
    if (e != hipSuccess) return e;
    SpreadSlot o = one;
    void* args[] = {(void*)&dev_slots, (void*)&n_slots, (void*)&o};
    return hipLaunchCooperativeKernel((const void*)&k_spread<Real>, dim3(n_blocks),
                                      dim3(kSpreadThreads), args,
                                      spread_lds_bytes(sizeof(Real) == 8), stream);
}

__global__ void k_zero_barriers(const SpreadSlot* __restrict__ slots, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *slots[i].sys->g_bar = 0u;
}

}  // namespace

hipError_t spread_max_blocks(bool fp64, uint32_t* n_blocks)
{
    return fp64 ? spread_max_blocks_t<double>(n_blocks) : spread_max_blocks_t<float>(n_blocks);
}

hipError_t launch_spread(bool fp64, const SpreadSlot* dev_slots, uint32_t n_slots,
                         const SpreadSlot& one, uint32_t n_blocks, hipStream_t stream)
{
    return fp64 ? launch_spread_t<double>(dev_slots, n_slots, one, n_blocks, stream)
                : launch_spread_t<float>(dev_slots, n_slots, one, n_blocks, stream);
}

hipError_t launch_zero_barriers(const SpreadSlot* dev_slots, uint32_t n_slots, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_barriers, dim3((n_slots + 63) / 64), dim3(64), 0, stream, dev_slots, n_slots);
    return hipGetLastError();
}

hipError_t launch_event_parts(const PartList& list, uint32_t n_blocks, hipStream_t stream)
{
    hipLaunchKernelGGL(k_event_parts, dim3(n_blocks), dim3(kThreads), 0, stream, list);
    return hipGetLastError();
}

hipError_t launch_init_lattice(SysDev* dev_sys, uint32_t M, hipStream_t stream)
{
    uint32_t n = 1;
    while ((n + 1) * (n + 1) * (n + 1) <= M) ++n;
    hipLaunchKernelGGL(k_init_lattice, dim3((M + 255) / 256), dim3(256), 0, stream, dev_sys, n);
    return hipGetLastError();
}

}  // namespace flipmc
