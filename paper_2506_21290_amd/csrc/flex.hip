// flex.hip -- flip Monte Carlo of FLEXIBLE molecules on gfx950 (the paper's
// own model, Sec. II.A, and the squares and tetrahedra of Sec. VII): the event
// kernels (FP64 re-sum, g(r) frames, C_2 / F_s / F_s^cm samples and their
// per-particle moments, the lattice start) and the host code behind the mcf_*
// calls of the C ABI.  The sweep kernel is in flex_sweep.h.

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"
#include "flipmc.h"
#include "flex_sweep.h"
#include "wave.h"

namespace flipmc {

// LDS bytes one workgroup may use on the current device (defined with the
// rigid engine's host code).
size_t device_lds_limit();

namespace {

// Event work, the O(N^2) part: each workgroup's partial energy (every pair of
// atoms once, Eq. 1, plus Eq. 2 over the bonds) into D.part and one g(r)
// frame (Eq. 3 numerator, every ordered pair) into the histograms.  Workgroup
// b works on part b % parts of system b / parts of the list (a system of N
// atoms has ceil(N / 512) parts; workgroups past them return).
__global__ void __launch_bounds__(kFxThreads) k_fx_event_parts(FxList list, uint32_t flags, uint32_t parts)
{
    __shared__ double red[kFxWaves];
    __shared__ uint32_t bins[2][kGofrBins];
    const FxDev& D = *list.d[blockIdx.x / parts];
    const uint32_t part = blockIdx.x % parts;
    const uint32_t N = D.N, n = D.n, half = N / 2;
    if (part * kFxThreads >= N) return;
    const uint32_t i = part * kFxThreads + threadIdx.x;
    if (flags & (kFlagResumSet | kFlagResumReport | kFlagResumPeriodic)) {
        double e = 0.0;
        if (i < N) {
            const double xi = D.pos[i], yi = D.pos[N + i], zi = D.pos[2 * N + i];
            const double si = D.sigma[D.type[i]];
            for (uint32_t dj = 1; dj <= half; ++dj) {
                if ((N & 1u) == 0u && dj == half && i >= half) break;
                uint32_t j = i + dj;
                if (j >= N) j -= N;
                const double dx = fx_mi(D.pos[j] - xi, D.L, D.invL), dy = fx_mi(D.pos[N + j] - yi, D.L, D.invL),
                             dz = fx_mi(D.pos[2 * N + j] - zi, D.L, D.invL);
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double s = 0.5 * (si + D.sigma[D.type[j]]);
                e += fx_wca(s * s, r2, D.rc2f);
                if (i / n == j / n) {
                    const uint32_t a = i % n, b = j % n;
                    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
                    if ((D.bonded >> (4 * lo + hi)) & 1u) e += fx_fene(s, r2);
                }
            }
        }
        // fixed-order sum over the workgroup
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        e = wave_sum_dpp(e);
        if (lane == 0) red[wave] = e;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kFxWaves; ++w) t += red[w];
            D.part[part] = t;
        }
    }
    if (flags & kFlagGofr) {
        for (uint32_t b = threadIdx.x; b < 2 * kGofrBins; b += kFxThreads) (&bins[0][0])[b] = 0;
        __syncthreads();
        if (i < N) {
            const double xi = D.pos[i], yi = D.pos[N + i], zi = D.pos[2 * N + i];
            for (uint32_t j = 0; j < N; ++j) {
                if (j == i) continue;
                const double dx = fx_mi(D.pos[j] - xi, D.L, D.invL), dy = fx_mi(D.pos[N + j] - yi, D.L, D.invL),
                             dz = fx_mi(D.pos[2 * N + j] - zi, D.L, D.invL);
                const int b = (int)floor(sqrt(dx * dx + dy * dy + dz * dz) / D.gofr_dr);
                if (b >= 0 && b < (int)D.gofr_nbins) {
                    atomicAdd(&bins[0][b], 1u);
                    if (i / n != j / n) atomicAdd(&bins[1][b], 1u);
                }
            }
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < D.gofr_nbins; b += kFxThreads) {
            if (bins[0][b]) atomicAdd((unsigned long long*)&D.gofr_all[b], (unsigned long long)bins[0][b]);
            if (bins[1][b]) atomicAdd((unsigned long long*)&D.gofr_inter[b], (unsigned long long)bins[1][b]);
        }
    }
}

// Centre of mass of molecule m (equal masses): atom 0 plus the mean of the
// nearest-image offsets of the molecule's atoms from it (wrapped positions).
__device__ void fx_centre(const FxDev& D, uint32_t m, double c[3])
{
    const uint32_t N = D.N, base = D.n * m;
    for (int d = 0; d < 3; ++d) {
        const double x0 = D.pos[d * N + base];
        double acc = 0.0;
        for (uint32_t s = 0; s < D.n; ++s) acc += fx_mi(D.pos[d * N + base + s] - x0, D.L, D.invL);
        c[d] = x0 + acc / (double)D.n;
    }
}

__device__ double fx_sinc(double x) { return x < 1e-4 ? 1.0 - x * x / 6.0 : sin(x) / x; }

// Event work on one workgroup: the re-sum from the partial energies (drift,
// re-anchoring), the frame count, the observable origin, a C_2 / F_s sample.
// Workgroup b takes the events of system b of the list.
__global__ void __launch_bounds__(kFxThreads) k_fx_events(FxList list, uint32_t flags)
{
    __shared__ double red[kFxWaves];
    const FxDev& D = *list.d[blockIdx.x];
    const uint32_t nparts = (D.N + kFxThreads - 1) / kFxThreads;
    Stats* st = D.stats;
    const uint32_t N = D.N, M = D.M, n = D.n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    auto block_sum = [&](double v) {
        v = wave_sum_dpp(v);
        __syncthreads();
        if (lane == 0) red[wave] = v;
        __syncthreads();
        double t = 0.0;
        for (int w = 0; w < kFxWaves; ++w) t += red[w];
        return t;
    };
    const uint64_t sweep = st->sweep;
    if (flags & kFlagObsReset) {
        for (uint32_t i = tid; i < N; i += kFxThreads)
            for (int d = 0; d < 3; ++d) D.r0[d * N + i] = D.pos[d * N + i] + D.L * (double)D.img[d * N + i];
        for (uint32_t m = tid; m < M; m += kFxThreads) {
            double c[3];
            fx_centre(D, m, c);
            const uint32_t base = n * m;
            uint32_t kb = 0;
            for (uint32_t s = 0; s < n; ++s)
                if (D.type[base + s] == 1u) kb = s;
            D.kref[m] = (uint8_t)kb;
            double u[3], nrm = 0.0;
            for (int d = 0; d < 3; ++d) {
                u[d] = fx_mi(D.pos[d * N + base + kb] - c[d], D.L, D.invL);
                nrm += u[d] * u[d];
                // unwrapped centre: unwrapped atom 0 plus the offsets
                D.rcm0[d * M + m] = c[d] - D.pos[d * N + base] + D.pos[d * N + base] +
                                    D.L * (double)D.img[d * N + base];
            }
            nrm = sqrt(nrm);
            for (int d = 0; d < 3; ++d) D.u0[d * M + m] = u[d] / nrm;
        }
        for (uint32_t b = tid; b < kGofrBins; b += kFxThreads) {
            D.gofr_all[b] = 0;
            D.gofr_inter[b] = 0;
        }
        if (tid == 0) {
            st->obs_origin = sweep;
            st->n_e = st->n_drift = st->n_gofr = st->n_c2 = 0;
            st->e_sum = st->e_sumsq = 0.0;
            st->max_abs_drift = 0.0;
        }
        __syncthreads();
    }
    if (flags & (kFlagResumSet | kFlagResumReport | kFlagResumPeriodic)) {
        if (tid == 0) {
            double e = 0.0;
            for (uint32_t b = 0; b < nparts; ++b) e += D.part[b];
            const double acc = (flags & kFlagResumSet) ? e : st->e_acc;
            if (flags & (kFlagResumSet | kFlagResumPeriodic)) st->e_acc = e;
            const double drift = acc - e;
            st->e_resum = e;
            st->drift = drift;
            st->resum_sweep = sweep;
            if (flags & kFlagResumPeriodic) {
                st->n_resum += 1;
                if (st->n_drift < D.max_samples) D.drift_samples[st->n_drift] = drift;
                st->n_drift += 1;
                if (sweep > D.resum_interval && fabs(drift) > st->max_abs_drift) st->max_abs_drift = fabs(drift);
            }
        }
        __syncthreads();
    }
    if ((flags & kFlagGofr) && tid == 0) st->n_gofr += 1;
    if (flags & kFlagC2) {
        // means of C_2^i, F_s^cm,i, F_s^i and of (C_2^i)^2, (F_s^cm,i)^2,
        // C_2^i F_s^cm,i, (F_s^i)^2 (Sec. V.A)
        double a2 = 0.0, afs = 0.0, acm = 0.0, a2sq = 0.0, acmsq = 0.0, a2cm = 0.0, afssq = 0.0;
        for (uint32_t m = tid; m < M; m += kFxThreads) {
            double c[3], u[3], nrm = 0.0, dot = 0.0, dc2 = 0.0;
            fx_centre(D, m, c);
            const uint32_t base = n * m, kb = D.kref[m];
            for (int d = 0; d < 3; ++d) {
                u[d] = fx_mi(D.pos[d * N + base + kb] - c[d], D.L, D.invL);
                nrm += u[d] * u[d];
                const double cu = c[d] + D.L * (double)D.img[d * N + base];
                const double dd = cu - D.rcm0[d * M + m];
                dc2 += dd * dd;
            }
            nrm = sqrt(nrm);
            for (int d = 0; d < 3; ++d) dot += (u[d] / nrm) * D.u0[d * M + m];
            const double c2i = 0.5 * (3.0 * dot * dot - 1.0);
            const double fcmi = fx_sinc(D.fs_q_cm * sqrt(dc2));
            a2 += c2i;
            acm += fcmi;
            a2sq += c2i * c2i;
            acmsq += fcmi * fcmi;
            a2cm += c2i * fcmi;
        }
        for (uint32_t i = tid; i < N; i += kFxThreads) {
            double d2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double dd = D.pos[d * N + i] + D.L * (double)D.img[d * N + i] - D.r0[d * N + i];
                d2 += dd * dd;
            }
            const double fsi = fx_sinc(D.fs_q * sqrt(d2));
            afs += fsi;
            afssq += fsi * fsi;
        }
        const double c2 = block_sum(a2) / (double)M;
        const double fcm = block_sum(acm) / (double)M;
        const double fs = block_sum(afs) / (double)N;
        const double c2sq = block_sum(a2sq) / (double)M;
        const double fcmsq = block_sum(acmsq) / (double)M;
        const double c2fcm = block_sum(a2cm) / (double)M;
        const double fssq = block_sum(afssq) / (double)N;
        if (tid == 0 && st->n_c2 < kC2Max) {
            const uint32_t j = st->n_c2;
            D.c2[j] = c2;
            D.fs_cm[j] = fcm;
            D.fs[j] = fs;
            D.mom[j] = c2sq;
            D.mom[kC2Max + j] = fcmsq;
            D.mom[2 * kC2Max + j] = c2fcm;
            D.mom[3 * kC2Max + j] = fssq;
            D.c2_sweep[j] = sweep - st->obs_origin;
            st->n_c2 = j + 1;
        }
    }
}

// Zero n 8-byte words (instead of a memset node, which some callers cannot record).
__global__ void k_fx_zero(uint64_t* __restrict__ p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Host positions staged as xyz per atom in `aos` -> the SoA state, wrapped.
__global__ void k_fx_from_aos(FxDev* __restrict__ Dp, const double* __restrict__ aos)
{
    const FxDev& D = *Dp;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= D.N) return;
    for (int d = 0; d < 3; ++d) D.pos[(size_t)d * D.N + i] = fx_wrap(aos[3 * (size_t)i + d], D.L);
}

__global__ void k_fx_init_lattice(FxDev* __restrict__ Dp, uint32_t nl, double side)
{
    const FxDev& D = *Dp;
    const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= D.M) return;
    const uint32_t N = D.N, n = D.n;
    const double a = D.L / (double)nl;
    const double c[3] = {((double)(m % nl) + 0.5) * a, ((double)((m / nl) % nl) + 0.5) * a,
                         ((double)(m / (nl * nl)) + 0.5) * a};
    const U4 g = philox10(m, 0xFFFFFFFFu, 0xFFFFFFFFu, 2u, D.seed_lo, D.seed_hi);
    const double u1 = unit_open(g.x), u2 = unit_open(g.y), u3 = unit_open(g.z);
    const double r1 = sqrt(1.0 - u1), r2 = sqrt(u1);
    const double qw = r2 * cos(kTwoPi * u3), qx = r1 * sin(kTwoPi * u2), qy = r1 * cos(kTwoPi * u2),
                 qz = r2 * sin(kTwoPi * u3);
    const double R[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
                         2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                         2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
    // the ideal body of side `side` around its centre, atom s in row s
    double b[12] = {0};
    if (D.geometry == MC_TRIANGLE) {
        const double r = side / sqrt(3.0);
        b[0] = r;
        b[3] = -0.5 * r; b[4] = 0.5 * side;
        b[6] = -0.5 * r; b[7] = -0.5 * side;
    } else if (D.geometry == MC_SQUARE) {
        const double hs = 0.5 * side;
        b[0] = hs;  b[1] = hs;
        b[3] = -hs; b[4] = hs;
        b[6] = -hs; b[7] = -hs;
        b[9] = hs;  b[10] = -hs;
    } else {
        const double t = side / (2.0 * sqrt(2.0));
        const double v[12] = {1, 1, 1, 1, -1, -1, -1, 1, -1, -1, -1, 1};
        for (int i = 0; i < 12; ++i) b[i] = t * v[i];
    }
    for (uint32_t s = 0; s < n; ++s) {
        const uint32_t at = n * m + s;
        for (int d = 0; d < 3; ++d) {
            const double v = c[d] + (R[3 * d] * b[3 * s] + R[3 * d + 1] * b[3 * s + 1] + R[3 * d + 2] * b[3 * s + 2]);
            D.pos[d * N + at] = fx_wrap(v, D.L);
            D.img[d * N + at] = 0;
        }
        D.type[at] = (uint8_t)s;
    }
}

}  // namespace
}  // namespace flipmc

// ------------------------------------------------------------------ host --

namespace {

using namespace flipmc;

int fx_fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return api_error(code, buf);
}

#define FXCHK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) return fx_fail(MC_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

constexpr int kBondsOf[3][6][2] = {
    {{0, 1}, {1, 2}, {0, 2}, {-1, -1}, {-1, -1}, {-1, -1}},
    {{0, 1}, {1, 2}, {2, 3}, {0, 3}, {-1, -1}, {-1, -1}},
    {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}},
};
constexpr int kGraphDiam[3] = {1, 2, 1};
// new type of atom s = old type of atom perm[s]: the 180 degree rotations of
// the ideal body (triangle: about the median through atom q; square: the
// diagonal through atom 0, the one through atom 1, the bisector of edge 01,
// the bisector of edge 12; tetrahedron: the axes through the midpoints of
// edges 01, 02, 03 and of the opposite edges)
constexpr uint8_t kPerm[3][4][4] = {
    {{0, 2, 1, 3}, {2, 1, 0, 3}, {1, 0, 2, 3}, {0, 1, 2, 3}},
    {{0, 3, 2, 1}, {2, 1, 0, 3}, {1, 0, 3, 2}, {3, 2, 1, 0}},
    {{1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}, {0, 1, 2, 3}},
};
constexpr uint32_t kNPerm[3] = {3, 4, 3};

// Side of the ideal body at the lattice start: the minimum of WCA + FENE of a
// sigma_ij = 1 bond, by Newton's method on the slope.
double fx_bond_star()
{
    auto slope = [](double x) {
        return -48.0 * std::pow(x, -13.0) + 24.0 * std::pow(x, -7.0) + 30.0 * x / (1.0 - x * x / 2.25);
    };
    auto curv = [](double x) {
        const double d = 1.0 - x * x / 2.25;
        return 624.0 * std::pow(x, -14.0) - 168.0 * std::pow(x, -8.0) + 30.0 / d +
               30.0 * x * (2.0 * x / 2.25) / (d * d);
    };
    double x = 0.96;
    for (int it = 0; it < 100; ++it) {
        const double nx = x - slope(x) / curv(x);
        if (nx == x) break;
        x = nx;
    }
    return x;
}

struct FxGeom {
    uint32_t n, N, k, nc, ncell;
    double L, w, D, rc, reach;
    double D_est;  // the ideal body's largest atom distance, 15 % stretched
};

// Is (k, nc) a valid decomposition?  A cell must be r_c + 2 sqrt(3) d wide so
// that the 27 cells around an atom's cell hold its partners however the two
// have moved since the sort at the start of the sweep.  The cells of a colour
// are attempted in ascending index (that order defines the chain); when they
// are at least the reach 2 D + r_c apart they cannot interact and run side by
// side, and when (k - 1) w is below the worst-case reach the sweep kernel
// decides so per sweep from the largest intramolecular distance it finds.
bool fx_valid(const FxGeom& g0, double dmax, uint32_t k, uint32_t nc, FxGeom* out)
{
    if (k < 2 || nc < 2 || nc % k != 0) return false;
    const double w = g0.L / (double)nc;
    if (w < g0.rc + 2.0 * std::sqrt(3.0) * dmax) return false;
    if ((double)nc * nc * nc > 16777216.0) return false;
    if (out) {
        *out = g0;
        out->k = k;
        out->nc = nc;
        out->ncell = nc * nc * nc;
        out->w = w;
    }
    return true;
}

int fx_geometry(const mcf_params* p, FxGeom* gout)
{
    if (!p) return fx_fail(MC_EINVAL, "null parameters");
    if (p->geometry > MC_TETRAHEDRON) return fx_fail(MC_EINVAL, "unknown geometry %u", p->geometry);
    const uint32_t n = p->geometry == MC_TRIANGLE ? 3u : 4u;
    if (p->n_molecules < 1 || (uint64_t)p->n_molecules * n > (1u << 24))
        return fx_fail(MC_EINVAL, "n_molecules must be in [1, 2^24 / %u]", n);
    if (!(p->density > 0) || !(p->temperature > 0))
        return fx_fail(MC_EINVAL, "density and temperature must be positive");
    if (!(p->p_flip >= 0) || p->p_flip > 1.0 || !(p->max_displacement >= 0))
        return fx_fail(MC_EINVAL, "p_flip or max_displacement out of range");
    for (uint32_t t = 0; t < n; ++t)
        if (!(p->sigma[t] > 0)) return fx_fail(MC_EINVAL, "sigma must be positive");
    if (!(p->gofr_dr > 0)) return fx_fail(MC_EINVAL, "gofr_dr must be positive");
    FxGeom g{};
    g.n = n;
    g.N = n * p->n_molecules;
    g.L = std::cbrt((double)g.N / p->density);
    double smax = 0.0, bmax = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        smax = std::max(smax, p->sigma[i]);
        for (uint32_t j = i + 1; j < n; ++j) bmax = std::max(bmax, 1.5 * 0.5 * (p->sigma[i] + p->sigma[j]));
    }
    g.rc = std::pow(2.0, 1.0 / 6.0) * smax;
    g.D = kGraphDiam[p->geometry] * bmax;
    g.reach = (2.0 * g.D + g.rc) * (1.0 + 1e-12);
    const double side = p->bond_length > 0 ? p->bond_length : fx_bond_star();
    g.D_est = 1.15 * side * (p->geometry == MC_SQUARE ? std::sqrt(2.0) : 1.0);
    const double need = 2.0 * (std::max(g.D, g.rc) + 2.0 * p->max_displacement);
    if (g.L < need)
        return fx_fail(MC_EGEOM, "box side %.4f below %.4f (minimum image)", g.L, need);
    uint32_t k = p->colours_per_axis, nc = p->cells_per_side;
    if (k == 0 && nc == 0) {
        // most cells per colour that can run side by side when the bodies
        // stay within 15 % of their ideal size, then the smallest cells (the
        // fewest candidates per attempt)
        const double reach_est = 2.0 * (g.D_est + 2.0 * std::sqrt(3.0) * p->max_displacement) + g.rc;
        double best = -1.0;
        for (uint32_t kk = 2; kk <= 8; ++kk)
            for (uint32_t cc = kk; cc <= 256; cc += kk) {
                if (!fx_valid(g, p->max_displacement, kk, cc, nullptr)) continue;
                if ((double)(kk - 1) * g.L / (double)cc < std::min(reach_est, g.reach)) continue;
                const double act = std::pow((double)(cc / kk), 3.0);
                if (act > best || (act == best && cc > nc)) {
                    best = act;
                    k = kk;
                    nc = cc;
                }
            }
        if (best < 0) return fx_fail(MC_EGEOM, "no checkerboard fits a box of side %.4f", g.L);
    } else if (k == 0 || nc == 0) {
        return fx_fail(MC_EINVAL, "give both colours_per_axis and cells_per_side, or neither");
    }
    if (!fx_valid(g, p->max_displacement, k, nc, gout))
        return fx_fail(MC_EGEOM, "k = %u, n_c = %u: cells of %.4f need w >= %.4f (and n_c a multiple of k >= 2)", k,
                       nc, g.L / nc, g.rc + 2.0 * std::sqrt(3.0) * p->max_displacement);
    return MC_OK;
}

}  // namespace

namespace {

size_t fx_al(size_t x) { return (x + 255) & ~size_t(255); }

struct FxLayout {
    size_t dev, stats, pos, type, img, esamp, dsamp, gall, ginter, c2, c2s, fs, fscm, mom, u0, kref, r0, rcm0;
    size_t cstart, clist, cid, ecell, part, total;
};

FxLayout fx_layout(const mcf_params* p, const FxGeom& g)
{
    FxLayout l{};
    const size_t N = g.N, M = p->n_molecules;
    size_t o = 0;
    l.dev = o;    o = fx_al(o + sizeof(FxDev));
    l.stats = o;  o = fx_al(o + sizeof(Stats));
    l.pos = o;    o = fx_al(o + 3 * N * sizeof(double));
    l.type = o;   o = fx_al(o + N);
    l.img = o;    o = fx_al(o + 3 * N * sizeof(int32_t));
    l.esamp = o;  o = fx_al(o + size_t(p->max_samples) * sizeof(double));
    l.dsamp = o;  o = fx_al(o + size_t(p->max_samples) * sizeof(double));
    l.gall = o;   o = fx_al(o + kGofrBins * sizeof(uint64_t));
    l.ginter = o; o = fx_al(o + kGofrBins * sizeof(uint64_t));
    l.c2 = o;     o = fx_al(o + kC2Max * sizeof(double));
    l.c2s = o;    o = fx_al(o + kC2Max * sizeof(uint64_t));
    l.fs = o;     o = fx_al(o + kC2Max * sizeof(double));
    l.fscm = o;   o = fx_al(o + kC2Max * sizeof(double));
    l.mom = o;    o = fx_al(o + 4 * kC2Max * sizeof(double));
    l.u0 = o;     o = fx_al(o + 3 * M * sizeof(double));
    l.kref = o;   o = fx_al(o + M);
    l.r0 = o;     o = fx_al(o + 3 * N * sizeof(double));
    l.rcm0 = o;   o = fx_al(o + 3 * M * sizeof(double));
    l.cstart = o; o = fx_al(o + (size_t(g.ncell) + 1) * sizeof(uint32_t));
    l.clist = o;  o = fx_al(o + N * sizeof(uint32_t));
    l.cid = o;    o = fx_al(o + N * sizeof(uint32_t));
    l.ecell = o;  o = fx_al(o + size_t(g.ncell) * sizeof(double));
    l.part = o;   o = fx_al(o + kFxParts * sizeof(double));
    l.total = o;
    return l;
}

bool fx_c2_time(uint64_t t)
{
    if (t == 0) return false;
    while (t % 10 == 0) t /= 10;
    return t == 1 || t == 2 || t == 5;
}

}  // namespace

struct mcf_system {
    mcf_params p;
    FxGeom g;
    FxLayout lay;
    FxDev host;
    FxDev* dev;
    hipStream_t stream;
    uint64_t sweep, origin;
    size_t lds;  // dynamic LDS of the resident sweep kernel; 0 = state in the buffer
    int pooled;  // index + 1 of the static handle slot (mcf_init_system_noalloc), 0 otherwise
};

namespace {

// Dynamic LDS of the resident sweep kernel for these parameters, 0 when the
// state stays in the buffer (MC_FLAG_HBM_STATE, or too large for one
// workgroup next to the kernel's static LDS).
size_t fx_resident_lds(const mcf_params* p, const FxGeom& g)
{
    if (p->flags & MC_FLAG_HBM_STATE) return 0;
    const size_t lds = fx_lds_layout(g.N, g.ncell).total;
    return lds + kFxStaticLds <= device_lds_limit() ? lds : 0;
}

uint32_t fx_parts(const mcf_system* s) { return (s->g.N + kFxThreads - 1) / kFxThreads; }

// The same events (flags) of systems s[0 .. n), n <= kFxMany, on `stream`:
// one launch of the O(N^2) parts of all of them, one of the rest.
int fx_events_of(mcf_system* const* s, uint32_t n, uint32_t flags, hipStream_t stream)
{
    FxList list{};
    uint32_t np = 1;
    for (uint32_t i = 0; i < n; ++i) {
        np = std::max(np, fx_parts(s[i]));
        list.d[i] = s[i]->dev;
    }
    if (np > kFxParts) return fx_fail(MC_EINVAL, "too many atoms for the event kernel");
    if (flags & (kFlagResumSet | kFlagResumReport | kFlagResumPeriodic | kFlagGofr)) {
        hipLaunchKernelGGL(k_fx_event_parts, dim3(n * np), dim3(kFxThreads), 0, stream, list, flags, np);
        FXCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_fx_events, dim3(n), dim3(kFxThreads), 0, stream, list, flags);
    FXCHK(hipGetLastError());
    return MC_OK;
}

int fx_events(mcf_system* s, uint32_t flags) { return fx_events_of(&s, 1, flags, s->stream); }

uint32_t fx_events_at(const mcf_system* s, uint64_t sweep)
{
    uint32_t f = 0;
    const mcf_params& p = s->p;
    if (p.resum_interval && sweep % p.resum_interval == 0) f |= kFlagResumPeriodic;
    const uint64_t t = sweep - s->origin;
    if (p.gofr_interval && t >= p.obs_start && t % p.gofr_interval == 0) f |= kFlagGofr;
    if (fx_c2_time(t)) f |= kFlagC2;
    return f;
}

uint64_t fx_next_event(const mcf_system* s)
{
    const mcf_params& p = s->p;
    const uint64_t now = s->sweep, t = now - s->origin;
    uint64_t best = now + (1u << 16);  // bounded launches
    if (p.resum_interval) best = std::min(best, (now / p.resum_interval + 1) * p.resum_interval);
    if (p.gofr_interval) {
        uint64_t nx = (t / p.gofr_interval + 1) * p.gofr_interval;
        if (nx < p.obs_start) nx = ((p.obs_start + p.gofr_interval - 1) / p.gofr_interval) * p.gofr_interval;
        best = std::min(best, s->origin + nx);
    }
    for (uint64_t dec = 1; dec <= (uint64_t)1e18; dec *= 10) {
        bool found = false;
        for (uint64_t m : {1ull, 2ull, 5ull})
            if (m * dec > t) {
                best = std::min(best, s->origin + m * dec);
                found = true;
                break;
            }
        if (found) break;
    }
    return best;
}

int fx_read_stats(mcf_system* s, Stats* st)
{
    FXCHK(hipMemcpyAsync(st, s->host.stats, sizeof(Stats), hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipStreamSynchronize(s->stream));
    return MC_OK;
}

int fx_upload_desc(mcf_system* s)
{
    FXCHK(hipMemcpyAsync(s->dev, &s->host, sizeof(FxDev), hipMemcpyHostToDevice, s->stream));
    FXCHK(hipStreamSynchronize(s->stream));
    return MC_OK;
}

int fx_upload_state(mcf_system* s, const double* pos, const uint8_t* types)
{
    const uint32_t N = s->g.N, n = s->g.n;
    std::vector<double> x(3 * (size_t)N);
    for (uint32_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            const double v = pos[3 * i + d];
            if (!std::isfinite(v)) return fx_fail(MC_EINVAL, "position of atom %u is not finite", i);
            x[(size_t)d * N + i] = v - s->g.L * std::floor(v / s->g.L);
        }
    for (uint32_t m = 0; m < s->p.n_molecules; ++m) {
        uint32_t seen = 0;
        for (uint32_t t = 0; t < n; ++t) {
            const uint32_t ty = types[n * m + t];
            if (ty >= n || (seen >> ty) & 1u)
                return fx_fail(MC_EINVAL, "types of molecule %u are not a permutation of 0..%u", m, n - 1);
            seen |= 1u << ty;
        }
    }
    FXCHK(hipMemcpyAsync(s->host.pos, x.data(), x.size() * sizeof(double), hipMemcpyHostToDevice, s->stream));
    FXCHK(hipMemcpyAsync(s->host.type, types, N, hipMemcpyHostToDevice, s->stream));
    FXCHK(hipMemsetAsync(s->host.img, 0, 3 * sizeof(int32_t) * N, s->stream));
    FXCHK(hipStreamSynchronize(s->stream));
    return MC_OK;
}

}  // namespace

extern "C" {

void mcf_params_default(mcf_params* p, uint32_t geometry)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->geometry = geometry;
    p->n_molecules = 1000;
    p->density = 1.2;
    p->temperature = 3.0;
    if (geometry == MC_TRIANGLE) {
        p->sigma[0] = 0.9; p->sigma[1] = 1.0; p->sigma[2] = 1.1;
    } else {
        for (int t = 0; t < 4; ++t) p->sigma[t] = 0.9 + 0.2 * t / 3.0;
    }
    p->bond_length = 0.0;
    p->p_flip = 0.2;
    p->max_displacement = 0.1;
    p->seed = 1;
    p->resum_interval = 100;
    p->obs_interval = 10;
    p->gofr_interval = 100;
    p->max_samples = 4096;
    p->gofr_dr = 0.02;
    p->fs_q = 7.4;
    p->fs_q_cm = 5.1;
}

int mcf_geometry(const mcf_params* p, double* box, uint32_t* k, uint32_t* nc)
{
    FxGeom g;
    const int rc = fx_geometry(p, &g);
    if (rc) return rc;
    if (box) *box = g.L;
    if (k) *k = g.k;
    if (nc) *nc = g.nc;
    return MC_OK;
}

int mcf_placement(const mcf_params* p, int* resident, size_t* lds_bytes)
{
    FxGeom g;
    const int rc = fx_geometry(p, &g);
    if (rc) return rc;
    const size_t lds = fx_resident_lds(p, g);
    if (resident) *resident = lds ? 1 : 0;
    if (lds_bytes) *lds_bytes = lds;
    return MC_OK;
}

int mcf_required_bytes(const mcf_params* p, size_t* bytes)
{
    FxGeom g;
    const int rc = fx_geometry(p, &g);
    if (rc) return rc;
    if (!bytes) return fx_fail(MC_EINVAL, "null output");
    *bytes = fx_layout(p, g).total;
    return MC_OK;
}

}  // extern "C"

namespace {

// Scratch of the allocation-free entry point: the work arrays (cell lists,
// per-cell energies, partial sums) of one flexible system at a time per
// device.  Host code takes its address per device with hipGetSymbolAddress.
constexpr size_t kFxScratchBytes = size_t(4) << 20;
__device__ __align__(256) unsigned char fx_scratch[kFxScratchBytes];

constexpr int kFxMaxDevices = 64;
constexpr int kFxPool = 16;  // handles of allocation-free systems alive at once
std::mutex g_fx_mu;
void* g_fx_scratch[kFxMaxDevices];
mcf_system g_fx_pool[kFxPool];
bool g_fx_used[kFxPool];

// The device address of this device's scratch (once per device).
int fx_scratch_ptr(void** out)
{
    int dev = 0;
    FXCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kFxMaxDevices) return fx_fail(MC_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_fx_mu);
    if (!g_fx_scratch[dev]) {
        void* p = nullptr;
        FXCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(fx_scratch)));
        g_fx_scratch[dev] = p;
    }
    *out = g_fx_scratch[dev];
    return MC_OK;
}

int fx_validate_input(const mcf_system* s, const double* pos, const uint8_t* types)
{
    const uint32_t N = s->g.N, n = s->g.n;
    for (size_t i = 0; i < 3 * (size_t)N; ++i)
        if (!std::isfinite(pos[i])) return fx_fail(MC_EINVAL, "position of atom %zu is not finite", i / 3);
    for (uint32_t m = 0; m < s->p.n_molecules; ++m) {
        uint32_t seen = 0;
        for (uint32_t t = 0; t < n; ++t) {
            const uint32_t ty = types[n * m + t];
            if (ty >= n || (seen >> ty) & 1u)
                return fx_fail(MC_EINVAL, "types of molecule %u are not a permutation of 0..%u", m, n - 1);
            seen |= 1u << ty;
        }
    }
    return MC_OK;
}

// Lay out, clear and start system s: its state in `state` (the layout's
// regions before the work arrays), its work arrays at `work` (work_off = the
// layout offset that lands on `work`).  no_alloc: clear with a kernel and
// stage host positions through the state's own r0 region, so that nothing is
// allocated.
int fx_init(mcf_system* s, const mcf_params* p, const FxGeom& g, const FxLayout& lay, const double* pos,
            const uint8_t* types, uint8_t* state, uint8_t* work, size_t work_off, hipStream_t stream,
            bool no_alloc)
{
    const bool lattice = !pos && !types;
    uint32_t nl = 1;
    while ((nl + 1) * (nl + 1) * (nl + 1) <= p->n_molecules) ++nl;
    s->p = *p;
    s->g = g;
    s->lay = lay;
    s->stream = stream;
    s->sweep = s->origin = 0;
    s->lds = fx_resident_lds(p, g);
    if (s->lds) {
        static std::mutex mu;
        static size_t configured = 0;
        std::lock_guard<std::mutex> lk(mu);
        if (s->lds > configured) {
            FXCHK(hipFuncSetAttribute((const void*)&k_fx_sweeps<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)s->lds));
            configured = s->lds;
        }
    }
    if (!lattice)
        if (int rc = fx_validate_input(s, pos, types)) return rc;
    FxDev& D = s->host;
    std::memset(&D, 0, sizeof D);
    uint8_t* b = state;
    D.geometry = p->geometry;
    D.n = g.n;
    D.M = p->n_molecules;
    D.N = g.N;
    D.k = g.k;
    D.nc = g.nc;
    D.ncell = g.ncell;
    D.nflip = kNPerm[p->geometry];
    D.seed_lo = (uint32_t)p->seed;
    D.seed_hi = (uint32_t)(p->seed >> 32);
    for (int bnd = 0; bnd < 6; ++bnd) {
        const int i = kBondsOf[p->geometry][bnd][0], j = kBondsOf[p->geometry][bnd][1];
        if (i >= 0) D.bonded |= 1u << (4 * std::min(i, j) + std::max(i, j));
    }
    D.resum_interval = p->resum_interval;
    D.obs_interval = p->obs_interval;
    D.gofr_interval = p->gofr_interval;
    D.obs_start = p->obs_start;
    D.max_samples = p->max_samples;
    D.L = g.L;
    D.invL = 1.0 / g.L;
    D.w = g.w;
    D.T = p->temperature;
    D.p_flip = p->p_flip;
    D.dmax = p->max_displacement;
    D.rc2f = std::cbrt(2.0);
    D.sep = (double)(g.k - 1) * g.w;
    D.dyn_base = g.rc + 4.0 * std::sqrt(3.0) * p->max_displacement + 1e-9;
    D.together = (p->flags & MC_FLAG_SERIAL_CELLS) ? 2u : (D.sep >= g.reach ? 1u : 0u);
    for (int t = 0; t < 4; ++t) D.sigma[t] = t < (int)g.n ? p->sigma[t] : 1.0;
    const double rmax = std::min(0.5 * g.L, 5.0);
    D.gofr_nbins = std::min((uint32_t)kGofrBins, (uint32_t)std::floor(rmax / p->gofr_dr + 1e-6));
    D.gofr_dr = p->gofr_dr;
    D.gofr_rmax = rmax;
    D.fs_q = p->fs_q;
    D.fs_q_cm = p->fs_q_cm;
    std::memcpy(D.flips, kPerm[p->geometry], sizeof D.flips);
    D.pos = (double*)(b + lay.pos);
    D.type = b + lay.type;
    D.img = (int32_t*)(b + lay.img);
    D.stats = (Stats*)(b + lay.stats);
    D.e_samples = (double*)(b + lay.esamp);
    D.drift_samples = (double*)(b + lay.dsamp);
    D.gofr_all = (uint64_t*)(b + lay.gall);
    D.gofr_inter = (uint64_t*)(b + lay.ginter);
    D.c2 = (double*)(b + lay.c2);
    D.c2_sweep = (uint64_t*)(b + lay.c2s);
    D.fs = (double*)(b + lay.fs);
    D.fs_cm = (double*)(b + lay.fscm);
    D.mom = (double*)(b + lay.mom);
    D.u0 = (double*)(b + lay.u0);
    D.kref = b + lay.kref;
    D.r0 = (double*)(b + lay.r0);
    D.rcm0 = (double*)(b + lay.rcm0);
    D.cell_start = (uint32_t*)(work + (lay.cstart - work_off));
    D.cell_list = (uint32_t*)(work + (lay.clist - work_off));
    D.cell_id = (uint32_t*)(work + (lay.cid - work_off));
    D.ecell = (double*)(work + (lay.ecell - work_off));
    D.part = (double*)(work + (lay.part - work_off));
    s->dev = (FxDev*)(b + lay.dev);
    int rc;
    if (no_alloc) {
        // both regions are multiples of 256 bytes
        hipLaunchKernelGGL(k_fx_zero, dim3(256), dim3(256), 0, stream, (uint64_t*)state, lay.cstart / 8);
        FXCHK(hipGetLastError());
        hipLaunchKernelGGL(k_fx_zero, dim3(256), dim3(256), 0, stream, (uint64_t*)(work), (lay.total - lay.cstart) / 8);
        FXCHK(hipGetLastError());
    } else {
        FXCHK(hipMemsetAsync(state, 0, lay.total, stream));
    }
    if ((rc = fx_upload_desc(s))) return rc;
    if (lattice) {
        const double side = p->bond_length > 0 ? p->bond_length : fx_bond_star();
        hipLaunchKernelGGL(k_fx_init_lattice, dim3((p->n_molecules + 255) / 256), dim3(256), 0, stream,
                           s->dev, nl, side);
        FXCHK(hipGetLastError());
    } else if (no_alloc) {
        FXCHK(hipMemcpyAsync(D.r0, pos, 3 * sizeof(double) * g.N, hipMemcpyHostToDevice, stream));
        FXCHK(hipMemcpyAsync(D.type, types, g.N, hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(k_fx_from_aos, dim3((g.N + 255) / 256), dim3(256), 0, stream, s->dev,
                           (const double*)D.r0);
        FXCHK(hipGetLastError());
    } else if ((rc = fx_upload_state(s, pos, types))) {
        return rc;
    }
    if ((rc = fx_events(s, kFlagResumSet | kFlagObsReset))) return rc;
    Stats st;
    if ((rc = fx_read_stats(s, &st))) return rc;
    if (!std::isfinite(st.e_acc)) return fx_fail(MC_ENONFINITE, "initial energy is not finite");
    return MC_OK;
}

int fx_check_request(const mcf_params* p, const double* pos, const uint8_t* types, FxGeom* g)
{
    int rc = fx_geometry(p, g);
    if (rc) return rc;
    const bool lattice = !pos && !types;
    if (!lattice && !(pos && types)) return fx_fail(MC_EINVAL, "give pos and types together, or neither");
    uint32_t nl = 1;
    while ((nl + 1) * (nl + 1) * (nl + 1) <= p->n_molecules) ++nl;
    if (lattice && nl * nl * nl != p->n_molecules)
        return fx_fail(MC_EINVAL, "lattice start needs n_molecules = n^3 (got %u)", p->n_molecules);
    return MC_OK;
}

}  // namespace

extern "C" {

int mcf_init_system(const mcf_params* p, const double* pos, const uint8_t* types, void* device_buf,
                    size_t buf_bytes, void* hip_stream, mcf_system** out)
{
    if (!out) return fx_fail(MC_EINVAL, "null output handle");
    *out = nullptr;
    FxGeom g;
    if (int rc = fx_check_request(p, pos, types, &g)) return rc;
    if (!device_buf) return fx_fail(MC_EINVAL, "null device buffer");
    if (((uintptr_t)device_buf & 255u) != 0) return fx_fail(MC_EINVAL, "device buffer must be 256-byte aligned");
    const FxLayout lay = fx_layout(p, g);
    if (buf_bytes < lay.total) return fx_fail(MC_ENOMEM, "device buffer of %zu bytes, %zu needed", buf_bytes, lay.total);
    mcf_system* s = new mcf_system();
    s->pooled = 0;
    uint8_t* b = (uint8_t*)device_buf;
    if (int rc = fx_init(s, p, g, lay, pos, types, b, b, 0, (hipStream_t)hip_stream, false)) {
        delete s;
        return rc;
    }
    *out = s;
    return MC_OK;
}

int mcf_init_system_noalloc(const mcf_params* p, const double* pos, const uint8_t* types,
                            void* device_state, size_t state_bytes, size_t* state_bytes_needed,
                            void* hip_stream, mcf_system** out)
{
    FxGeom g;
    if (int rc = fx_check_request(p, pos, types, &g)) return rc;
    const FxLayout lay = fx_layout(p, g);
    const size_t need = lay.cstart, work = lay.total - lay.cstart;
    if (state_bytes_needed) *state_bytes_needed = need;
    if (work > kFxScratchBytes)
        return fx_fail(MC_ENOMEM, "work arrays of %zu bytes exceed the static scratch of %zu bytes", work,
                       kFxScratchBytes);
    if (!device_state) return MC_OK;  // size query
    if (!out) return fx_fail(MC_EINVAL, "null output handle");
    *out = nullptr;
    if (((uintptr_t)device_state & 255u) != 0) return fx_fail(MC_EINVAL, "device buffer must be 256-byte aligned");
    if (state_bytes < need) return fx_fail(MC_ENOMEM, "device buffer of %zu bytes, %zu needed", state_bytes, need);
    void* scratch = nullptr;
    if (int rc = fx_scratch_ptr(&scratch)) return rc;
    int slot = -1;
    {
        std::lock_guard<std::mutex> lk(g_fx_mu);
        for (int i = 0; i < kFxPool && slot < 0; ++i)
            if (!g_fx_used[i]) {
                g_fx_used[i] = true;
                slot = i;
            }
    }
    if (slot < 0) return fx_fail(MC_EBUSY, "%d allocation-free systems are alive already", kFxPool);
    mcf_system* s = &g_fx_pool[slot];
    s->pooled = slot + 1;
    if (int rc = fx_init(s, p, g, lay, pos, types, (uint8_t*)device_state, (uint8_t*)scratch, lay.cstart,
                         (hipStream_t)hip_stream, true)) {
        std::lock_guard<std::mutex> lk(g_fx_mu);
        g_fx_used[slot] = false;
        return rc;
    }
    *out = s;
    return MC_OK;
}

namespace {

// `chunk` sweeps of systems s[0 .. n), n <= kFxMany, on `stream`: one launch
// for those with their state in LDS, one for the others.
int fx_launch_sweeps(mcf_system* const* s, uint32_t n, uint64_t chunk, hipStream_t stream)
{
    FxList res{}, buf{};
    uint32_t nr = 0, nb = 0;
    size_t lds = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (s[i]->lds) {
            res.d[nr++] = s[i]->dev;
            lds = std::max(lds, s[i]->lds);
        } else {
            buf.d[nb++] = s[i]->dev;
        }
    }
    if (nr) {
        hipLaunchKernelGGL(k_fx_sweeps<true>, dim3(nr), dim3(kFxThreads), lds, stream, res, chunk);
        FXCHK(hipGetLastError());
    }
    if (nb) {
        hipLaunchKernelGGL(k_fx_sweeps<false>, dim3(nb), dim3(kFxThreads), 0, stream, buf, chunk);
        FXCHK(hipGetLastError());
    }
    return MC_OK;
}

// n sweeps of the systems s[0 .. count), split at every sweep where one of
// them has events.
int fx_sweep_systems(mcf_system* const* s, uint32_t count, uint64_t n)
{
    while (n > 0) {
        uint64_t chunk = n;
        for (uint32_t i = 0; i < count; ++i) chunk = std::min<uint64_t>(chunk, fx_next_event(s[i]) - s[i]->sweep);
        for (uint32_t i0 = 0; i0 < count; i0 += kFxMany)
            if (int rc = fx_launch_sweeps(s + i0, std::min(kFxMany, count - i0), chunk, s[0]->stream)) return rc;
        n -= chunk;
        // the systems' events, those with the same flags in one launch pair
        // (no heap memory: mcf_sweep allocates nothing)
        for (uint32_t i0 = 0; i0 < count; i0 += kFxMany) {
            const uint32_t nb = std::min(kFxMany, count - i0);
            uint32_t flags[kFxMany];
            for (uint32_t i = 0; i < nb; ++i) {
                mcf_system* x = s[i0 + i];
                x->sweep += chunk;
                flags[i] = fx_events_at(x, x->sweep);
            }
            for (uint32_t i = 0; i < nb; ++i) {
                const uint32_t f = flags[i];
                if (!f) continue;
                mcf_system* group[kFxMany];
                uint32_t ng = 0;
                for (uint32_t j = i; j < nb; ++j)
                    if (flags[j] == f) {
                        group[ng++] = s[i0 + j];
                        flags[j] = 0;
                    }
                if (int rc = fx_events_of(group, ng, f, s[0]->stream)) return rc;
            }
        }
    }
    return MC_OK;
}

}  // namespace

int mcf_sweep(mcf_system* s, uint64_t n)
{
    if (!s) return fx_fail(MC_EINVAL, "null system");
    return fx_sweep_systems(&s, 1, n);
}

int mcf_sweep_many(mcf_system* const* systems, uint32_t count, uint64_t n)
{
    if (!systems || count == 0) return fx_fail(MC_EINVAL, "no systems");
    std::vector<mcf_system*> v(systems, systems + count);
    for (uint32_t i = 0; i < count; ++i) {
        if (!v[i]) return fx_fail(MC_EINVAL, "null system at %u", i);
        if (v[i]->stream != v[0]->stream) return fx_fail(MC_EINVAL, "system %u is on another stream", i);
    }
    std::vector<mcf_system*> sorted(v);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fx_fail(MC_EINVAL, "a system appears twice");
    return fx_sweep_systems(v.data(), count, n);
}

int mcf_energy(mcf_system* s, double* e_total, double* e_per_molecule, double* drift)
{
    if (!s) return fx_fail(MC_EINVAL, "null system");
    int rc = fx_events(s, kFlagResumReport);
    if (rc) return rc;
    Stats st;
    if ((rc = fx_read_stats(s, &st))) return rc;
    if (e_total) *e_total = st.e_resum;
    if (e_per_molecule) *e_per_molecule = st.e_resum / (double)s->p.n_molecules;
    if (drift) *drift = st.e_acc - st.e_resum;
    if (!std::isfinite(st.e_resum)) return fx_fail(MC_ENONFINITE, "energy is not finite");
    return MC_OK;
}

int mcf_observables(mcf_system* s, mc_obs* o)
{
    if (!s || !o) return fx_fail(MC_EINVAL, "null argument");
    Stats st;
    int rc = fx_read_stats(s, &st);
    if (rc) return rc;
    std::memset(o, 0, sizeof *o);
    o->sweep = st.sweep;
    for (int i = 0; i < 3; ++i) {
        o->attempts[i] = st.attempts[i];
        o->accepts[i] = st.accepts[i];
    }
    o->exits = st.exits;
    o->pair_terms = st.pair_terms;
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
    FXCHK(hipMemcpyAsync(o->gofr_all, s->host.gofr_all, sizeof o->gofr_all, hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipMemcpyAsync(o->gofr_inter, s->host.gofr_inter, sizeof o->gofr_inter, hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipMemcpyAsync(o->c2, s->host.c2, sizeof o->c2, hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipMemcpyAsync(o->fs, s->host.fs, sizeof o->fs, hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipMemcpyAsync(o->fs_cm, s->host.fs_cm, sizeof o->fs_cm, hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipMemcpyAsync(o->c2_sweep, s->host.c2_sweep, sizeof o->c2_sweep, hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipMemcpyAsync(o->c2_sq, s->host.mom, sizeof o->c2_sq, hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipMemcpyAsync(o->fs_cm_sq, s->host.mom + kC2Max, sizeof o->fs_cm_sq, hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipMemcpyAsync(o->c2_fs_cm, s->host.mom + 2 * kC2Max, sizeof o->c2_fs_cm, hipMemcpyDeviceToHost,
                         s->stream));
    FXCHK(hipMemcpyAsync(o->fs_sq, s->host.mom + 3 * kC2Max, sizeof o->fs_sq, hipMemcpyDeviceToHost, s->stream));
    FXCHK(hipStreamSynchronize(s->stream));
    // Eq. (3) normalised with N atoms at number density N / L^3
    const double N = (double)s->g.N, rho = N / (s->g.L * s->g.L * s->g.L), fr = (double)o->n_gofr_frames;
    for (uint32_t b = 0; b < o->gofr_nbins && fr > 0.0; ++b) {
        const double r0 = o->gofr_dr * b, r1 = o->gofr_dr * (b + 1);
        const double ideal = fr * N * rho * 4.0 * M_PI / 3.0 * (r1 * r1 * r1 - r0 * r0 * r0);
        o->gofr_norm_all[b] = (double)o->gofr_all[b] / ideal;
        o->gofr_norm_inter[b] = (double)o->gofr_inter[b] / ideal;
    }
    return MC_OK;
}

int mcf_reset_observables(mcf_system* s)
{
    if (!s) return fx_fail(MC_EINVAL, "null system");
    s->origin = s->sweep;
    return fx_events(s, kFlagObsReset);
}

int mcf_get_state(mcf_system* s, double* pos, uint8_t* types, uint64_t* sweep, double* e_acc)
{
    if (!s) return fx_fail(MC_EINVAL, "null system");
    const uint32_t N = s->g.N;
    std::vector<double> x(3 * (size_t)N);
    FXCHK(hipMemcpyAsync(x.data(), s->host.pos, x.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (types) FXCHK(hipMemcpyAsync(types, s->host.type, N, hipMemcpyDeviceToHost, s->stream));
    Stats st;
    if (int rc = fx_read_stats(s, &st)) return rc;
    if (pos)
        for (uint32_t i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d) pos[3 * i + d] = x[(size_t)d * N + i];
    if (sweep) *sweep = st.sweep;
    if (e_acc) *e_acc = st.e_acc;
    return MC_OK;
}

int mcf_set_state(mcf_system* s, const double* pos, const uint8_t* types, uint64_t sweep, double e_acc)
{
    if (!s || !pos || !types) return fx_fail(MC_EINVAL, "null argument");
    int rc = fx_upload_state(s, pos, types);
    if (rc) return rc;
    Stats st;
    if ((rc = fx_read_stats(s, &st))) return rc;
    st.sweep = sweep;
    st.e_acc = std::isnan(e_acc) ? 0.0 : e_acc;
    if (sweep < s->origin) {
        st.obs_origin = sweep;
        s->origin = sweep;
    }
    FXCHK(hipMemcpyAsync(s->host.stats, &st, sizeof st, hipMemcpyHostToDevice, s->stream));
    FXCHK(hipStreamSynchronize(s->stream));
    s->sweep = sweep;
    if (std::isnan(e_acc)) {
        if ((rc = fx_events(s, kFlagResumSet))) return rc;
        if ((rc = fx_read_stats(s, &st))) return rc;
        if (!std::isfinite(st.e_acc)) return fx_fail(MC_ENONFINITE, "energy of the new state is not finite");
    }
    return MC_OK;
}

int mcf_decision_log(mcf_system* s, void* device_records, size_t capacity)
{
    if (!s) return fx_fail(MC_EINVAL, "null system");
    Stats st;
    if (int rc = fx_read_stats(s, &st)) return rc;
    s->host.log = (MoveRecord*)device_records;
    s->host.log_sweep0 = st.sweep;
    s->host.log_sweeps = device_records ? capacity / s->g.N : 0;
    return fx_upload_desc(s);
}

void mcf_destroy(mcf_system* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->pooled) {
        std::lock_guard<std::mutex> lk(g_fx_mu);
        g_fx_used[s->pooled - 1] = false;
        return;
    }
    delete s;
}

}  // extern "C"
