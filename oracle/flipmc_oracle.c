/*
 * flipmc_oracle.c -- serial FP64 oracle for flip Monte Carlo of rigid
 * three-site A/B/C molecules.  TEST INFRASTRUCTURE ONLY (see the header).
 *
 * What it computes, and where the paper defines it:
 *   - the molecule (Sec. II.A): atoms A, B, C with diameters 0.9, 1, 1.1,
 *     sigma_ij = (sigma_i + sigma_j) / 2, site-site WCA potential (Eq. 1)
 *     with cut-off 2^(1/6) sigma_ij, FENE bonds (Eq. 2);
 *   - the box (Sec. II.A): cubic, periodic, N / V = 1.2 with N = 3 M sites;
 *   - flip Monte Carlo (Sec. II.B): pick a molecule, pick one of the three
 *     median axes, exchange the chemical identity of the two other summits,
 *     Metropolis acceptance; mixed with ordinary moves, flips with
 *     probability p_flip = 0.2; a timestep is N attempted moves;
 *   - observables (Sec. III.A Eq. 3, Sec. III.B Eq. 7).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - the molecule is a rigid equilateral triangle whose side b* minimises
 *     WCA + FENE of a sigma_ij = 1 bond, so the intramolecular energy is a
 *     constant and drops out of every energy difference;
 *   - ordinary moves are whole-molecule translations (uniform per component in
 *     [-d, d)) and rotations (axis uniform on the sphere, angle uniform in
 *     [-theta, theta)), split 0.4 / 0.4 next to 0.2 flips;
 *   - a flip swaps the types of sites (a+1)%3 and (a+2)%3 at fixed positions;
 *     for an equilateral triangle this equals a 180 degree rotation about the
 *     median through site a;
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
 *     keyed by the seed and counted by (slot, sweep low, sweep high, tag);
 *   - sweeps: either the checkerboard schedule (a random shift of a cubic
 *     cell grid per sweep; colours in order; every molecule tried once, in
 *     ascending index inside its cell, and confined to its cell) or the
 *     random-sequential schedule (M trials on uniformly drawn molecules).
 */
#include "flipmc_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define TWO_PI 6.283185307179586 /* closest double to 2 pi */

struct or_system {
    or_params p;
    double    L;          /* box side */
    double    w;          /* cell width L / n_c */
    double    bond;       /* triangle side */
    double    reach;      /* W */
    double    body[9];    /* body-frame site offsets, rows = sites */
    double*   com;        /* 3 M */
    double*   quat;       /* 4 M, (w, x, y, z) */
    uint8_t*  type;       /* 3 M */
    double*   site;       /* 9 M: site positions c + R(q) b, refreshed on change */
    int32_t*  img;        /* 3 M: periodic images crossed by accepted translations */
    uint64_t  sweep;
    double    e_acc;
    uint64_t  attempts[3], accepts[3], exits, pair_terms;
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the description in Salmon et al., SC'11: ten rounds of
 * two 32x32->64 multiplications; the key is bumped by the Weyl constants
 * between rounds.                                                           */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * x0;
        uint64_t p1 = (uint64_t)M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double or_u32(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

double or_u53(uint32_t lo, uint32_t hi)
{
    uint64_t v = ((uint64_t)hi << 32) | lo;
    return (double)((v >> 11) + 1) * 0x1p-53;
}

double or_u53_left(uint32_t lo, uint32_t hi)
{
    uint64_t v = ((uint64_t)hi << 32) | lo;
    return (double)(v >> 11) * 0x1p-53;
}

static void draw(const or_system* s, uint32_t slot, uint64_t sweep, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = {slot, (uint32_t)sweep, (uint32_t)(sweep >> 32), tag};
    uint32_t key[2] = {(uint32_t)s->p.seed, (uint32_t)(s->p.seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Model (Sec. II.A). */

double or_wca(double r2, double sigma_ij)
{
    /* Eq. (1): 4 eps [(s/r)^12 - (s/r)^6 + 1/4] for r < 2^(1/6) s, else 0. */
    double rc2 = cbrt(2.0) * sigma_ij * sigma_ij;
    if (!(r2 < rc2)) return 0.0;
    double s2 = sigma_ij * sigma_ij / r2;
    double s6 = s2 * s2 * s2;
    double s12 = s6 * s6;
    return 4.0 * (s12 - s6 + 0.25);
}

double or_fene(double r, double sigma_ij)
{
    /* Eq. (2): -33.75 eps ln(1 - (r / 1.5 s)^2). */
    double x = r / (1.5 * sigma_ij);
    return -33.75 * log(1.0 - x * x);
}

static double bond_energy_slope(double x)
{
    /* d/dx [WCA + FENE] at sigma_ij = 1, for x below the WCA cut-off. */
    double wca = 4.0 * (-12.0 * pow(x, -13.0) + 6.0 * pow(x, -7.0));
    double fene = 33.75 * (2.0 * x / 2.25) / (1.0 - x * x / 2.25);
    return wca + fene;
}

double or_bond_length_star(void)
{
    /* Bisection for the zero of the slope on [0.9, 1.1]: the slope is
     * negative at 0.9 (WCA dominates) and positive at 1.1. */
    double a = 0.9, b = 1.1;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (a + b);
        if (m == a || m == b) break;
        if (bond_energy_slope(m) < 0.0) a = m; else b = m;
    }
    return 0.5 * (a + b);
}

double or_box_length(uint32_t n_molecules, double density)
{
    return cbrt(3.0 * (double)n_molecules / density);
}

double or_stencil_reach(const double sigma[3], double bond_length)
{
    double smax = sigma[0];
    if (sigma[1] > smax) smax = sigma[1];
    if (sigma[2] > smax) smax = sigma[2];
    double radius = bond_length / sqrt(3.0);
    return pow(2.0, 1.0 / 6.0) * smax + 2.0 * radius;
}

void or_rotation_matrix(const double q[4], double r[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    r[0] = 1.0 - 2.0 * (y * y + z * z);
    r[1] = 2.0 * (x * y - w * z);
    r[2] = 2.0 * (x * z + w * y);
    r[3] = 2.0 * (x * y + w * z);
    r[4] = 1.0 - 2.0 * (x * x + z * z);
    r[5] = 2.0 * (y * z - w * x);
    r[6] = 2.0 * (x * z - w * y);
    r[7] = 2.0 * (y * z + w * x);
    r[8] = 1.0 - 2.0 * (x * x + y * y);
}

void or_body_frame(double bond_length, double b[9])
{
    /* Equilateral triangle of side b centred on its centroid, in the xy plane. */
    double radius = bond_length / sqrt(3.0);
    b[0] = radius;        b[1] = 0.0;                b[2] = 0.0;
    b[3] = -0.5 * radius; b[4] = 0.5 * bond_length;  b[5] = 0.0;
    b[6] = -0.5 * radius; b[7] = -0.5 * bond_length; b[8] = 0.0;
}

static void place_sites(const double body[9], const double c[3], const double q[4], double out[9])
{
    double r[9];
    or_rotation_matrix(q, r);
    for (int s = 0; s < 3; ++s)
        for (int a = 0; a < 3; ++a)
            out[3 * s + a] = c[a] + (r[3 * a + 0] * body[3 * s + 0] +
                                     r[3 * a + 1] * body[3 * s + 1] +
                                     r[3 * a + 2] * body[3 * s + 2]);
}

static void refresh_sites(or_system* s, uint32_t m)
{
    place_sites(s->body, &s->com[3 * m], &s->quat[4 * m], &s->site[9 * m]);
}

static double sigma_pair(const or_system* s, int ti, int tj)
{
    return 0.5 * (s->p.sigma[ti] + s->p.sigma[tj]);
}

static double min_image(double d, double L) { return d - L * nearbyint(d / L); }

static double dist2(const double* a, const double* b, double L)
{
    double dx = min_image(a[0] - b[0], L);
    double dy = min_image(a[1] - b[1], L);
    double dz = min_image(a[2] - b[2], L);
    return dx * dx + dy * dy + dz * dz;
}

static double wrap(double x, double L) { return x - L * floor(x / L); }

/* ------------------------------------------------------------------------ */

or_system* or_create(const or_params* p, char* err)
{
    char buf[256];
    if (!err) err = buf;
    err[0] = 0;
    if (p->n_molecules < 1) { snprintf(err, 256, "n_molecules must be >= 1"); return NULL; }
    if (!(p->density > 0) || !(p->temperature > 0)) {
        snprintf(err, 256, "density and temperature must be positive"); return NULL;
    }
    if (!(p->p_flip >= 0) || !(p->p_translate >= 0) || p->p_flip + p->p_translate > 1.0) {
        snprintf(err, 256, "move probabilities out of range"); return NULL;
    }
    or_system* s = (or_system*)calloc(1, sizeof(or_system));
    s->p = *p;
    s->bond = p->bond_length > 0 ? p->bond_length : or_bond_length_star();
    s->L = or_box_length(p->n_molecules, p->density);
    s->reach = or_stencil_reach(p->sigma, s->bond);
    or_body_frame(s->bond, s->body);
    uint32_t k = p->colours_per_axis, nc = p->cells_per_side;
    if (k < 2 || nc < 2 || nc % k != 0) {
        snprintf(err, 256, "need k >= 2, n_c >= 2, n_c %% k == 0 (k=%u n_c=%u)", k, nc);
        free(s); return NULL;
    }
    s->w = s->L / (double)nc;
    if ((double)(k - 1) * s->w < s->reach) {
        snprintf(err, 256, "(k-1) w = %.6f is below the interaction reach %.6f",
                 (double)(k - 1) * s->w, s->reach);
        free(s); return NULL;
    }
    double smax = fmax(p->sigma[0], fmax(p->sigma[1], p->sigma[2]));
    if (s->L < 2.0 * (pow(2.0, 1.0 / 6.0) * smax + 2.0 * p->max_displacement)) {
        snprintf(err, 256, "box too small for the minimum-image convention");
        free(s); return NULL;
    }
    size_t M = p->n_molecules;
    s->com = (double*)calloc(3 * M, sizeof(double));
    s->quat = (double*)calloc(4 * M, sizeof(double));
    s->type = (uint8_t*)calloc(3 * M, 1);
    s->site = (double*)calloc(9 * M, sizeof(double));
    s->img = (int32_t*)calloc(3 * M, sizeof(int32_t));
    for (size_t m = 0; m < M; ++m) {
        s->quat[4 * m] = 1.0;
        s->type[3 * m + 0] = 0; s->type[3 * m + 1] = 1; s->type[3 * m + 2] = 2;
    }
    return s;
}

void or_destroy(or_system* s)
{
    if (!s) return;
    free(s->com); free(s->quat); free(s->type); free(s->site); free(s->img); free(s);
}

double or_box(const or_system* s) { return s->L; }
double or_cell_width(const or_system* s) { return s->w; }

int or_init_lattice(or_system* s)
{
    /* Simple-cubic lattice of n^3 molecules at the centres of the lattice
     * cells; orientations uniform on SO(3) by Shoemake's method (Graphics
     * Gems III, 1992); types (A, B, C) on sites (0, 1, 2). */
    uint32_t M = s->p.n_molecules;
    uint32_t n = (uint32_t)llround(cbrt((double)M));
    if (n * n * n != M) return -1;
    double a = s->L / (double)n;
    for (uint32_t m = 0; m < M; ++m) {
        uint32_t i = m % n, j = (m / n) % n, l = m / (n * n);
        s->com[3 * m + 0] = ((double)i + 0.5) * a;
        s->com[3 * m + 1] = ((double)j + 0.5) * a;
        s->com[3 * m + 2] = ((double)l + 0.5) * a;
        uint32_t ctr[4] = {m, 0xFFFFFFFFu, 0xFFFFFFFFu, 2u};
        uint32_t key[2] = {(uint32_t)s->p.seed, (uint32_t)(s->p.seed >> 32)};
        uint32_t g[4];
        or_philox4x32_10(ctr, key, g);
        double u1 = or_u32(g[0]), u2 = or_u32(g[1]), u3 = or_u32(g[2]);
        double r1 = sqrt(1.0 - u1), r2 = sqrt(u1);
        s->quat[4 * m + 0] = r2 * cos(TWO_PI * u3);
        s->quat[4 * m + 1] = r1 * sin(TWO_PI * u2);
        s->quat[4 * m + 2] = r1 * cos(TWO_PI * u2);
        s->quat[4 * m + 3] = r2 * sin(TWO_PI * u3);
        s->type[3 * m + 0] = 0; s->type[3 * m + 1] = 1; s->type[3 * m + 2] = 2;
        refresh_sites(s, m);
    }
    memset(s->img, 0, 3 * sizeof(int32_t) * M);
    s->sweep = 0;
    s->e_acc = or_energy(s);
    memset(s->attempts, 0, sizeof s->attempts);
    memset(s->accepts, 0, sizeof s->accepts);
    s->exits = 0; s->pair_terms = 0;
    return 0;
}

int or_set_state(or_system* s, const double* com, const double* quat, const uint8_t* types,
                 uint64_t sweep, double e_acc)
{
    uint32_t M = s->p.n_molecules;
    memcpy(s->com, com, 3 * sizeof(double) * M);
    memcpy(s->quat, quat, 4 * sizeof(double) * M);
    memcpy(s->type, types, 3 * (size_t)M);
    for (uint32_t m = 0; m < M; ++m) refresh_sites(s, m);
    memset(s->img, 0, 3 * sizeof(int32_t) * M);
    s->sweep = sweep;
    s->e_acc = e_acc;
    return 0;
}

void or_get_state(const or_system* s, double* com, double* quat, uint8_t* types, uint64_t* sweep,
                  double* e_acc)
{
    uint32_t M = s->p.n_molecules;
    if (com) memcpy(com, s->com, 3 * sizeof(double) * M);
    if (quat) memcpy(quat, s->quat, 4 * sizeof(double) * M);
    if (types) memcpy(types, s->type, 3 * (size_t)M);
    if (sweep) *sweep = s->sweep;
    if (e_acc) *e_acc = s->e_acc;
}

void or_sites(const or_system* s, double* xyz)
{
    memcpy(xyz, s->site, 9 * sizeof(double) * s->p.n_molecules);
}

void or_unwrapped(const or_system* s, double* com, double* site)
{
    /* Positions followed through the periodic boundaries: the centre plus
     * the box lengths its accepted translations crossed, and each site index
     * at that centre plus R(q) b_k.  A flip exchanges types only, so it moves
     * no site index (Sec. III.B). */
    for (uint32_t m = 0; m < s->p.n_molecules; ++m) {
        double c[3], r[9];
        for (int a = 0; a < 3; ++a) c[a] = s->com[3 * m + a] + s->L * (double)s->img[3 * m + a];
        if (com) memcpy(&com[3 * m], c, sizeof c);
        if (!site) continue;
        or_rotation_matrix(&s->quat[4 * m], r);
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a)
                site[9 * m + 3 * k + a] = c[a] + (r[3 * a + 0] * s->body[3 * k + 0] +
                                                  r[3 * a + 1] * s->body[3 * k + 1] +
                                                  r[3 * a + 2] * s->body[3 * k + 2]);
    }
}

void or_counters(const or_system* s, uint64_t attempts[3], uint64_t accepts[3], uint64_t* exits,
                 uint64_t* pair_terms)
{
    for (int i = 0; i < 3; ++i) { attempts[i] = s->attempts[i]; accepts[i] = s->accepts[i]; }
    *exits = s->exits;
    *pair_terms = s->pair_terms;
}

/* ------------------------------------------------------------------------ */
/* Energies. */

double or_energy(const or_system* s)
{
    /* Sum over unordered pairs of distinct molecules and all 3 x 3 site pairs. */
    uint32_t M = s->p.n_molecules;
    double e = 0.0;
    for (uint32_t m = 0; m < M; ++m)
        for (uint32_t j = m + 1; j < M; ++j)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double r2 = dist2(&s->site[9 * m + 3 * a], &s->site[9 * j + 3 * b], s->L);
                    e += or_wca(r2, sigma_pair(s, s->type[3 * m + a], s->type[3 * j + b]));
                }
    return e;
}

double or_energy_intra(const or_system* s)
{
    /* WCA + FENE of the three bonds of each (rigid) molecule. */
    double e = 0.0;
    for (uint32_t m = 0; m < s->p.n_molecules; ++m)
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b) {
                double sij = sigma_pair(s, s->type[3 * m + a], s->type[3 * m + b]);
                double r2 = dist2(&s->site[9 * m + 3 * a], &s->site[9 * m + 3 * b], s->L);
                e += or_wca(r2, sij) + or_fene(sqrt(r2), sij);
            }
    return e;
}

/* Energy of the sites of molecule m selected by `mask`, placed at pos with
 * types ty, against every site of every other molecule. */
static double site_energy(const or_system* s, uint32_t m, const double pos[9], const uint8_t ty[3],
                          unsigned mask, uint32_t* terms)
{
    double e = 0.0;
    for (uint32_t j = 0; j < s->p.n_molecules; ++j) {
        if (j == m) continue;
        for (int a = 0; a < 3; ++a) {
            if (!(mask & (1u << a))) continue;
            for (int b = 0; b < 3; ++b) {
                double sij = sigma_pair(s, ty[a], s->type[3 * j + b]);
                double r2 = dist2(&pos[3 * a], &s->site[9 * j + 3 * b], s->L);
                if (r2 < cbrt(2.0) * sij * sij) ++*terms;
                e += or_wca(r2, sij);
            }
        }
    }
    return e;
}

/* ------------------------------------------------------------------------ */
/* Cells and shift of the checkerboard schedule. */

void or_shift(const or_system* s, uint64_t sweep, double h[3])
{
    uint32_t g[4];
    draw(s, 0xFFFFFFFFu, sweep, 3u, g);
    for (int a = 0; a < 3; ++a) h[a] = s->w * or_u32(g[a]);
}

static int cell_axis(const or_system* s, double x, double h)
{
    double g = wrap(x - h, s->L);
    int c = (int)floor(g / s->w);
    int nc = (int)s->p.cells_per_side;
    if (c >= nc) c = nc - 1;
    if (c < 0) c = 0;
    return c;
}

int or_cell_of(const or_system* s, const double c[3], uint64_t sweep)
{
    double h[3];
    or_shift(s, sweep, h);
    int nc = (int)s->p.cells_per_side;
    int cx = cell_axis(s, c[0], h[0]), cy = cell_axis(s, c[1], h[1]), cz = cell_axis(s, c[2], h[2]);
    return cx + nc * (cy + nc * cz);
}

/* ------------------------------------------------------------------------ */
/* One trial (the Metropolis step of Sec. II.B). */

static void trial(or_system* s, uint32_t m, uint32_t slot, const double* h, or_record* rec)
{
    uint64_t sweep = s->sweep;
    uint32_t b0[4], b1[4];
    draw(s, slot, sweep, 0u, b0);
    draw(s, slot, sweep, 1u, b1);
    double u_acc = or_u53(b0[0], b0[1]);
    double u_type = or_u32(b0[2]);
    double p0 = or_u32(b1[0]), p1 = or_u32(b1[1]), p2 = or_u32(b1[2]);

    int move;
    if (u_type < s->p.p_flip) move = OR_FLIP;
    else if (u_type < s->p.p_flip + s->p.p_translate) move = OR_TRANSLATE;
    else move = OR_ROTATE;

    double c_new[3], q_new[4], pos_new[9];
    uint8_t ty_new[3];
    const double* c_old = &s->com[3 * m];
    const double* q_old = &s->quat[4 * m];
    memcpy(c_new, c_old, sizeof c_new);
    memcpy(q_new, q_old, sizeof q_new);
    memcpy(ty_new, &s->type[3 * m], 3);
    unsigned mask = 7u;
    int axis = 255;
    int32_t crossed[3] = {0, 0, 0};

    rec->sweep = sweep; rec->molecule = m; rec->slot = slot; rec->move = (uint8_t)move;
    rec->accepted = 0; rec->exited = 0; rec->axis = 255; rec->pair_terms = 0;
    rec->delta_e = 0.0; rec->scale = 0.0;
    rec->t_log_u = s->p.temperature * log(u_acc);
    s->attempts[move]++;

    if (move == OR_TRANSLATE) {
        double p[3] = {p0, p1, p2};
        for (int a = 0; a < 3; ++a) {
            double x = c_old[a] + s->p.max_displacement * (2.0 * p[a] - 1.0);
            c_new[a] = wrap(x, s->L);
            crossed[a] = (int32_t)floor(x / s->L);  /* the box lengths wrap removed */
        }
        if (h) {
            int nc = (int)s->p.cells_per_side;
            int old_cell = cell_axis(s, c_old[0], h[0]) +
                           nc * (cell_axis(s, c_old[1], h[1]) + nc * cell_axis(s, c_old[2], h[2]));
            int new_cell = cell_axis(s, c_new[0], h[0]) +
                           nc * (cell_axis(s, c_new[1], h[1]) + nc * cell_axis(s, c_new[2], h[2]));
            if (old_cell != new_cell) {
                rec->exited = 1;
                s->exits++;
                return;
            }
        }
    } else if (move == OR_ROTATE) {
        double z = 2.0 * p0 - 1.0;
        double phi = TWO_PI * p1;
        double st = sqrt(1.0 - z * z);
        double n[3] = {st * cos(phi), st * sin(phi), z};
        double theta = s->p.max_rotation * (2.0 * p2 - 1.0);
        double ch = cos(0.5 * theta), sh = sin(0.5 * theta);
        double d[4] = {ch, n[0] * sh, n[1] * sh, n[2] * sh};
        /* q_new = d (x) q_old (Hamilton product), then normalised. */
        double w1 = d[0], x1 = d[1], y1 = d[2], z1 = d[3];
        double w2 = q_old[0], x2 = q_old[1], y2 = q_old[2], z2 = q_old[3];
        double r[4];
        r[0] = w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2;
        r[1] = w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2;
        r[2] = w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2;
        r[3] = w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2;
        double norm = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
        for (int i = 0; i < 4; ++i) q_new[i] = r[i] / norm;
    } else {
        axis = (int)(3.0 * p0);
        if (axis > 2) axis = 2;
        int s1 = (axis + 1) % 3, s2 = (axis + 2) % 3;
        uint8_t t = ty_new[s1]; ty_new[s1] = ty_new[s2]; ty_new[s2] = t;
        mask = (1u << s1) | (1u << s2);
        rec->axis = (uint8_t)axis;
    }
    place_sites(s->body, c_new, q_new, pos_new);

    uint32_t terms = 0;
    double e_old = site_energy(s, m, &s->site[9 * m], &s->type[3 * m], mask, &terms);
    double e_new = site_energy(s, m, pos_new, ty_new, mask, &terms);
    double de = e_new - e_old;
    rec->delta_e = de;
    rec->scale = e_new + e_old;
    rec->pair_terms = terms;
    s->pair_terms += terms;

    int accept = (de <= 0.0) || (rec->t_log_u < -de);
    if (accept) {
        memcpy(&s->com[3 * m], c_new, sizeof c_new);
        memcpy(&s->quat[4 * m], q_new, sizeof q_new);
        memcpy(&s->type[3 * m], ty_new, 3);
        for (int a = 0; a < 3; ++a) s->img[3 * m + a] += crossed[a];
        refresh_sites(s, m);
        s->e_acc += de;
        s->accepts[move]++;
        rec->accepted = 1;
    }
}

/* ------------------------------------------------------------------------ */
/* Sweeps. */

int or_sweep_checkerboard(or_system* s, uint64_t n_sweeps, or_record* log, uint64_t cell_order_seed)
{
    uint32_t M = s->p.n_molecules;
    int k = (int)s->p.colours_per_axis, nc = (int)s->p.cells_per_side;
    int ncell = nc * nc * nc;
    int* cell_of = (int*)malloc(sizeof(int) * M);
    int* count = (int*)malloc(sizeof(int) * (ncell + 1));
    int* start = (int*)malloc(sizeof(int) * (ncell + 1));
    uint32_t* members = (uint32_t*)malloc(sizeof(uint32_t) * M);
    int* order = (int*)malloc(sizeof(int) * ncell);
    for (uint64_t it = 0; it < n_sweeps; ++it) {
        double h[3];
        or_shift(s, s->sweep, h);
        /* cell of every molecule, lists in ascending molecule index */
        memset(count, 0, sizeof(int) * (ncell + 1));
        for (uint32_t m = 0; m < M; ++m) {
            const double* c = &s->com[3 * m];
            cell_of[m] = cell_axis(s, c[0], h[0]) +
                         nc * (cell_axis(s, c[1], h[1]) + nc * cell_axis(s, c[2], h[2]));
            count[cell_of[m]]++;
        }
        start[0] = 0;
        for (int c = 0; c < ncell; ++c) start[c + 1] = start[c] + count[c];
        memset(count, 0, sizeof(int) * (ncell + 1));
        for (uint32_t m = 0; m < M; ++m) {
            int c = cell_of[m];
            members[start[c] + count[c]++] = m;
        }
        uint32_t seq = 0;
        for (int colour = 0; colour < k * k * k; ++colour) {
            int kx = colour % k, ky = (colour / k) % k, kz = colour / (k * k);
            int n_in = 0;
            for (int cz = kz; cz < nc; cz += k)
                for (int cy = ky; cy < nc; cy += k)
                    for (int cx = kx; cx < nc; cx += k)
                        order[n_in++] = cx + nc * (cy + nc * cz);
            if (cell_order_seed) {
                /* Fisher-Yates shuffle driven by Philox on (i, colour, sweep). */
                for (int i = n_in - 1; i > 0; --i) {
                    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)colour, (uint32_t)s->sweep, 77u};
                    uint32_t key[2] = {(uint32_t)cell_order_seed, (uint32_t)(cell_order_seed >> 32)};
                    uint32_t g[4];
                    or_philox4x32_10(ctr, key, g);
                    int j = (int)(g[0] % (uint32_t)(i + 1));
                    int t = order[i]; order[i] = order[j]; order[j] = t;
                }
            }
            for (int ci = 0; ci < n_in; ++ci) {
                int c = order[ci];
                for (int q = start[c]; q < start[c + 1]; ++q) {
                    uint32_t m = members[q];
                    or_record rec;
                    trial(s, m, m, h, &rec);
                    rec.seq = seq++;
                    rec.pad = 0;
                    if (log) log[it * M + m] = rec;
                }
            }
        }
        s->sweep++;
    }
    free(cell_of); free(count); free(start); free(members); free(order);
    return 0;
}

int or_sweep_random(or_system* s, uint64_t n_sweeps, or_record* log)
{
    uint32_t M = s->p.n_molecules;
    for (uint64_t it = 0; it < n_sweeps; ++it) {
        for (uint32_t t = 0; t < M; ++t) {
            uint32_t g[4];
            draw(s, t, s->sweep, 4u, g);
            uint32_t m = (uint32_t)((double)M * or_u53_left(g[0], g[1]));
            if (m >= M) m = M - 1;
            or_record rec;
            trial(s, m, t, NULL, &rec);
            rec.seq = t;
            rec.pad = 0;
            if (log) log[it * M + t] = rec;
        }
        s->sweep++;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Observables. */

int or_gofr_bins(double box, double dr, double* r_max)
{
    double rm = 0.5 * box;
    if (rm > 5.0) rm = 5.0;
    if (r_max) *r_max = rm;
    return (int)floor(rm / dr + 1e-6);
}

void or_gofr_accumulate(const or_system* s, double dr, int nbins, uint64_t* counts_all,
                        uint64_t* counts_inter)
{
    /* Eq. (3) numerator: every ordered pair of distinct sites, binned by
     * distance; bin b holds [b dr, (b+1) dr). */
    uint32_t N = 3 * s->p.n_molecules;
    for (uint32_t i = 0; i < N; ++i)
        for (uint32_t j = 0; j < N; ++j) {
            if (i == j) continue;
            double r = sqrt(dist2(&s->site[3 * i], &s->site[3 * j], s->L));
            int b = (int)floor(r / dr);
            if (b < 0 || b >= nbins) continue;
            counts_all[b]++;
            if (i / 3 != j / 3) counts_inter[b]++;
        }
}

static void orientation(const or_system* s, uint32_t m, int k, double u[3])
{
    /* unit vector from the centre of mass to site k: R(q) b_k / |b_k| */
    double r[9];
    double radius = s->bond / sqrt(3.0);
    or_rotation_matrix(&s->quat[4 * m], r);
    for (int a = 0; a < 3; ++a)
        u[a] = (r[3 * a + 0] * s->body[3 * k + 0] + r[3 * a + 1] * s->body[3 * k + 1] +
                r[3 * a + 2] * s->body[3 * k + 2]) / radius;
}

void or_orientation_ref(const or_system* s, double* u0, uint8_t* kref)
{
    /* The orientation vector points from the centre of mass to the site that
     * carries type B at the reference time; later it follows that site index
     * whatever its type (Sec. III.B). */
    for (uint32_t m = 0; m < s->p.n_molecules; ++m) {
        int k = 0;
        for (int a = 0; a < 3; ++a)
            if (s->type[3 * m + a] == 1) k = a;
        kref[m] = (uint8_t)k;
        orientation(s, m, k, &u0[3 * m]);
    }
}

void or_c2_terms(const or_system* s, const double* u0, const uint8_t* kref, double* c2i)
{
    /* Contribution of each molecule to C_2 (Sec. V.A): P_2(u(t) . u(0)). */
    for (uint32_t m = 0; m < s->p.n_molecules; ++m) {
        double u[3];
        orientation(s, m, kref[m], u);
        double dot = u[0] * u0[3 * m] + u[1] * u0[3 * m + 1] + u[2] * u0[3 * m + 2];
        c2i[m] = 0.5 * (3.0 * dot * dot - 1.0);
    }
}

double or_c2(const or_system* s, const double* u0, const uint8_t* kref)
{
    /* Eq. (7) with l = 2: mean of P_2(u(t) . u(0)) over molecules. */
    double acc = 0.0;
    for (uint32_t m = 0; m < s->p.n_molecules; ++m) {
        double u[3];
        orientation(s, m, kref[m], u);
        double dot = u[0] * u0[3 * m] + u[1] * u0[3 * m + 1] + u[2] * u0[3 * m + 2];
        acc += 0.5 * (3.0 * dot * dot - 1.0);
    }
    return acc / (double)s->p.n_molecules;
}
