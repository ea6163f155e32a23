/*
 * flex_oracle.c -- serial FP64 oracle of flip Monte Carlo for flexible
 * molecules (triangles, squares, tetrahedra).  TEST INFRASTRUCTURE ONLY (see
 * flex_oracle.h).
 *
 * What it computes, and where the paper defines it:
 *   - atoms of diameters sigma_t, sigma_ij = (sigma_i + sigma_j) / 2, the WCA
 *     potential of Eq. 1 between every pair of atoms (intramolecular pairs
 *     included) and FENE bonds of Eq. 2 between the bonded atoms of a
 *     molecule (Sec. II.A); a bond cannot reach 1.5 sigma_ij, so a move that
 *     would stretch one that far has infinite energy and is rejected;
 *   - the box: cubic, periodic, N / V = density, N = n M atoms;
 *   - Monte Carlo (Sec. II.B): atom translations and flips (intramolecular
 *     type exchanges), Metropolis acceptance, a timestep is N attempts.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - a translation moves one atom by a uniform vector of [-d, d)^3;
 *   - a triangle's atoms are all bonded (three bonds); a square's four atoms
 *     form a ring of four bonds; a tetrahedron's four atoms are all bonded;
 *     the square and the tetrahedron carry four types of diameters evenly
 *     spaced over [0.9, 1.1];
 *   - a flip is one of the 180 degree rotations of the ideal body written as
 *     a permutation of the types at fixed positions; the rotation is uniform
 *     over the body's list;
 *   - the attempt order: the checkerboard over atoms (a random shift of a
 *     cubic cell grid per sweep, colours in order, the cells of a colour in
 *     ascending index, every atom attempted once in ascending index inside
 *     its cell, translations confined to the cell), or N attempts on
 *     uniformly drawn atoms (random sequential).  When same-colour cells are
 *     at least the reach 2 D + r_c apart the order of the cells of a colour
 *     does not matter (cell_order_seed shuffles it to show that); closer,
 *     the ascending order defines the chain;
 *   - the start: a simple-cubic lattice of ideal bodies of side b* with
 *     uniformly random orientations, types 0, 1, ... on atoms 0, 1, ...;
 *   - random numbers: Philox4x32-10 on (slot, sweep low, sweep high, tag) as in
 *     the rigid oracle (tags 0, 1 attempt; 2 lattice; 3 shift; 4 selection).
 */
#include "flex_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "flipmc_oracle.h"

#define TWO_PI 6.283185307179586

/* Bonds (pairs of atom indices inside a molecule) of each body. */
static const int kBonds[3][6][2] = {
    {{0, 1}, {1, 2}, {0, 2}, {-1, -1}, {-1, -1}, {-1, -1}},
    {{0, 1}, {1, 2}, {2, 3}, {0, 3}, {-1, -1}, {-1, -1}},
    {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}},
};
static const int kNBonds[3] = {3, 4, 6};
/* Largest number of bonds between two atoms of one molecule. */
static const int kGraphDiameter[3] = {1, 2, 1};

/* Flips: new type of atom s = old type of atom perm[s]. */
static const int kFlips[3][4][4] = {
    /* triangle: 180 degrees about the median through atom q swaps the other two */
    {{0, 2, 1, -1}, {2, 1, 0, -1}, {1, 0, 2, -1}, {-1, -1, -1, -1}},
    /* square (ring 0-1-2-3): the diagonals through 0, 2 and through 1, 3,
     * the bisectors of edges 01 / 23 and of edges 12 / 30 */
    {{0, 3, 2, 1}, {2, 1, 0, 3}, {1, 0, 3, 2}, {3, 2, 1, 0}},
    /* tetrahedron: the axes through the midpoints of opposite edges */
    {{1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}, {-1, -1, -1, -1}},
};
static const uint32_t kNFlips[3] = {3, 4, 3};

struct fx_system {
    fx_params p;
    uint32_t  n;          /* atoms per molecule */
    uint32_t  N;          /* atoms */
    double    L, w, bond, reach, bond_max, rc_max;
    double*   pos;        /* 3 N, wrapped into [0, L) */
    uint8_t*  type;       /* N */
    int32_t*  img;        /* 3 N periodic images crossed by accepted translations */
    uint8_t   bonded[4][4];
    uint64_t  sweep;
    double    e_acc;
    uint64_t  attempts[3], accepts[3], exits, pair_terms;
};

uint32_t fx_sites(uint32_t g) { return g == FX_TRIANGLE ? 3u : (g <= FX_TETRAHEDRON ? 4u : 0u); }
uint32_t fx_flip_kinds(uint32_t g) { return g <= FX_TETRAHEDRON ? kNFlips[g] : 0u; }

double fx_box_length(uint32_t g, uint32_t M, double density)
{
    return cbrt((double)fx_sites(g) * (double)M / density);
}

static double max_sigma(const fx_params* p, uint32_t n)
{
    double m = p->sigma[0];
    for (uint32_t t = 1; t < n; ++t) if (p->sigma[t] > m) m = p->sigma[t];
    return m;
}

/* Longest a bond can be: 1.5 sigma_ij for the largest pair of distinct types. */
static double bond_limit(const fx_params* p, uint32_t n)
{
    double b = 0.0;
    for (uint32_t i = 0; i < n; ++i)
        for (uint32_t j = i + 1; j < n; ++j) {
            double s = 1.5 * 0.5 * (p->sigma[i] + p->sigma[j]);
            if (s > b) b = s;
        }
    return b;
}

double fx_reach(const fx_params* p)
{
    uint32_t n = fx_sites(p->geometry);
    if (!n) return 0.0;
    double D = kGraphDiameter[p->geometry] * bond_limit(p, n);
    return 2.0 * D + pow(2.0, 1.0 / 6.0) * max_sigma(p, n);
}

static double min_image(double d, double L) { return d - L * nearbyint(d / L); }
static double wrap(double x, double L) { return x - L * floor(x / L); }

static double dist2(const double* a, const double* b, double L)
{
    double dx = min_image(a[0] - b[0], L);
    double dy = min_image(a[1] - b[1], L);
    double dz = min_image(a[2] - b[2], L);
    return dx * dx + dy * dy + dz * dz;
}

static void draw(const fx_system* s, uint32_t slot, uint64_t sweep, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = {slot, (uint32_t)sweep, (uint32_t)(sweep >> 32), tag};
    uint32_t key[2] = {(uint32_t)s->p.seed, (uint32_t)(s->p.seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* Energy of one pair of atoms at squared distance r2 with types ti, tj:
 * Eq. 1, plus Eq. 2 when they are bonded (infinite at or beyond 1.5 sigma_ij).
 * Counts the terms in range. */
static double pair_energy(const fx_system* s, double r2, int ti, int tj, int bonded, uint32_t* terms)
{
    double sij = 0.5 * (s->p.sigma[ti] + s->p.sigma[tj]);
    double e = or_wca(r2, sij);
    if (r2 < cbrt(2.0) * sij * sij) ++*terms;
    if (bonded) {
        double lim = 1.5 * sij;
        if (!(r2 < lim * lim)) return INFINITY;
        e += or_fene(sqrt(r2), sij);
        ++*terms;
    }
    return e;
}

static int same_molecule(const fx_system* s, uint32_t i, uint32_t j) { return i / s->n == j / s->n; }

static int is_bonded(const fx_system* s, uint32_t i, uint32_t j)
{
    return same_molecule(s, i, j) && s->bonded[i % s->n][j % s->n];
}

/* Energy of the pairs that involve at least one atom of the set S (flags
 * in_s, N entries) in the configuration (pos, type): every pair counted once. */
static double local_energy(const fx_system* s, const double* pos, const uint8_t* type,
                           const uint8_t* in_s, const uint32_t* list, int ns, uint32_t* terms)
{
    double e = 0.0;
    for (int q = 0; q < ns; ++q) {
        uint32_t i = list[q];
        for (uint32_t j = 0; j < s->N; ++j) {
            if (j == i || (in_s[j] && j < i)) continue;
            double r2 = dist2(&pos[3 * i], &pos[3 * j], s->L);
            e += pair_energy(s, r2, type[i], type[j], is_bonded(s, i, j), terms);
        }
    }
    return e;
}

fx_system* fx_create(const fx_params* p, char* err)
{
    char buf[256];
    if (!err) err = buf;
    err[0] = 0;
    uint32_t n = fx_sites(p->geometry);
    if (!n) { snprintf(err, 256, "unknown geometry %u", p->geometry); return NULL; }
    if (p->n_molecules < 1) { snprintf(err, 256, "n_molecules must be >= 1"); return NULL; }
    if (!(p->density > 0) || !(p->temperature > 0)) {
        snprintf(err, 256, "density and temperature must be positive"); return NULL;
    }
    if (!(p->p_flip >= 0) || p->p_flip > 1.0 || !(p->max_displacement >= 0)) {
        snprintf(err, 256, "p_flip or max_displacement out of range"); return NULL;
    }
    for (uint32_t t = 0; t < n; ++t)
        if (!(p->sigma[t] > 0)) { snprintf(err, 256, "sigma must be positive"); return NULL; }
    fx_system* s = (fx_system*)calloc(1, sizeof(fx_system));
    s->p = *p;
    s->n = n;
    s->N = n * p->n_molecules;
    s->L = fx_box_length(p->geometry, p->n_molecules, p->density);
    s->bond = p->bond_length > 0 ? p->bond_length : or_bond_length_star();
    s->bond_max = bond_limit(p, n);
    s->rc_max = pow(2.0, 1.0 / 6.0) * max_sigma(p, n);
    s->reach = fx_reach(p);
    for (int b = 0; b < kNBonds[p->geometry]; ++b) {
        int i = kBonds[p->geometry][b][0], j = kBonds[p->geometry][b][1];
        s->bonded[i][j] = s->bonded[j][i] = 1;
    }
    uint32_t k = p->colours_per_axis, nc = p->cells_per_side;
    if (k < 2 || nc < 2 || nc % k != 0) {
        snprintf(err, 256, "need k >= 2, n_c >= 2, n_c %% k == 0 (k=%u n_c=%u)", k, nc);
        free(s); return NULL;
    }
    s->w = s->L / (double)nc;
    if (s->w < s->rc_max + 2.0 * sqrt(3.0) * p->max_displacement) {
        snprintf(err, 256, "cell side %.6f is below r_c + 2 sqrt(3) d = %.6f", s->w,
                 s->rc_max + 2.0 * sqrt(3.0) * p->max_displacement);
        free(s); return NULL;
    }
    double D = kGraphDiameter[p->geometry] * s->bond_max;
    double need = 2.0 * ((D > s->rc_max ? D : s->rc_max) + 2.0 * p->max_displacement);
    if (s->L < need) {
        snprintf(err, 256, "box side %.6f below %.6f (minimum image)", s->L, need);
        free(s); return NULL;
    }
    s->pos = (double*)calloc(3 * (size_t)s->N, sizeof(double));
    s->type = (uint8_t*)calloc(s->N, 1);
    s->img = (int32_t*)calloc(3 * (size_t)s->N, sizeof(int32_t));
    for (uint32_t i = 0; i < s->N; ++i) s->type[i] = (uint8_t)(i % n);
    return s;
}

void fx_destroy(fx_system* s)
{
    if (!s) return;
    free(s->pos); free(s->type); free(s->img); free(s);
}

double fx_box(const fx_system* s) { return s->L; }

/* Atom offsets of the ideal body of side b around its centre (rows = atoms). */
static void ideal_body(uint32_t g, double b, double out[12])
{
    memset(out, 0, 12 * sizeof(double));
    if (g == FX_TRIANGLE) {
        double r = b / sqrt(3.0);
        out[0] = r;
        out[3] = -0.5 * r; out[4] = 0.5 * b;
        out[6] = -0.5 * r; out[7] = -0.5 * b;
    } else if (g == FX_SQUARE) {
        double h = 0.5 * b;
        out[0] = h;  out[1] = h;
        out[3] = -h; out[4] = h;
        out[6] = -h; out[7] = -h;
        out[9] = h;  out[10] = -h;
    } else {
        double c = b / (2.0 * sqrt(2.0));
        const double v[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) out[3 * s + a] = c * v[s][a];
    }
}

int fx_init_lattice(fx_system* s)
{
    uint32_t M = s->p.n_molecules;
    uint32_t nl = (uint32_t)llround(cbrt((double)M));
    if (nl * nl * nl != M) return -1;
    double a = s->L / (double)nl;
    double body[12];
    ideal_body(s->p.geometry, s->bond, body);
    for (uint32_t m = 0; m < M; ++m) {
        uint32_t i = m % nl, j = (m / nl) % nl, l = m / (nl * nl);
        double c[3] = {((double)i + 0.5) * a, ((double)j + 0.5) * a, ((double)l + 0.5) * a};
        uint32_t g[4];
        draw(s, m, 0xFFFFFFFFFFFFFFFFull, 2u, g);
        double u1 = or_u32(g[0]), u2 = or_u32(g[1]), u3 = or_u32(g[2]);
        double r1 = sqrt(1.0 - u1), r2 = sqrt(u1);
        double q[4] = {r2 * cos(TWO_PI * u3), r1 * sin(TWO_PI * u2), r1 * cos(TWO_PI * u2),
                       r2 * sin(TWO_PI * u3)};
        double R[9];
        or_rotation_matrix(q, R);
        for (uint32_t t = 0; t < s->n; ++t) {
            uint32_t at = s->n * m + t;
            for (int x = 0; x < 3; ++x) {
                double v = c[x] + (R[3 * x] * body[3 * t] + R[3 * x + 1] * body[3 * t + 1] +
                                   R[3 * x + 2] * body[3 * t + 2]);
                s->pos[3 * at + x] = wrap(v, s->L);
            }
            s->type[at] = (uint8_t)t;
        }
    }
    memset(s->img, 0, 3 * sizeof(int32_t) * s->N);
    s->sweep = 0;
    s->e_acc = fx_energy(s);
    return 0;
}

int fx_set_state(fx_system* s, const double* pos, const uint8_t* types, uint64_t sweep, double e_acc)
{
    memcpy(s->pos, pos, 3 * sizeof(double) * s->N);
    memcpy(s->type, types, s->N);
    memset(s->img, 0, 3 * sizeof(int32_t) * s->N);
    s->sweep = sweep;
    s->e_acc = isnan(e_acc) ? fx_energy(s) : e_acc;
    return 0;
}

void fx_get_state(const fx_system* s, double* pos, uint8_t* types, uint64_t* sweep, double* e_acc)
{
    if (pos) memcpy(pos, s->pos, 3 * sizeof(double) * s->N);
    if (types) memcpy(types, s->type, s->N);
    if (sweep) *sweep = s->sweep;
    if (e_acc) *e_acc = s->e_acc;
}

double fx_energy(const fx_system* s)
{
    double e = 0.0;
    uint32_t t = 0;
    for (uint32_t i = 0; i < s->N; ++i)
        for (uint32_t j = i + 1; j < s->N; ++j) {
            double r2 = dist2(&s->pos[3 * i], &s->pos[3 * j], s->L);
            e += pair_energy(s, r2, s->type[i], s->type[j], is_bonded(s, i, j), &t);
        }
    return e;
}

double fx_energy_inter(const fx_system* s)
{
    double e = 0.0;
    for (uint32_t i = 0; i < s->N; ++i)
        for (uint32_t j = i + 1; j < s->N; ++j) {
            if (same_molecule(s, i, j)) continue;
            double sij = 0.5 * (s->p.sigma[s->type[i]] + s->p.sigma[s->type[j]]);
            e += or_wca(dist2(&s->pos[3 * i], &s->pos[3 * j], s->L), sij);
        }
    return e;
}

static void shift(const fx_system* s, uint64_t sweep, double h[3])
{
    uint32_t g[4];
    draw(s, 0xFFFFFFFFu, sweep, 3u, g);
    for (int a = 0; a < 3; ++a) h[a] = s->w * or_u32(g[a]);
}

static int cell_axis(const fx_system* s, double x, double h)
{
    int c = (int)floor(wrap(x - h, s->L) / s->w);
    int nc = (int)s->p.cells_per_side;
    if (c >= nc) c = nc - 1;
    if (c < 0) c = 0;
    return c;
}

static int cell_of(const fx_system* s, const double* x, const double* h)
{
    int nc = (int)s->p.cells_per_side;
    return cell_axis(s, x[0], h[0]) + nc * (cell_axis(s, x[1], h[1]) + nc * cell_axis(s, x[2], h[2]));
}

/* One attempt (Sec. II.B) on atom a with random numbers of `slot`. */
static void attempt(fx_system* s, uint32_t a, uint32_t slot, const double* h, fx_record* rec)
{
    uint64_t sweep = s->sweep;
    uint32_t b0[4], b1[4];
    draw(s, slot, sweep, 0u, b0);
    draw(s, slot, sweep, 1u, b1);
    double u_acc = or_u53(b0[0], b0[1]);
    double u_type = or_u32(b0[2]);
    double pr[3] = {or_u32(b1[0]), or_u32(b1[1]), or_u32(b1[2])};
    int move = u_type < s->p.p_flip ? FX_FLIP : FX_TRANSLATE;
    uint32_t n = s->n, base = n * (a / n);

    memset(rec, 0, sizeof *rec);
    rec->sweep = sweep; rec->atom = a; rec->slot = slot; rec->move = (uint8_t)move;
    rec->kind = 255;
    rec->t_log_u = s->p.temperature * log(u_acc);
    s->attempts[move]++;

    /* the changed atoms and their new positions / types, in scratch copies */
    uint32_t list[4];
    int ns = 0;
    double newpos[12];
    uint8_t newtype[4];
    int32_t crossed[3] = {0, 0, 0};
    for (uint32_t t = 0; t < n; ++t) {
        memcpy(&newpos[3 * t], &s->pos[3 * (base + t)], 3 * sizeof(double));
        newtype[t] = s->type[base + t];
    }
    if (move == FX_TRANSLATE) {
        double* x = &newpos[3 * (a - base)];
        for (int d = 0; d < 3; ++d) {
            double v = s->pos[3 * a + d] + s->p.max_displacement * (2.0 * pr[d] - 1.0);
            x[d] = wrap(v, s->L);
            crossed[d] = (int32_t)floor(v / s->L);
        }
        if (h && cell_of(s, x, h) != cell_of(s, &s->pos[3 * a], h)) {
            rec->exited = 1;
            s->exits++;
            return;
        }
        list[ns++] = a;
    } else {
        uint32_t K = kNFlips[s->p.geometry];
        uint32_t q = (uint32_t)((double)K * pr[0]);
        if (q >= K) q = K - 1;
        rec->kind = (uint8_t)q;
        for (uint32_t t = 0; t < n; ++t) {
            newtype[t] = s->type[base + (uint32_t)kFlips[s->p.geometry][q][t]];
            if (newtype[t] != s->type[base + t]) list[ns++] = base + t;
        }
    }

    /* energies of the pairs touching a changed atom, before and after */
    uint8_t* in_s = (uint8_t*)calloc(s->N, 1);
    for (int q = 0; q < ns; ++q) in_s[list[q]] = 1;
    uint32_t terms = 0;
    double e_old = local_energy(s, s->pos, s->type, in_s, list, ns, &terms);
    /* the new configuration: the molecule's atoms replaced */
    double saved_pos[12];
    uint8_t saved_type[4];
    memcpy(saved_pos, &s->pos[3 * base], 3 * n * sizeof(double));
    memcpy(saved_type, &s->type[base], n);
    memcpy(&s->pos[3 * base], newpos, 3 * n * sizeof(double));
    memcpy(&s->type[base], newtype, n);
    double e_new = local_energy(s, s->pos, s->type, in_s, list, ns, &terms);
    free(in_s);
    double de = e_new - e_old;
    rec->delta_e = de;
    rec->scale = e_new + e_old;
    rec->pair_terms = terms;
    s->pair_terms += terms;
    int accept = (de <= 0.0) || (rec->t_log_u < -de);
    if (accept) {
        if (move == FX_TRANSLATE)
            for (int d = 0; d < 3; ++d) s->img[3 * a + d] += crossed[d];
        s->e_acc += de;
        s->accepts[move]++;
        rec->accepted = 1;
    } else {
        memcpy(&s->pos[3 * base], saved_pos, 3 * n * sizeof(double));
        memcpy(&s->type[base], saved_type, n);
    }
}

int fx_sweep_checkerboard(fx_system* s, uint64_t n_sweeps, fx_record* log, uint64_t cell_order_seed)
{
    uint32_t N = s->N;
    int k = (int)s->p.colours_per_axis, nc = (int)s->p.cells_per_side;
    int ncell = nc * nc * nc;
    int* cell = (int*)malloc(sizeof(int) * N);
    int* count = (int*)malloc(sizeof(int) * (ncell + 1));
    int* start = (int*)malloc(sizeof(int) * (ncell + 1));
    uint32_t* members = (uint32_t*)malloc(sizeof(uint32_t) * N);
    int* order = (int*)malloc(sizeof(int) * ncell);
    for (uint64_t it = 0; it < n_sweeps; ++it) {
        double h[3];
        shift(s, s->sweep, h);
        memset(count, 0, sizeof(int) * (ncell + 1));
        for (uint32_t i = 0; i < N; ++i) {
            cell[i] = cell_of(s, &s->pos[3 * i], h);
            count[cell[i]]++;
        }
        start[0] = 0;
        for (int c = 0; c < ncell; ++c) start[c + 1] = start[c] + count[c];
        memset(count, 0, sizeof(int) * (ncell + 1));
        for (uint32_t i = 0; i < N; ++i) members[start[cell[i]] + count[cell[i]]++] = i;
        uint32_t seq = 0;
        for (int colour = 0; colour < k * k * k; ++colour) {
            int kx = colour % k, ky = (colour / k) % k, kz = colour / (k * k);
            int n_in = 0;
            for (int cz = kz; cz < nc; cz += k)
                for (int cy = ky; cy < nc; cy += k)
                    for (int cx = kx; cx < nc; cx += k) order[n_in++] = cx + nc * (cy + nc * cz);
            if (cell_order_seed) {
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
                    uint32_t a = members[q];
                    fx_record rec;
                    attempt(s, a, a, h, &rec);
                    rec.seq = seq++;
                    if (log) log[it * N + a] = rec;
                }
            }
        }
        s->sweep++;
    }
    free(cell); free(count); free(start); free(members); free(order);
    return 0;
}

int fx_sweep_random(fx_system* s, uint64_t n_sweeps, fx_record* log)
{
    uint32_t N = s->N;
    for (uint64_t it = 0; it < n_sweeps; ++it) {
        for (uint32_t t = 0; t < N; ++t) {
            uint32_t g[4];
            draw(s, t, s->sweep, 4u, g);
            uint32_t a = (uint32_t)((double)N * or_u53_left(g[0], g[1]));
            if (a >= N) a = N - 1;
            fx_record rec;
            attempt(s, a, t, NULL, &rec);
            rec.seq = t;
            if (log) log[it * N + t] = rec;
        }
        s->sweep++;
    }
    return 0;
}

void fx_counters(const fx_system* s, uint64_t attempts[3], uint64_t accepts[3], uint64_t* exits,
                 uint64_t* pair_terms)
{
    for (int i = 0; i < 3; ++i) {
        attempts[i] = s->attempts[i];
        accepts[i] = s->accepts[i];
    }
    *exits = s->exits;
    *pair_terms = s->pair_terms;
}

void fx_gofr_accumulate(const fx_system* s, double dr, int nbins, uint64_t* counts_all,
                        uint64_t* counts_inter)
{
    /* Eq. (3) numerator: every ordered pair of distinct atoms */
    for (uint32_t i = 0; i < s->N; ++i)
        for (uint32_t j = 0; j < s->N; ++j) {
            if (i == j) continue;
            int b = (int)floor(sqrt(dist2(&s->pos[3 * i], &s->pos[3 * j], s->L)) / dr);
            if (b < 0 || b >= nbins) continue;
            counts_all[b]++;
            if (!same_molecule(s, i, j)) counts_inter[b]++;
        }
}

/* Centre of mass of molecule m (equal masses): atom 0 plus the mean of the
 * nearest-image offsets of the molecule's atoms from it. */
static void centre(const fx_system* s, uint32_t m, double c[3])
{
    uint32_t base = s->n * m;
    for (int d = 0; d < 3; ++d) {
        double acc = 0.0;
        for (uint32_t t = 0; t < s->n; ++t)
            acc += min_image(s->pos[3 * (base + t) + d] - s->pos[3 * base + d], s->L);
        c[d] = s->pos[3 * base + d] + acc / (double)s->n;
    }
}

static void orientation(const fx_system* s, uint32_t m, int k, double u[3])
{
    /* unit vector from the centre of mass to atom k of the molecule */
    double c[3], nrm = 0.0;
    centre(s, m, c);
    for (int d = 0; d < 3; ++d) {
        u[d] = min_image(s->pos[3 * (s->n * m + (uint32_t)k) + d] - c[d], s->L);
        nrm += u[d] * u[d];
    }
    nrm = sqrt(nrm);
    for (int d = 0; d < 3; ++d) u[d] /= nrm;
}

void fx_orientation_ref(const fx_system* s, double* u0, uint8_t* kref)
{
    for (uint32_t m = 0; m < s->p.n_molecules; ++m) {
        int k = 0;
        for (uint32_t t = 0; t < s->n; ++t)
            if (s->type[s->n * m + t] == 1) k = (int)t;
        kref[m] = (uint8_t)k;
        orientation(s, m, k, &u0[3 * m]);
    }
}

void fx_c2_terms(const fx_system* s, const double* u0, const uint8_t* kref, double* c2i)
{
    for (uint32_t m = 0; m < s->p.n_molecules; ++m) {
        double u[3];
        orientation(s, m, kref[m], u);
        double dot = u[0] * u0[3 * m] + u[1] * u0[3 * m + 1] + u[2] * u0[3 * m + 2];
        c2i[m] = 0.5 * (3.0 * dot * dot - 1.0);
    }
}

void fx_unwrapped(const fx_system* s, double* atoms, double* centres)
{
    for (uint32_t i = 0; i < s->N; ++i)
        for (int d = 0; d < 3; ++d)
            atoms[3 * i + d] = s->pos[3 * i + d] + s->L * (double)s->img[3 * i + d];
    for (uint32_t m = 0; m < s->p.n_molecules; ++m) {
        uint32_t base = s->n * m;
        for (int d = 0; d < 3; ++d) {
            double acc = 0.0;
            for (uint32_t t = 0; t < s->n; ++t)
                acc += min_image(s->pos[3 * (base + t) + d] - s->pos[3 * base + d], s->L);
            centres[3 * m + d] = atoms[3 * base + d] + acc / (double)s->n;
        }
    }
}
