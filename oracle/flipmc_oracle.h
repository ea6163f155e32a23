/*
 * flipmc_oracle.h -- serial FP64 reference implementation of flip Monte Carlo
 * for rigid three-site A/B/C molecules (Simon, Barrat & Berthier, "Molecular
 * motion at the experimental glass transition", Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the oracle that the GPU path is
 * checked against.  Only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg may load it.  It shares no code, header, table or helper
 * with the HIP library in paper_2506_21290_amd/.
 *
 * Everything is plain, slow and serial on purpose: every energy sum loops over
 * all other molecules and all their sites, site positions are r = c + R(q) b
 * refreshed whenever a molecule changes, and there is no blocking or
 * reordering beyond what the method states.
 */
#ifndef FLIPMC_ORACLE_H
#define FLIPMC_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Move kinds. */
enum { OR_TRANSLATE = 0, OR_ROTATE = 1, OR_FLIP = 2 };

typedef struct {
    uint32_t n_molecules;    /* M */
    double   density;        /* sites per unit volume (Sec. II.A: rho = N/V = 1.2) */
    double   temperature;    /* T, k_B = 1 */
    double   sigma[3];       /* diameters of A, B, C (Sec. II.A: 0.9, 1.0, 1.1) */
    double   bond_length;    /* side of the rigid equilateral triangle; <= 0 selects b* */
    double   p_flip;         /* Sec. II.B: 0.2 */
    double   p_translate;    /* translation share; rotation gets 1 - p_flip - p_translate */
    double   max_displacement;
    double   max_rotation;
    uint64_t seed;
    uint32_t colours_per_axis;  /* k of the checkerboard */
    uint32_t cells_per_side;    /* n_c */
} or_params;

/* One attempted move, as the oracle saw it. */
typedef struct {
    double   delta_e;   /* E_m(new) - E_m(old) over the moved sites */
    double   scale;     /* E_m(new) + E_m(old): the condition scale S_m   */
    double   t_log_u;   /* T * ln(u_acc)                                   */
    uint64_t sweep;
    uint32_t molecule;
    uint32_t slot;      /* RNG slot of the trial                           */
    uint8_t  move;      /* OR_TRANSLATE / OR_ROTATE / OR_FLIP              */
    uint8_t  accepted;
    uint8_t  exited;    /* translation left the cell: rejected, no dE      */
    uint8_t  axis;      /* flip axis site a, 255 otherwise                 */
    uint32_t pair_terms;/* site-pair terms inside the cut-off (old + new)  */
    uint32_t seq;       /* position of the trial inside its sweep          */
    uint32_t pad;
} or_record;

typedef struct or_system or_system;

/* ---- building blocks ---------------------------------------------------- */
void   or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_u32(uint32_t w);                    /* (w + 1/2) 2^-32, in (0,1)   */
double or_u53(uint32_t lo, uint32_t hi);      /* in (0,1]                    */
double or_u53_left(uint32_t lo, uint32_t hi); /* in [0,1)                    */
double or_bond_length_star(void);             /* argmin of WCA + FENE at sigma_ij = 1 */
double or_wca(double r2, double sigma_ij);    /* Eq. (1), zero beyond 2^(1/6) sigma_ij */
double or_fene(double r, double sigma_ij);    /* Eq. (2)                       */
double or_box_length(uint32_t n_molecules, double density);
double or_stencil_reach(const double sigma[3], double bond_length); /* W = max cut-off + 2 R */
void   or_rotation_matrix(const double q[4], double r[9]);
void   or_body_frame(double bond_length, double b[9]);  /* rows: site 0, 1, 2 */

/* ---- system ------------------------------------------------------------- */
/* Returns NULL and fills err (if non-NULL, 256 bytes) on invalid parameters. */
or_system* or_create(const or_params* p, char* err);
void       or_destroy(or_system* s);
int        or_init_lattice(or_system* s);
int        or_set_state(or_system* s, const double* com, const double* quat,
                        const uint8_t* types, uint64_t sweep, double e_acc);
void       or_get_state(const or_system* s, double* com, double* quat, uint8_t* types,
                        uint64_t* sweep, double* e_acc);
double     or_box(const or_system* s);
double     or_cell_width(const or_system* s);
void       or_sites(const or_system* s, double* xyz /* 9 M: molecule-major, site, axis */);

double or_energy(const or_system* s);     /* brute-force O(M^2) inter-molecular energy */
double or_energy_intra(const or_system* s); /* constant intramolecular WCA + FENE, total */

/* Sweeps.  log may be NULL; otherwise it must hold M records per sweep.
 * cell_order_seed != 0 visits the cells of each colour in a pseudo-random
 * order (used to show the order does not matter).                         */
int or_sweep_checkerboard(or_system* s, uint64_t n_sweeps, or_record* log,
                          uint64_t cell_order_seed);
int or_sweep_random(or_system* s, uint64_t n_sweeps, or_record* log);

/* Cell of a COM position for the shift of sweep `sweep` (linear index). */
int  or_cell_of(const or_system* s, const double c[3], uint64_t sweep);
void or_shift(const or_system* s, uint64_t sweep, double h[3]);

/* Counters: attempts[3], accepts[3], exits, pair_terms. */
void or_counters(const or_system* s, uint64_t attempts[3], uint64_t accepts[3],
                 uint64_t* exits, uint64_t* pair_terms);

/* Observables (Sec. III, Eq. 3 and Eq. 7). */
int  or_gofr_bins(double box, double dr, double* r_max);
void or_gofr_accumulate(const or_system* s, double dr, int nbins,
                        uint64_t* counts_all, uint64_t* counts_inter);
/* u0: 3 M reference orientation unit vectors and kref: M site indices, both
 * filled by or_orientation_ref from the current state (Sec. III.B, Eq. 7). */
void   or_orientation_ref(const or_system* s, double* u0, uint8_t* kref);
double or_c2(const or_system* s, const double* u0, const uint8_t* kref);
/* Per-molecule contributions C_2^i = P_2(u_i(t) . u_i(0)) (Sec. V.A), M values. */
void   or_c2_terms(const or_system* s, const double* u0, const uint8_t* kref, double* c2i);

/* Unwrapped positions for F_s(q, t) and F_s^cm(q, t) (Sec. III.B, Eqs. 5 and
 * 6): com (3 M) = wrapped centre + L * images crossed by accepted
 * translations since the last or_init_lattice / or_set_state; site (9 M) =
 * that centre + R(q) b_k for site index k.  Either pointer may be NULL. */
void   or_unwrapped(const or_system* s, double* com, double* site);

#ifdef __cplusplus
}
#endif
#endif
