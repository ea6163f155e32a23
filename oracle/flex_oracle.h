/*
 * flex_oracle.h -- serial FP64 oracle of flip Monte Carlo for FLEXIBLE
 * molecules: the paper's own model (Simon, Barrat & Berthier, Sec. II.A:
 * three atoms A, B, C joined by FENE bonds, Eq. 2, with the WCA potential of
 * Eq. 1 between all atom pairs, intramolecular ones included) and the two
 * other geometries its outlook names (Sec. VII): squares and tetrahedra.
 *
 * TEST INFRASTRUCTURE ONLY, like flipmc_oracle.h: only tests/,
 * __graft_entry__.smoke() and bench.py's cpu_baseline leg may load it, and it
 * shares no code with the HIP library.
 *
 * Moves (Sec. II.B): each attempt picks one atom; with probability p_flip it
 * proposes a flip of the atom's molecule -- a permutation of the types of its
 * atoms at fixed positions, chosen uniformly among the 180 degree rotations
 * of the ideal body (triangle: the three medians; square: the two diagonals
 * and the two edge bisectors; tetrahedron: the three axes through midpoints
 * of opposite edges) -- otherwise a translation of that atom, uniform in
 * [-d, d) per component.  A Monte Carlo timestep is N = n M attempts.
 */
#ifndef FLEX_ORACLE_H
#define FLEX_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { FX_TRIANGLE = 0, FX_SQUARE = 1, FX_TETRAHEDRON = 2 };
enum { FX_TRANSLATE = 0, FX_FLIP = 2 };

typedef struct {
    uint32_t geometry;        /* FX_TRIANGLE, FX_SQUARE, FX_TETRAHEDRON            */
    uint32_t n_molecules;     /* M                                                */
    double   density;         /* atoms per unit volume, N / V, N = n M            */
    double   temperature;
    double   sigma[4];        /* diameter of each type; n types for n-atom bodies */
    double   bond_length;     /* side of the ideal body at the lattice start;
                                 <= 0 selects b*, the minimum of WCA + FENE of a
                                 sigma_ij = 1 bond                                 */
    double   p_flip;          /* Sec. II.B: 0.2                                   */
    double   max_displacement;
    uint64_t seed;
    uint32_t colours_per_axis;
    uint32_t cells_per_side;
} fx_params;

typedef struct {
    double   delta_e;   /* E(new) - E(old) of the terms the move changes; +inf
                           when a bond would stretch to 1.5 sigma_ij or beyond */
    double   scale;     /* E(new) + E(old) of those terms (+inf likewise)      */
    double   t_log_u;   /* T ln(u_acc)                                          */
    uint64_t sweep;
    uint32_t atom;      /* the atom the attempt picked                          */
    uint32_t slot;      /* RNG slot                                             */
    uint8_t  move;      /* FX_TRANSLATE or FX_FLIP                              */
    uint8_t  accepted;
    uint8_t  exited;    /* translation left the atom's cell (checkerboard)      */
    uint8_t  kind;      /* flip kind, 255 for translations                      */
    uint32_t pair_terms;/* pair terms inside their range (WCA cut-off, bonds), old + new */
    uint32_t seq;       /* position of the attempt inside its sweep            */
    uint32_t pad;
} fx_record;

typedef struct fx_system fx_system;

uint32_t   fx_sites(uint32_t geometry);                 /* n: 3, 4, 4 (0 if invalid) */
uint32_t   fx_flip_kinds(uint32_t geometry);            /* 3, 4, 3                   */
double     fx_box_length(uint32_t geometry, uint32_t n_molecules, double density);
/* Separation same-colour cells need: 2 D + r_c, D the largest distance
 * between two atoms of one molecule that its bonds allow, r_c the largest
 * WCA cut-off. */
double     fx_reach(const fx_params* p);

fx_system* fx_create(const fx_params* p, char* err);
void       fx_destroy(fx_system* s);
int        fx_init_lattice(fx_system* s);
/* pos: 3 N (xyz per atom, atom i = n m + s), types: N */
int        fx_set_state(fx_system* s, const double* pos, const uint8_t* types, uint64_t sweep,
                        double e_acc);
void       fx_get_state(const fx_system* s, double* pos, uint8_t* types, uint64_t* sweep,
                        double* e_acc);
double     fx_box(const fx_system* s);
double     fx_energy(const fx_system* s);          /* brute force: all WCA pairs + all bonds */
double     fx_energy_inter(const fx_system* s);    /* WCA between atoms of distinct molecules */
int        fx_sweep_checkerboard(fx_system* s, uint64_t n_sweeps, fx_record* log,
                                 uint64_t cell_order_seed);
int        fx_sweep_random(fx_system* s, uint64_t n_sweeps, fx_record* log);
void       fx_counters(const fx_system* s, uint64_t attempts[3], uint64_t accepts[3],
                       uint64_t* exits, uint64_t* pair_terms);
void       fx_gofr_accumulate(const fx_system* s, double dr, int nbins, uint64_t* counts_all,
                              uint64_t* counts_inter);
/* Sec. III.B: u0 (3 M) = unit vector from the centre of mass to the atom
 * of type B, kref (M) its index in the molecule; c2i (M) = P_2(u(t).u(0)). */
void       fx_orientation_ref(const fx_system* s, double* u0, uint8_t* kref);
void       fx_c2_terms(const fx_system* s, const double* u0, const uint8_t* kref, double* c2i);
/* Unwrapped atom positions (3 N) and centres of mass (3 M) for F_s. */
void       fx_unwrapped(const fx_system* s, double* atoms, double* centres);

#ifdef __cplusplus
}
#endif
#endif
