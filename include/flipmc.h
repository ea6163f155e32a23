/*
 * flipmc.h -- C ABI of the MI355X (gfx950) flip Monte Carlo engine.
 *
 * The engine samples the NVT ensemble of M identical rigid triangular
 * molecules with sites A, B, C (diameters 0.9, 1.0, 1.1) interacting through
 * the site-site WCA potential (Simon, Barrat & Berthier, Sec. II.A, Eq. 1) in
 * a cubic periodic box at site density 1.2, with Metropolis sweeps that mix
 * whole-molecule translations, rotations and the intramolecular "flip" move
 * of Sec. II.B (exchange the types of two sites of one molecule).
 *
 * Conventions for every call:
 *   - Return value: MC_OK (0) or a negative MC_E* code; mc_last_error() then
 *     returns a thread-local message.  No call aborts or throws.
 *   - Device memory and streams are owned by the caller: mc_init_system()
 *     carves a system out of one caller-provided device buffer of at least
 *     mc_required_bytes() bytes, mc_batch_create() its slot tables out of one
 *     of at least mc_batch_required_bytes(); each buffer must outlive its
 *     system or batch.  The library owns only the opaque handles, small host
 *     mirrors, the pinned host staging of a batch's slot tables and HIP
 *     events; it never allocates device memory and never creates a stream.
 *   - All GPU work of a system is enqueued on the HIP stream given at
 *     mc_init_system() (NULL = the null stream).  mc_sweep() and
 *     mc_batch_run() only enqueue; calls that return host data (mc_energy,
 *     mc_observables, mc_get_state, mc_samples) synchronise that stream.
 *   - Host arrays are plain C arrays in the layouts stated per call; device
 *     pointers are marked as such.
 */
#ifndef FLIPMC_H
#define FLIPMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    MC_OK = 0,
    MC_EINVAL = -1,      /* invalid argument or parameter                      */
    MC_ENOMEM = -2,      /* buffer too small or host allocation failed         */
    MC_EDEVICE = -3,     /* a HIP runtime call failed                          */
    MC_EGEOM = -4,       /* cell decomposition does not fit the box            */
    MC_ENONFINITE = -5,  /* total energy is not finite (overlapping sites)     */
    MC_EBUSY = -6,       /* batch has no free slot                             */
    MC_ENOTIMPL = -7     /* combination not supported                          */
};

/* Precision of the pair-energy differences.  The state (centres of mass,
 * quaternions), the proposals, the acceptance test, the accumulated energy
 * and the periodic total-energy re-sum are always FP64. */
enum { MC_FP64 = 0, MC_FP32_DE = 1 };

enum { MC_TRANSLATE = 0, MC_ROTATE = 1, MC_FLIP = 2 };

/* mc_params.flags: MC_FLAG_HBM_STATE keeps the working arrays in HBM even
 * when the system would fit in one workgroup's LDS; MC_FLAG_SINGLE_WORKGROUP
 * runs a system on one workgroup (as inside a batch) instead of the
 * multi-workgroup engine. */
enum { MC_FLAG_HBM_STATE = 1, MC_FLAG_SINGLE_WORKGROUP = 2 };

/* mcf_params.flags only: MC_FLAG_SERIAL_CELLS attempts the cells of a colour
 * one at a time even when they cannot interact (the same chain, slower; for
 * checking the side-by-side execution). */
enum { MC_FLAG_SERIAL_CELLS = 4 };

/* Engines (mc_engine): one workgroup with the state in LDS, one workgroup
 * with the state in HBM, many workgroups in one cooperative launch with the
 * state in HBM and each cell's neighbourhood staged in LDS. */
enum { MC_ENGINE_LDS = 0, MC_ENGINE_HBM = 1, MC_ENGINE_SPREAD = 2 };

#define MC_GOFR_MAX_BINS 256
#define MC_C2_MAX 32

/* Parameters of one system: the model of Sec. II.A (three atom sizes, the WCA
 * potential of Eq. 1 between sites of different molecules, number density
 * N / V in a cubic periodic box) and the flip MC of Sec. II.B (flip
 * probability, step sizes, NVT at temperature T).  mc_params_default() fills
 * the paper's values (sigma = 0.9 / 1.0 / 1.1, density 1.2, p_flip = 0.2). */
typedef struct {
    uint32_t n_molecules;      /* M (>= 1, <= 65535)                                 */
    uint32_t precision;        /* MC_FP64 or MC_FP32_DE                              */
    double   density;          /* sites per unit volume, N / V with N = 3 M          */
    double   temperature;      /* T > 0, k_B = 1                                     */
    double   sigma[3];         /* diameters of types A, B, C                         */
    double   bond_length;      /* side of the rigid equilateral triangle; <= 0 picks
                                  b*, the minimum of WCA + FENE (Eq. 1 + Eq. 2) of a
                                  sigma_ij = 1 bond                                   */
    double   p_flip;           /* probability that a trial is a flip                 */
    double   p_translate;      /* probability of a translation; rotations get the rest */
    double   max_displacement; /* translation: uniform in [-d, d) per component      */
    double   max_rotation;     /* rotation: angle uniform in [-theta, theta), axis
                                  uniform on the sphere                               */
    uint64_t seed;             /* Philox4x32-10 key                                  */
    uint32_t colours_per_axis; /* k of the checkerboard (>= 2); 0 = choose           */
    uint32_t cells_per_side;   /* n_c, multiple of k, (k-1) L / n_c >= W; 0 = choose  */
    uint32_t resum_interval;   /* sweeps between FP64 re-sums of E (0 = never); each
                                  records the window's drift e_acc - E and then resets
                                  e_acc to the re-summed E                           */
    uint32_t obs_interval;     /* sweeps between E/M samples (0 = never)             */
    uint32_t gofr_interval;    /* sweeps between g(r) frames (0 = never)             */
    uint32_t obs_start;        /* samples are taken from this sweep on (relative to
                                  the observable origin, see mc_reset_observables)    */
    uint32_t max_samples;      /* capacity of the E/M and drift sample arrays        */
    uint32_t flags;            /* MC_FLAG_* bits                                     */
    double   gofr_dr;          /* g(r) bin width; r_max = min(L/2, 5)                */
    uint32_t barrier_polls;    /* multi-workgroup engine: polls a workgroup waits at
                                  a barrier of its system before it gives up and the
                                  system is marked faulted (reads then return
                                  MC_EDEVICE); 0 = default (about 2^23, seconds)       */
    uint32_t workgroups;       /* workgroups of mc_sweep's launches: 0 = the engine's
                                  cost model; 1 = one workgroup (as
                                  MC_FLAG_SINGLE_WORKGROUP); n >= 2 = the
                                  multi-workgroup engine on min(n, cells of a colour
                                  / 4 rounded up, device limit) workgroups, also the
                                  most a batch gives the system.  Every choice gives
                                  bitwise the same chain (an autotuner's knob)       */
    double   fs_q;             /* |q| of F_s(q, t) over the sites (Sec. III.B: 7.4,
                                  the first peak of the structure factor)             */
    double   fs_q_cm;          /* |q| of F_s^cm(q, t) over the centres (5.1)         */
} mc_params;

typedef struct mc_system mc_system;
typedef struct mc_batch mc_batch;

/* One attempted move of Sec. II.B (trial, Metropolis test), written by the
 * device when a decision log is enabled (mc_decision_log). */
typedef struct {
    double   delta_e;    /* E_m(new) - E_m(old) over the moved sites, as computed  */
    double   scale;      /* E_m(new) + E_m(old) over the moved sites               */
    double   t_log_u;    /* T ln(u_acc) of the Metropolis test                     */
    uint64_t sweep;
    uint32_t molecule;
    uint8_t  move;       /* MC_TRANSLATE / MC_ROTATE / MC_FLIP                     */
    uint8_t  accepted;
    uint8_t  exited;     /* translation left the molecule's cell: rejected        */
    uint8_t  axis;       /* flip axis site, 255 for other moves                    */
    uint32_t pair_terms; /* site-pair terms inside the cut-off, old + new          */
    uint32_t pad;
} mc_move_record;        /* 48 bytes */

/* Host-side snapshot of a system's accumulators (mc_observables). */
typedef struct {
    uint64_t sweep;              /* sweeps done since mc_init_system              */
    uint64_t attempts[3];        /* per move kind                                  */
    uint64_t accepts[3];
    uint64_t exits;              /* translations rejected for leaving their cell   */
    uint64_t pair_terms;         /* interacting site-pair terms evaluated          */
    uint64_t pair_tests;         /* candidate site-pair distance tests             */
    uint64_t near_overflows;     /* cells whose list of nearby molecules overflowed
                                    (then every stencil molecule is a candidate)  */
    double   e_acc;              /* E_0 + sum of accepted dE (FP64)                */
    double   e_resum;            /* last FP64 re-sum                               */
    double   drift;              /* e_acc - e_resum at the last re-sum: the error
                                    accumulated since the previous re-sum          */
    double   max_abs_drift;      /* over all re-sums except the first window       */
    uint64_t resum_sweep;        /* sweep of the last re-sum                        */
    uint32_t n_energy_samples;
    uint32_t n_drift_samples;
    double   energy_sum;         /* sum of E/M samples                             */
    double   energy_sumsq;
    uint32_t n_gofr_frames;
    uint32_t gofr_nbins;
    double   gofr_dr;
    double   gofr_rmax;
    uint64_t gofr_all[MC_GOFR_MAX_BINS];   /* ordered site pairs, all              */
    uint64_t gofr_inter[MC_GOFR_MAX_BINS]; /* ordered site pairs of distinct molecules */
    uint32_t n_c2;
    uint32_t pad;
    uint64_t c2_sweep[MC_C2_MAX];          /* sweeps after the observable origin   */
    double   c2[MC_C2_MAX];                /* C_2(t) (Sec. III.B, Eq. 7, l = 2)    */
    double   fs[MC_C2_MAX];                /* F_s(q, t) of the sites at the same sweeps
                                              (Sec. III.B, Eq. 5; averaged over all
                                              directions of q: mean of sin(q d)/(q d)
                                              over the site displacements d since the
                                              observable origin, centres unwrapped)   */
    double   fs_cm[MC_C2_MAX];             /* F_s^cm(q, t) of the centres (Eq. 6)     */
    /* Moments of the per-particle contributions (Sec. V.A) at the same sweeps,
     * from which the self parts of the four-point susceptibilities (Sec. V.B,
     * chi_4^self = mean of squares - square of the mean) and the Pearson
     * coefficient of Eq. 13 follow.  C_2^i = P_2(u_i(t).u_i(0)); F_s^cm,i and
     * F_s^i are the direction-averaged sin(q d)/(q d) of one centre or site. */
    double   c2_sq[MC_C2_MAX];             /* mean over molecules of (C_2^i)^2        */
    double   fs_cm_sq[MC_C2_MAX];          /* mean over molecules of (F_s^cm,i)^2     */
    double   c2_fs_cm[MC_C2_MAX];          /* mean over molecules of C_2^i F_s^cm,i   */
    double   fs_sq[MC_C2_MAX];             /* mean over sites of (F_s^i)^2            */
    /* Eq. (3) normalised: counts / (frames N rho (4 pi / 3)(r_{b+1}^3 - r_b^3)),
     * N = 3 M, rho = N / L^3; bin b covers [b dr, (b + 1) dr).  0 without frames. */
    double   gofr_norm_all[MC_GOFR_MAX_BINS];
    double   gofr_norm_inter[MC_GOFR_MAX_BINS];
} mc_obs;

/* ---- single system ------------------------------------------------------ */

/* Fill *p with the paper's model values (Sec. II.A sizes and density,
 * Sec. II.B p_flip) and this engine's defaults (move mixture 0.2 flip / 0.4
 * translation / 0.4 rotation, steps 0.1 and 0.2 rad, re-sum every 100 sweeps,
 * F_s at q = 7.4 and 5.1 as in Sec. III.B).  Never fails. */
void mc_params_default(mc_params* p);

/* Box side L = (3 M / density)^(1/3) (Sec. II.A: rho = N / V, N = 3 M) and
 * the checkerboard decomposition (k, n_c) the engine will use (after "choose"
 * defaults).  MC_EGEOM when the box is below 2 (W + 2 d_max), W the reach of
 * a molecule (largest cut-off + 2 circumradii), or when (k - 1) L / n_c < W.
 * Any output may be NULL. */
int mc_geometry(const mc_params* p, double* box, uint32_t* colours_per_axis,
                uint32_t* cells_per_side);

/* Where a system with these parameters keeps its working arrays: *resident = 1
 * when they fit in one workgroup's LDS (then *lds_bytes of dynamic LDS per
 * launch), 0 when they stay in HBM.  Either output may be NULL. */
int mc_placement(const mc_params* p, int* resident, size_t* lds_bytes);

/* The engine mc_sweep uses for a system with these parameters (MC_ENGINE_*)
 * and, for MC_ENGINE_SPREAD, the number of workgroups of its launches
 * (*workgroups = 1 otherwise).  A system beyond one workgroup's LDS runs on
 * the multi-workgroup engine; one within it runs there too when a wave per
 * cell of a colour gives it enough workgroups to be modelled 25 % faster
 * (FP32 systems of 1114 - 1728 molecules with k = 2, n_c = 6), else on its
 * LDS workgroup.  Inside a batch the engine is chosen per run (see
 * mc_batch_run).  Either output may be NULL. */
int mc_engine(const mc_params* p, int* engine, uint32_t* workgroups);

/* Bytes of device memory mc_init_system needs for these parameters (state of
 * Sec. II.A's M molecules, observable accumulators of Sec. III and the
 * engine's work arrays, 256-byte aligned regions).  Host only. */
int mc_required_bytes(const mc_params* p, size_t* bytes);

/* Create a system of the model of Sec. II.A (M molecules, density, box) in
 * device_buf (caller-owned, 256-byte aligned, >= mc_required_bytes, must
 * outlive the system).  With com, quat and types all NULL the start is the
 * seeded simple-cubic lattice (M = n^3, random uniform orientations, types
 * A, B, C on sites 0, 1, 2); otherwise they are host arrays com[3M] (xyz per
 * molecule), quat[4M] (w, x, y, z, unit) and types[3M] (0 = A, 1 = B,
 * 2 = C, a permutation per molecule), copied at once.  Computes E_0 (Eq. 1
 * summed over site pairs of distinct molecules) by an FP64 re-sum; fails with
 * MC_ENONFINITE if it is not finite, MC_ENOMEM if the buffer is too small,
 * MC_EINVAL for a bad argument.  hip_stream is a hipStream_t (NULL = null
 * stream).  Synchronises the stream before returning. */
int mc_init_system(const mc_params* p, const double* com, const double* quat,
                   const uint8_t* types, void* device_buf, size_t buf_bytes,
                   void* hip_stream, mc_system** out);

/* Enqueue n Monte Carlo timesteps (Sec. II.B: a timestep is N attempted
 * moves; here each of the M molecules is attempted once per sweep, in the
 * checkerboard order).  Asynchronous on the system's stream; MC_EBUSY inside
 * a batch. */
int mc_sweep(mc_system* s, uint64_t n_sweeps);

/* FP64 total energy now (Eq. 1 over site pairs of distinct molecules, a fresh
 * re-sum), E/M, and the drift e_acc - e_total of the accumulated energy.
 * Synchronises.  Any output pointer may be NULL.  MC_ENONFINITE if E is not
 * finite, MC_EBUSY inside a batch. */
int mc_energy(mc_system* s, double* e_total, double* e_per_molecule, double* drift);

/* Copy the accumulators to *out (host): move counters, E/M moments, g(r) of
 * Eq. 3 as counts and normalised, C_2 of Eq. 7 and F_s, F_s^cm of Eqs. 5-6
 * with their per-particle moments (Sec. V).  Synchronises (the batch's
 * stream first inside a batch). */
int mc_observables(mc_system* s, mc_obs* out);

/* Copy up to cap E/M samples and drift samples to host arrays (NULL to skip
 * either); *n_energy / *n_drift get the counts copied.  Synchronises. */
int mc_samples(mc_system* s, double* energy, double* drift, size_t cap, size_t* n_energy,
               size_t* n_drift);

/* Clear the observable accumulators and take the current state as the time
 * origin of C_2 (Eq. 7) and F_s (Eqs. 5-6): the reference orientation and
 * unwrapped positions.  Asynchronous; MC_EBUSY inside a batch. */
int mc_reset_observables(mc_system* s);

/* Read / overwrite the state of Sec. II.A (host arrays in the layouts of
 * mc_init_system; any output pointer may be NULL).  Both synchronise.  mc_set_state also sets the sweep counter
 * (which keys the random numbers) and the accumulated energy; e_acc NaN means
 * "re-sum it".  It also clears the periodic-image counts that unwrap the
 * centres for F_s, so F_s needs a new origin (mc_reset_observables) after it. */
int mc_get_state(mc_system* s, double* com, double* quat, uint8_t* types, uint64_t* sweep,
                 double* e_acc);
int mc_set_state(mc_system* s, const double* com, const double* quat, const uint8_t* types,
                 uint64_t sweep, double e_acc);

/* Record every attempted move (Sec. II.B trial and Metropolis decision) of
 * the next sweeps into a caller-owned DEVICE array of capacity records:
 * record (sweep - first_sweep) * M + molecule.  Sweeps beyond capacity / M
 * are not recorded.  records = NULL disables.  Stays in force when the system
 * joins a batch; MC_EBUSY when called inside one. */
int mc_decision_log(mc_system* s, void* device_records, size_t capacity);

/* Measurement (not part of the method): time every launch of the sweep kernel
 * and of the event kernel of this system with HIP events recorded on its
 * stream (enable = 0 stops and clears).  The events are the library's. */
int mc_timing_enable(mc_system* s, int enable);

/* Sum of the recorded launch durations (ms) and launch counts.  Synchronises.
 * Any output pointer may be NULL. */
int mc_timing_read(mc_system* s, double* sweep_ms, uint64_t* sweep_launches, double* event_ms,
                   uint64_t* event_launches);

/* Release a system's handle after waiting for its stream (and its batch's
 * streams when it is in one); its device buffer is the caller's to free
 * afterwards.  NULL is ignored. */
void mc_destroy(mc_system* s);
/* Message of the last failing call of this thread (never NULL). */
const char* mc_last_error(void);

/* ---- flexible molecules: the paper's own model and other bodies ----------- */

/* The paper's molecule is not rigid (Sec. II.A): atoms A, B, C of diameters
 * 0.9, 1, 1.1 joined by FENE bonds (Eq. 2) that cannot reach 1.5 sigma_ij,
 * with the WCA potential of Eq. 1 between every pair of atoms, those of one
 * molecule included.  Its outlook (Sec. VII) names squares and tetrahedra as
 * further bodies for intramolecular swap moves; they are the same model with
 * four atoms: a ring of four bonds, or all six pairs bonded, and four types of
 * diameters evenly spaced over [0.9, 1.1].
 *
 * Monte Carlo (Sec. II.B): a timestep is N = n M attempts, here every atom
 * once per sweep in a checkerboard over atom cells (a random shift of the
 * grid per sweep, colours in order, ascending atom index in a cell).  An
 * attempt is a flip of the atom's molecule with probability p_flip -- a
 * permutation of its types at fixed positions, uniform over the 180 degree
 * rotations of the ideal body (triangle: the median through atom q; square:
 * the diagonal through atom 0, the one through atom 1, the bisector of edge
 * 01, the bisector of edge 12; tetrahedron: the axes through the midpoints of
 * edges 01, 02, 03) -- otherwise a translation of the atom, uniform in
 * [-d, d)^3 and rejected when it leaves the atom's cell.  A bond reaching
 * 1.5 sigma_ij has infinite energy: such a move is rejected.  All arithmetic
 * is FP64.  The energy and E/M include the intramolecular terms. */
enum { MC_TRIANGLE = 0, MC_SQUARE = 1, MC_TETRAHEDRON = 2 };

typedef struct {
    uint32_t geometry;         /* MC_TRIANGLE, MC_SQUARE or MC_TETRAHEDRON          */
    uint32_t n_molecules;      /* M; the lattice start needs M = n^3               */
    double   density;          /* atoms per unit volume, N / V, N = n M            */
    double   temperature;      /* T > 0                                            */
    double   sigma[4];         /* diameter of each type (3 used by triangles)      */
    double   bond_length;      /* side of the ideal body at the lattice start;
                                  <= 0 picks b*, the minimum of WCA + FENE of a
                                  sigma_ij = 1 bond                                 */
    double   p_flip;           /* probability that an attempt is a flip           */
    double   max_displacement; /* translation: uniform in [-d, d) per component   */
    uint64_t seed;             /* Philox4x32-10 key                                */
    uint32_t colours_per_axis; /* k (>= 2); 0 = choose                             */
    uint32_t cells_per_side;   /* n_c, multiple of k; 0 = choose                   */
    uint32_t resum_interval;   /* sweeps between FP64 re-sums (0 = never)          */
    uint32_t obs_interval;     /* sweeps between E/M samples (0 = never)           */
    uint32_t gofr_interval;    /* sweeps between g(r) frames (0 = never)           */
    uint32_t obs_start;        /* samples from this sweep after the origin on      */
    uint32_t max_samples;      /* capacity of the E/M and drift sample arrays      */
    uint32_t flags;            /* MC_FLAG_HBM_STATE: positions, types and cell
                                  lists stay in the buffer even when they fit one
                                  workgroup's LDS (same results, slower)           */
    double   gofr_dr;          /* g(r) bin width; r_max = min(L/2, 5)              */
    double   fs_q;             /* |q| of F_s over the atoms (Sec. III.B: 7.4)      */
    double   fs_q_cm;          /* |q| of F_s^cm over the centres of mass (5.1)     */
} mcf_params;

typedef struct mcf_system mcf_system;

/* Fill *p with the paper's values for `geometry` (Sec. II.A sizes and
 * density 1.2, Sec. II.B p_flip = 0.2) and this engine's defaults (step 0.1,
 * re-sum every 100 sweeps).  Never fails. */
void mcf_params_default(mcf_params* p, uint32_t geometry);

/* Box side L = (n M / density)^(1/3) and the decomposition (k, n_c, n_c a
 * multiple of k >= 2): cells at least r_c + 2 sqrt(3) d wide (r_c the largest
 * WCA cut-off, d the largest displacement per axis).  The cells of a colour
 * are attempted in ascending index; they run side by side when their gap
 * (k - 1) L / n_c is at least 2 D + r_c for the largest atom distance D any
 * body can have (one bond of 1.5 sigma_ij, two for the square's diagonal), or
 * at least 2 D + r_c + 4 sqrt(3) d for D measured over the molecules with an
 * atom in them when the colour starts; otherwise one at a time.  The chain
 * does not depend on it.  With k = n_c = 0 the choice is the most cells per
 * colour that run side by side while the bodies stay within 15 % of their
 * ideal size.  MC_EGEOM when no decomposition fits or the box is below
 * 2 (max(D, r_c) + 2 d), D the largest possible.  Any output may be NULL. */
int mcf_geometry(const mcf_params* p, double* box, uint32_t* colours_per_axis,
                 uint32_t* cells_per_side);

/* Where the sweep kernel keeps positions, types and cell lists for these
 * parameters: *resident = 1 when they fit in one workgroup's LDS on the
 * current device (then *lds_bytes of dynamic LDS per launch, loaded at the
 * start of a launch and written back at its end), 0 when it works on them in
 * the system's buffer (MC_FLAG_HBM_STATE in flags forces that).  Either
 * output may be NULL.  Host only. */
int mcf_placement(const mcf_params* p, int* resident, size_t* lds_bytes);

/* Bytes of device memory mcf_init_system needs.  Host only. */
int mcf_required_bytes(const mcf_params* p, size_t* bytes);

/* Create a system in device_buf (caller-owned, 256-byte aligned,
 * >= mcf_required_bytes, must outlive the system).  pos and types NULL: the
 * seeded lattice start (ideal bodies of side bond_length at simple-cubic
 * sites, uniformly random orientations, types 0, 1, ... on atoms 0, 1, ...);
 * otherwise host arrays pos[3 N] (xyz of atom n m + s) and types[N] (a
 * permutation of 0 .. n-1 per molecule).  MC_ENONFINITE when a bond is
 * stretched to its limit or atoms coincide; synchronises the stream. */
int mcf_init_system(const mcf_params* p, const double* pos, const uint8_t* types, void* device_buf,
                    size_t buf_bytes, void* hip_stream, mcf_system** out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid it): mcf_init_system without any
 * allocation by the library.  The caller's device_state (256-byte aligned,
 * at least *state_bytes_needed bytes, must outlive the system) holds the
 * state and the observables; the work arrays of the sweeps and events (cell
 * lists, per-cell energies, partial sums) live in one static per-device array
 * of 4 MiB, so MC_ENOMEM when they would exceed it.  Clearing is done by a
 * kernel (no memset), host positions are staged through the state buffer, and
 * the handle comes from a static pool of 16 (MC_EBUSY when all are alive).
 * With device_state NULL the call only stores *state_bytes_needed (and the
 * scratch check) and returns.  Every allocation-free system of a device
 * shares that array: calls on such systems whose work overlaps in time (other
 * streams, other threads) race; one after another on one stream is safe, as
 * every launch rewrites what it reads.  mcf_sweep, mcf_energy,
 * mcf_observables, mcf_reset_observables, mcf_decision_log and mcf_destroy
 * allocate nothing either. */
int mcf_init_system_noalloc(const mcf_params* p, const double* pos, const uint8_t* types,
                            void* device_state, size_t state_bytes, size_t* state_bytes_needed,
                            void* hip_stream, mcf_system** out);

/* Enqueue n timesteps of N attempts (Sec. II.B).  Asynchronous. */
int mcf_sweep(mcf_system* s, uint64_t n_sweeps);

/* Enqueue n timesteps (Sec. II.B) of each of `count` distinct systems -- the
 * independent replicas over which the paper's averages (Sec. III) are taken --
 * one workgroup per system, up to 256 systems per launch, so that many
 * systems fill the device.  Each system's chain and observables are bitwise
 * those of mcf_sweep on it alone; systems may differ in size and parameters.
 * All must have been created on the same stream, where the launches go.
 * MC_EINVAL for an empty or NULL list, a NULL or repeated system, or systems
 * on different streams (nothing is enqueued then).  Asynchronous. */
int mcf_sweep_many(mcf_system* const* systems, uint32_t count, uint64_t n_sweeps);

/* FP64 total energy now (Eq. 1 over all atom pairs + Eq. 2 over the bonds, a
 * fresh re-sum), E/M and the drift e_acc - E.  Synchronises. */
int mcf_energy(mcf_system* s, double* e_total, double* e_per_molecule, double* drift);

/* Accumulators as in mc_observables: attempts / accepts of translations
 * (index MC_TRANSLATE) and flips (MC_FLIP), exits, pair terms, E/M moments,
 * g(r) over atoms (Eq. 3, counts and normalised), C_2 (Eq. 7, the vector from
 * the centre of mass to the atom that was of type B at the origin), F_s over
 * atoms and F_s^cm over centres of mass (Eqs. 5-6), and at the same sweeps the
 * per-particle moments of Sec. V.A: means over molecules of (C_2^i)^2,
 * (F_s^cm,i)^2 and C_2^i F_s^cm,i and over atoms of (F_s^i)^2.  Synchronises. */
int mcf_observables(mcf_system* s, mc_obs* out);


/* New observable origin (C_2 reference, unwrapped positions).  Asynchronous. */
int mcf_reset_observables(mcf_system* s);

/* Read / overwrite the state: host pos[3 N], types[N] as in mcf_init_system
 * (NULL outputs skipped), the sweep counter and the accumulated energy (NaN =
 * re-sum it).  Both synchronise. */
int mcf_get_state(mcf_system* s, double* pos, uint8_t* types, uint64_t* sweep, double* e_acc);
int mcf_set_state(mcf_system* s, const double* pos, const uint8_t* types, uint64_t sweep,
                  double e_acc);

/* Record every attempt of the next sweeps into a caller-owned DEVICE array of
 * mc_move_record (record (sweep - first) * N + atom; `molecule` holds the
 * atom, `axis` the flip's rotation, delta_e = +inf at a bond's limit). */
int mcf_decision_log(mcf_system* s, void* device_records, size_t capacity);

/* Wait for the system's stream and release its handle.  NULL is ignored. */
void mcf_destroy(mcf_system* s);

/* ---- analysis of independent runs ------------------------------------------ */

/* Time correlations of n independent runs of one system (same M, same sample
 * sweeps), formed from what mc_observables returns.  Per sample time t_j:
 *   c2, fs, fs_cm  the ensemble means of C_2 (Eq. 7), F_s (Eq. 5), F_s^cm (Eq. 6);
 *   chi4_*         Eq. 10: M (3 M for the sites' F_s) times the variance over
 *                  runs of the run's value;
 *   chi4s_*        Eq. 11: mean over runs and particles of C_i^2 minus the
 *                  square of the ensemble mean (the self part);
 *   rho            Eq. 13: (mean of C_2^i F_s^cm,i - C_2 F_s^cm) over the
 *                  square root of the product of the two self parts;
 * and the relaxation times of Sec. III.C: the first time each mean falls to
 * 1/e, linear in ln t between the two samples around the crossing (NaN when
 * it does not fall that far).  Host only; MC_EINVAL when the runs do not
 * share their sample sweeps. */
typedef struct {
    uint32_t n_times;
    uint32_t n_runs;
    uint64_t t[MC_C2_MAX];          /* sweeps after the observable origin        */
    double   c2[MC_C2_MAX], fs[MC_C2_MAX], fs_cm[MC_C2_MAX];
    double   chi4_c2[MC_C2_MAX], chi4_fs[MC_C2_MAX], chi4_fs_cm[MC_C2_MAX];
    double   chi4s_c2[MC_C2_MAX], chi4s_fs[MC_C2_MAX], chi4s_fs_cm[MC_C2_MAX];
    double   rho[MC_C2_MAX];
    double   tau_c2, tau_fs, tau_fs_cm;
} mc_dyn;

int mc_dynamics(const mc_obs* runs, size_t n_runs, uint32_t n_molecules, mc_dyn* out);

/* mc_dynamics for flexible systems (Sec. III.C, Sec. V): the ensemble means,
 * chi_4 (Eq. 10; the atoms' F_s counts atoms_per_molecule * M particles),
 * chi_4^self (Eq. 11), rho (Eq. 13) and the 1/e times of n independent runs,
 * formed from what mcf_observables returns.  MC_EINVAL as mc_dynamics, or
 * when atoms_per_molecule is not 3 or 4.  Host only. */
int mcf_dynamics(const mc_obs* runs, size_t n_runs, uint32_t n_molecules, uint32_t atoms_per_molecule,
                 mc_dyn* out);

/* ---- batches: many systems in one persistent launch ---------------------- */

/* The batched and served patterns of this engine (not from the paper, which
 * runs independent samples, Sec. III.B): many independent Markov chains of
 * the same model, each with its own size, temperature and sweep count, share
 * persistent launches.
 *
 * A batch holds up to max_slots systems of one precision.  Each
 * mc_batch_run gives every system one workgroup; the workgroups left over
 * (up to the batch's workgroup limit, one per compute unit by default) go to
 * the systems with the most remaining work that can use several (those
 * beyond one workgroup's LDS, and those within it when enough workgroups are
 * idle to make them modelled 25 % faster), which then run on the
 * multi-workgroup engine, each on up to the workgroups its cells allow.
 * Systems on one workgroup share one persistent launch per
 * placement class (state in LDS / in HBM; the HBM class beside the LDS
 * class on a third caller stream when mc_batch_set_hbm_stream gives one);
 * systems on the multi-workgroup engine share one cooperative launch on the
 * caller's second stream (hip_stream_aux of mc_batch_create).
 * All engines make the same decisions and sum the energy in the same order,
 * so a system gives bitwise the same results in a batch as alone, whichever
 * engines its runs used. */
/* Bytes of caller-owned device memory a batch of max_slots slots needs (its
 * double-buffered slot tables).  MC_EINVAL when max_slots is 0 or above
 * 65536. */
int mc_batch_required_bytes(uint32_t max_slots, size_t* bytes);

/* Create a batch whose slot tables live in device_buf (caller-owned, 256-byte
 * aligned, >= mc_batch_required_bytes(max_slots), must outlive the batch).
 * Systems on one workgroup run on hip_stream; the multi-workgroup launches
 * run on hip_stream_aux (a second caller stream, so both overlap) or, when it
 * is NULL, on hip_stream after them.  The batch keeps pinned host staging of
 * its slot tables and a few HIP events of its own.  MC_ENOMEM when the
 * buffer is too small. */
int mc_batch_create(uint32_t max_slots, uint32_t precision, void* device_buf, size_t buf_bytes,
                    void* hip_stream, void* hip_stream_aux, mc_batch** out);

/* Put an initialised system into a free slot with n_sweeps of work; the
 * system must use the batch's precision.  MC_EBUSY when no slot is free.
 * While in a batch the system is advanced on the batch's stream: mc_sweep,
 * mc_energy, mc_set_state, mc_reset_observables and mc_decision_log return
 * MC_EBUSY, and the reading calls first synchronise the batch's stream. */
int mc_batch_add(mc_batch* b, mc_system* s, uint64_t n_sweeps, uint32_t* slot);

/* Enqueue one run in which each occupied slot runs a time slice of its
 * remaining sweeps (0 = all remaining); with more occupied slots than the
 * batch's workgroup limit, a run takes the largest multiple of the limit of
 * them, in turn from run to run, so that no run ends with a partly filled
 * round of workgroups.  Every launch of the run is sized to
 * the time a 1000-molecule system (k = 2, n_c = 4) takes for
 * max_moves_per_slot moves on one workgroup: each system's slice is that time
 * over its modelled sweep time (one-workgroup cost model, divided by its
 * workgroups on the multi-workgroup engine), scaled per engine by the time
 * per modelled cycle measured on the batch's earlier launches; at least one
 * sweep.  Slices also stop at each system's re-sum / g(r) / C_2 sweeps, whose
 * work follows in a second launch.  *n_launched = number of sweep launches
 * enqueued (one per placement class in use, one for the multi-workgroup
 * engine). */
int mc_batch_run(mc_batch* b, uint64_t max_moves_per_slot, uint32_t* n_launched);

/* Put the launch of the systems that run on one workgroup with their state in
 * HBM on a third caller stream, beside the launch of those whose state is in
 * LDS (on hip_stream), instead of after it; the run's event work and all
 * later work on hip_stream follow both.  NULL (the default) or hip_stream
 * itself: after it on hip_stream.  The stream must outlive the batch.  Either
 * way the results are the same; only the overlap changes.  MC_EINVAL for a
 * NULL batch.  Host only. */
int mc_batch_set_hbm_stream(mc_batch* b, void* hip_stream);

/* At most max_workgroups workgroups of the batch's runs at once (0 = one per
 * compute unit of the current device, the default): fewer leaves compute units
 * to other work and moves fewer systems onto the multi-workgroup engine. */
int mc_batch_set_workgroups(mc_batch* b, uint32_t max_workgroups);

/* Synchronise, then report (and free) the slots whose work is complete:
 * their slot indices and systems. */
int mc_batch_poll(mc_batch* b, uint32_t* slots, mc_system** systems, size_t cap, size_t* n);

/* Remove a system from its slot before its work is done. */
int mc_batch_cancel(mc_batch* b, uint32_t slot);

/* Wait for the batch's streams and release its handle; its systems leave it
 * and stay valid.  NULL is ignored. */
void mc_batch_destroy(mc_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* FLIPMC_H */
