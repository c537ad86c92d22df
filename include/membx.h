/*
 * membx.h -- C-ABI of the MI355X (gfx950) force/energy engine for MC-MD and
 * MDAS sampling of coarse-grained (Martini-style) lipid bilayers.
 *
 * Method: Cherniavskyi, Fathizadeh, Elber, Tieleman, "Computer Simulations of
 * a Heterogeneous Membrane with Enhanced Sampling Techniques" (arXiv
 * 2005.08348).  The library evaluates the potential of the paper's Methods
 * section (Martini nonbonded terms: Lennard-Jones 12-6 with a potential-shift
 * modifier at the 1.1 nm cutoff and reaction-field electrostatics; Martini
 * bonds and angles), steps the dynamics, and runs the two exchange schemes of
 * the Theory section: MC-MD (single-step Metropolis exchange of two
 * molecules' identities, Eq. 1) and MDAS (an alchemical trajectory with
 * linear coupling, work by Eq. 2 and acceptance by Eq. 3).
 *
 * Conventions
 *   units: nm, ps, amu, kJ/mol, elementary charge, K.
 *   Every call returns an int32 status (MEMBX_OK = 0).  No exception or
 *   signal crosses the ABI.  On error membx_last_error() gives a message.
 *   Host buffers are owned by the caller; the library reads input buffers
 *   only during the call and writes output buffers only in query calls.
 *   Device memory: the library allocates NOTHING on the device.  All device
 *   state lives in a caller-provided arena (e.g. a torch uint8 tensor) of at
 *   least membx_sys_bytes() bytes, owned by the system handle until
 *   membx_sys_destroy().  The library creates one HIP stream of its own per
 *   handle (default priority) and orders it after / before the caller's
 *   stream with events, so calls are ordered with respect to the caller's
 *   stream.  Query calls (energies, state, forces, results) synchronize.
 *   A handle is not thread-safe; distinct handles are independent and their
 *   results do not depend on each other.
 */
#ifndef MEMBX_H
#define MEMBX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define MEMBX_OK               0
#define MEMBX_E_INVAL          1  /* bad descriptor or argument               */
#define MEMBX_E_NOMEM          2  /* arena too small                          */
#define MEMBX_E_DEVICE         3  /* HIP runtime error                        */
#define MEMBX_E_LIST_OVERFLOW  4  /* neighbour list or ghost capacity exceeded */
                                  /* (sticky: the handle's results are void;  */
                                  /* the message names the capacity needed)   */
#define MEMBX_E_NONFINITE      5  /* non-finite energy or input state         */
#define MEMBX_E_STATE          6  /* call not valid in the current state      */
#define MEMBX_E_SKIN           7  /* a bead moved more than skin/2 between    */
                                  /* list rebuilds (pairs may have been lost) */

/* ------------------------------------------------------------ precision */
#define MEMBX_FP64   0   /* float64 state, forces and energies                 */
#define MEMBX_MIXED  1   /* float32 state, pair forces and integration; float64 */
                         /* energy, exchange dU, MDAS work and Metropolis test  */

/* A molecule kind: its beads, bonded topology and exchange family.
 * Bonds are harmonic, V = k/2 (r - b0)^2; angles are the cosine-squared form
 * used by Martini, V = k/2 (cos(theta) - cos(theta0))^2 (paper, Methods:
 * Martini 2.2).  Beads joined by a bond do not interact through the
 * nonbonded terms.  Kinds of one swap family (swap_family >= 0) must have the
 * same bead count and masses; an exchange changes the potential parameters
 * of the two molecules, not their coordinates (paper, Theory).  Kinds of a
 * family that differ in their bonded terms make a topology-changing
 * exchange (at most 16 beads per molecule): a kind with fewer real beads
 * fills its slots with dummy beads (a type with no Lennard-Jones and no
 * charge, held by bonds), whose appearing and vanishing the soft-core path
 * of membx_set_mdas_path handles (paper, Eq. 4); a family molecule then
 * excludes from the nonbonded terms the pairs bonded in any kind of its
 * family, and its bonded terms follow its current kind (mixed linearly in
 * lambda along an MDAS trajectory).  swap_family < 0: never exchanged. */
typedef struct membx_kind {
    int32_t n_beads;
    const int32_t* bead_type;     /* [n_beads] in [0, n_types)            */
    const double*  bead_charge;   /* [n_beads] e                          */
    const double*  bead_mass;     /* [n_beads] amu, > 0                   */
    int32_t n_bonds;
    const int32_t* bond_ij;       /* [2 n_bonds] local bead indices        */
    const double*  bond_b0;       /* [n_bonds] nm                          */
    const double*  bond_k;        /* [n_bonds] kJ mol^-1 nm^-2             */
    int32_t n_angles;
    const int32_t* angle_ijk;     /* [3 n_angles], middle index = vertex   */
    const double*  angle_theta0;  /* [n_angles] degrees                    */
    const double*  angle_k;       /* [n_angles] kJ/mol                     */
    int32_t swap_family;
} membx_kind;

/* System descriptor (host memory, read only during membx_sys_bytes and
 * membx_sys_create).  Molecule m's beads are contiguous; bead ids run over
 * the molecules in order.  Positions should lie in [0, L) per axis (others
 * are wrapped in float64 first); MEMBX_MIXED rounds positions, velocities and
 * box lengths to float32. */
typedef struct membx_desc {
    int32_t n_kinds;
    const membx_kind* kinds;
    int32_t n_mols;
    const int32_t* mol_kind;      /* [n_mols]                               */
    const double* pos;            /* [3 N]                                  */
    const double* vel;            /* [3 N] or NULL (zero)                   */
    double box[3];                /* rectangular, periodic, >= 3 (r_cut+skin) */
    int32_t n_types;              /* <= 16                                  */
    const double* lj_epsilon;     /* [n_types^2] kJ/mol, symmetric          */
    const double* lj_sigma;       /* [n_types^2] nm, symmetric              */
    double r_cut;                 /* nonbonded cutoff (paper: 1.1 nm)       */
    double eps_r;                 /* relative permittivity (paper: 15)      */
    double eps_rf;                /* reaction-field permittivity; <= 0 or   */
                                  /* +inf means infinity                    */
    double dt;                    /* ps                                     */
    double temperature;           /* K                                      */
    double gamma;                 /* Langevin friction, 1/ps (0: NVE)       */
    uint64_t seed;                /* Philox key of every random stream      */
    int32_t precision;            /* MEMBX_FP64 or MEMBX_MIXED              */
    /* tuning; 0 selects a default */
    double  skin;                 /* Verlet buffer, nm (default 0.3)        */
    double  skin_max;             /* largest skin the arena is sized for;   */
                                  /* <= 0: 0.4 nm where the box allows it   */
                                  /* (box >= 3 (r_cut + skin_max)), else    */
                                  /* skin                                   */
    int32_t rebuild_interval;     /* steps between list rebuilds (def. 5)   */
    int32_t lanes_per_bead;       /* 1, 2, 4 or 8 (default 8)               */
    int32_t list_capacity;        /* neighbour slots per bead (default auto; */
                                  /* rounded up to a multiple of 8)         */
    int32_t max_trials;           /* largest exchange batch (default 256)   */
    int32_t max_pairs;            /* largest MDAS pair count (default 64)   */
    /* dynamic pruning: every prune_interval force passes of plain MD the
     * pass that walks the Verlet list also writes an inner list of the pairs
     * within r_cut + skin_inner, which the passes in between walk instead;
     * exact while no bead moves more than skin_inner/2 between prunes
     * (counted like the skin violations).  prune_interval <= 1: off. */
    double  skin_inner;           /* nm, <= skin (default skin / 2)         */
    int32_t prune_interval;
} membx_desc;

/* Energies of the current state (float64). */
typedef struct membx_energy {
    double lj, rf, bond, angle, kinetic, potential, total;
    int64_t n_pairs_in_cutoff;    /* non-excluded pairs with r < r_cut      */
    int64_t fe_count;             /* force evaluations so far (paper's cost */
                                  /* unit, Methods)                         */
    int64_t step, batch, cycle;   /* MD step, exchange batch, MDAS cycle    */
    int64_t n_rebuilds;
    int64_t n_skin_violations;    /* (bead, step) events beyond skin/2 since */
                                  /* creation or the last retune, plus those */
                                  /* beyond skin_inner/2 since a prune      */
    double  max_displacement;     /* largest displacement from the position */
                                  /* at the last list build seen since then */
                                  /* (nm)                                   */
    int64_t n_list_entries;       /* entries of the Verlet list (both       */
                                  /* directions): the pair slots one force  */
                                  /* pass computes                          */
    double  virial[3];            /* W_aa: sum over pairs, bonds and angles */
                                  /* of (separation)_a (force)_a, kJ/mol    */
    double  mv2[3];               /* sum m v_a^2, kJ/mol                    */
    double  pressure[3];          /* P_aa = (mv2 + virial) / V, bar: the    */
                                  /* pressure the paper's barostat couples  */
                                  /* to (Methods)                           */
    int64_t list_retests;         /* 1 if a list build since the list       */
                                  /* geometry last changed (creation,       */
                                  /* membx_set_tuning, a box rescale) had a */
                                  /* lane whose LDS hit buffer overflowed,  */
                                  /* so that it tested its candidates again */
                                  /* while writing: a slower path giving    */
                                  /* the same list; else 0                  */
} membx_energy;

/* One admitted exchange trial of a batch. */
typedef struct membx_trial {
    int32_t draw;                 /* candidate index within the batch       */
    int32_t mol_x, mol_y;         /* exchanged molecules                    */
    int32_t accepted;
    double  delta_u;              /* U(after) - U(before), kJ/mol           */
    double  u;                    /* the Metropolis uniform in [0, 1)       */
} membx_trial;

typedef struct membx_sys membx_sys;

/* Bytes of device memory a system needs (arena size for membx_sys_create).
 * Errors: E_INVAL for an invalid descriptor, among them systems whose beads
 * plus periodic-image capacity reach 2^27 slots (the force pass addresses a
 * slot's coordinates by a 32-bit byte offset). */
int32_t membx_sys_bytes(const membx_desc* desc, uint64_t* bytes);

/* Build a system in `dev_arena` (device pointer, 256-byte aligned, at least
 * membx_sys_bytes bytes) ordered after `hip_stream` (a hipStream_t, may be
 * NULL for the default stream).  Copies the descriptor, uploads the state,
 * builds the cell grid and neighbour list and evaluates the forces.
 * Errors: E_INVAL, E_NOMEM (arena too small), E_DEVICE. */
int32_t membx_sys_create(const membx_desc* desc, void* dev_arena, uint64_t arena_bytes,
                         void* hip_stream, membx_sys** out);

/* Release the handle (the arena returns to the caller). */
int32_t membx_sys_destroy(membx_sys* sys);

/* Advance n_steps steps of Langevin dynamics in the BAOAB splitting
 * (v += dt/2 F/m; x += dt/2 v; v = c1 v + c2 sqrt(kT/m) xi; x += dt/2 v;
 * F = F(x); v += dt/2 F/m, with c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2)),
 * one force evaluation per step.  xi are Box-Muller normals from Philox
 * stream 0 (counter = bead id, step).  Under membx_set_ensemble(.., 1, ..)
 * the steps are velocity Verlet with stochastic velocity rescaling instead.
 * Asynchronous. */
int32_t membx_md_step(membx_sys* sys, int64_t n_steps);

/* One batch of MC-MD exchange trials (paper, Theory, Eq. 1).  Candidates are
 * drawn in counter order from Philox stream 1: molecule X uniform over the
 * exchangeable molecules, Y uniform over the molecules of X's family with a
 * different kind.  A candidate is admitted when neither molecule is in an
 * admitted trial and each of its changed beads is at least r_cut (float64
 * minimum image) from every changed bead of the admitted trials; drawing
 * stops after n_trials admissions or 64 n_trials draws.  Each admitted trial
 * is accepted iff u < exp(-dU/kT) with dU = U(after) - U(before) evaluated
 * against the state at batch start and u from Philox stream 2; accepted
 * exchanges are applied.  n_admitted / n_accepted / out (length n_trials)
 * may be NULL; when non-NULL the call synchronizes.  n_trials <= max_trials.
 * Errors: E_INVAL. */
int32_t membx_mc_swap_trials(membx_sys* sys, int32_t n_trials, int32_t* n_admitted,
                             int32_t* n_accepted, membx_trial* out);

/* One MDAS alchemical trajectory (paper, Theory, Eqs. 2-3).  Selects n_pairs
 * exchange pairs with distinct molecules (Philox stream 3), then, starting
 * at lambda = 0 with U(lambda) = (1-lambda) U_A + lambda U_B, repeats
 * k_increments times: m_steps dynamics steps at fixed lambda, then
 * lambda += 1/k_increments, adding U_{lambda+dl}(x) - U_lambda(x) to the
 * work w.  At lambda = 1 the move is accepted iff u < exp(-w/kT) (u from
 * Philox stream 4): on acceptance the molecules keep their exchanged kinds
 * and the run continues from the final coordinates; on rejection the state
 * before the trajectory is restored.  k_increments = 1 with m_steps = 0 is
 * the single-step exchange of Eq. 1.  Outputs may be NULL (non-NULL
 * synchronizes); pairs_out gets 2 n_pairs molecule ids.  n_pairs <=
 * max_pairs.  Errors: E_INVAL, E_STATE (no exchangeable pair). */
int32_t membx_mdas_cycle(membx_sys* sys, int32_t n_pairs, int32_t k_increments,
                         int32_t m_steps, double* work, int32_t* accepted,
                         int32_t* pairs_out);

/* Energies of the current state, accumulated in float64 in a fixed order
 * (deterministic).  Synchronizes.  Errors: E_NONFINITE, E_SKIN,
 * E_LIST_OVERFLOW when the device flagged it since the last call. */
int32_t membx_energies(membx_sys* sys, membx_energy* out);

/* membx_energies for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results (bit for bit), with the energy
 * pass's block partials and final sums in a file-scope device array of the
 * library (8 MiB, one per device, held until the process ends) instead of
 * the system's arena.  Allocates nothing.  Systems whose partials need more
 * than the array (16 doubles per 256 lanes of the pass, 16 final sums) get
 * E_NOMEM.  Every call on a device shares that device's array: calls that
 * overlap on one device (from several threads or streams) race; the array
 * needs no clearing, as each call overwrites what it reads.
 * Synchronizes.  Errors as membx_energies, plus E_NOMEM. */
int32_t membx_energies_noalloc(membx_sys* sys, membx_energy* out);

/* Copy the state out in bead-id order (any pointer may be NULL).
 * counters = {step, batch, cycle}.  Synchronizes. */
int32_t membx_get_state(membx_sys* sys, double* pos, double* vel, int32_t* mol_kind,
                        int64_t* counters);

/* Replace the state (any pointer may be NULL); rebuilds the neighbour list
 * and re-evaluates the forces.  Coordinates are wrapped into the box.  With
 * the counters of membx_get_state, restoring a state taken right after a
 * list rebuild (a step count that is a multiple of rebuild_interval since
 * creation or the last retune) continues bit for bit as the run it was taken
 * from.  Synchronizes.  Errors (the state is left unchanged): E_NONFINITE
 * for a non-finite coordinate or velocity, E_INVAL for a kind outside the
 * molecule's family or a negative counter. */
int32_t membx_set_state(membx_sys* sys, const double* pos, const double* vel,
                        const int32_t* mol_kind, const int64_t* counters);

/* Current forces (those the next half-kick uses) in bead-id order, [3 N]. */
int32_t membx_forces(membx_sys* sys, double* f);

/* Mixing observable (Results: mixing followed through the pair
 * correlation of the PO4 beads of one lipid type, whose highest peak decays
 * to its mixed value): histogram of the lateral separations d (x and y, each
 * by the minimum-image convention) over all unordered pairs of bead `po4`
 * of the molecules of kind `kind` that sit in the same leaflet.
 * leaflet[n_mols] (host, read during the call): 0 or 1 per molecule, -1
 * leaves the molecule out.  Bin k < n_bins (1..4096) counts the pairs with
 * (k w)^2 <= d^2 < ((k + 1) w)^2, w = bin_width > 0, from the float64
 * squared distance of the current coordinates; counts[n_bins] (host)
 * receives them.  Exact (integer counts).  Synchronizes.  E_INVAL (bad
 * arguments, kind or bead index out of range). */
int32_t membx_pair_histogram(membx_sys* sys, int32_t kind, int32_t po4, const int32_t* leaflet,
                             int32_t n_bins, double bin_width, int64_t* counts);

/* Rebuild the neighbour list at the current coordinates and export its pair
 * set {(i, j): i < j, not bonded, float64 |r_ij|^2 < (r_cut + skin)^2} as
 * bead-id pairs.  Writes min(n, cap) pairs to ij [2 cap]; *n = pair count. */
int32_t membx_pairset_export(membx_sys* sys, int32_t* ij, int64_t cap, int64_t* n);

/* Capped steepest descent for synthetic start structures: each bead moves
 * by alpha F_i, shortened to at most max_step nm, n_iter times. */
int32_t membx_minimize(membx_sys* sys, int32_t n_iter, double alpha, double max_step);

/* Change the tuning of an existing system (skin <= skin_max and, as the box
 * may have changed under pressure coupling, box >= 3 (r_cut + skin); lanes_per_bead
 * in {1,2,4,8}, rebuild_interval >= 1; prune_interval <= 1 turns the inner
 * list off, else skin_inner in (0, skin] and lanes_per_bead >= 2).  Rebuilds
 * the list.  E_INVAL. */
int32_t membx_set_tuning(membx_sys* sys, double skin, int32_t rebuild_interval,
                         int32_t lanes_per_bead, double skin_inner, int32_t prune_interval);

/* Autotune skin, rebuild interval, lanes per bead and the inner list by
 * timing short runs from the current state: per candidate, n_steps
 * (<= 0: 200) untimed, then the fastest of three timed runs of n_steps.
 * Candidates: skin from 0.2 nm to skin_max (at most what the current box
 * allows, box >= 3 (r_cut + skin)) in steps of 0.1 nm, lanes per
 * bead 4 and 8, prune interval 1 (no inner list), 2, 3 and 4.  A pilot run
 * gives the largest displacement d4 over 4 steps; in the ballistic regime
 * (interval << 1/gamma) displacements grow linearly with time, so the
 * rebuild interval is the largest that keeps every bead within 0.8 skin/2,
 * and the inner buffer the smallest that keeps it within 0.8 delta/2 over a
 * prune interval.  A candidate is rejected if, in its timed runs, a bead went
 * beyond 0.9 skin/2 or beyond delta/2.  Candidates whose list build had to
 * re-test a crowded cell's candidates (a lane's hit buffer overflowed) are
 * chosen only if every candidate did: that path grows as a fresh system
 * equilibrates.  Positions, velocities, kinds and
 * random-number counters are restored afterwards; forces are recomputed and
 * the list is rebuilt.  Writes the chosen values and leaves the system
 * tuned.  E_DEVICE. */
int32_t membx_autotune(membx_sys* sys, int32_t n_steps, double* skin, int32_t* rebuild_interval,
                       int32_t* lanes_per_bead, double* skin_inner, int32_t* prune_interval);

/* Partner rule of exchange trials and MDAS pair selection, with a region
 * (leaflet) per molecule.  X is drawn uniformly over the exchangeable
 * molecules as always; Y, uniformly in ascending molecule id over:
 *   mode 0 (default): the molecules of X's family of another kind;
 *   mode 1: the same, within X's region: leaflet compositions never change
 *           (an asymmetric bilayer stays asymmetric);
 *   mode 2: every molecule of X's family in the other region, whatever its
 *           kind: the interleaflet exchange the paper proposes in its
 *           Discussion.  A partner of X's own kind gives a trial that changes
 *           nothing (dU = 0, counted as accepted).
 * Each rule proposes a pair as often as its reverse, so Eq. 1's Metropolis
 * test applies unchanged.  region[n_mols] (host, read during the call; NULL:
 * all 0): 0 or 1 for the molecules of swap families, ignored for the rest.
 * Synchronizes.  E_INVAL (mode or a region out of range). */
int32_t membx_set_exchange_regions(membx_sys* sys, int32_t mode, const int32_t* region);

/* Pressure coupling of membx_md_step (the paper's semi-isotropic 1 bar
 * barostat, Methods), by stochastic cell rescaling (Bernetti and Bussi,
 * J. Chem. Phys. 153, 114107, 2020) in place of the paper's Parrinello-
 * Rahman dynamics: after every MD step whose index is a multiple of nst,
 * e_A = ln(Lx Ly) and e_z = ln Lz each take one Ito step over t = nst dt,
 *   d e = -(kappa / tau_p) (P0 - P) t + sqrt(2 kappa kT t / (V tau_p)) xi,
 * with P_A = (N kT + (W_xx + W_yy) / 2) / V, P_z = (N kT + W_zz) / V from
 * the virial of membx_energy, kappa = compressibility (1/bar), P0 =
 * p_ref_bar, tau_p in ps, xi from Philox stream 6 with the step index as
 * counter; x and y scale by exp(d e_A / 2), z by exp(d e_z), positions
 * about the origin; the list is rebuilt and the forces refreshed.  The
 * stationary law is the isothermal-isobaric one.  MDAS cycles and exchange
 * trials run at the current box.  nst <= 0 turns coupling off (default).
 * Under coupling, step sequences are not replayed from HIP graphs.
 * Errors: E_INVAL (arguments); membx_md_step returns E_STATE if an axis
 * shrinks below three list radii. */
int32_t membx_set_barostat(membx_sys* sys, int32_t nst, double p_ref_bar, double compressibility,
                           double tau_p);

/* Pressure coupling of membx_md_step by the paper's own barostat (Methods:
 * semi-isotropic Parrinello-Rahman, 1 bar, tau_p 12 ps; Parrinello and
 * Rahman, J. Appl. Phys. 52, 7182, 1981) for a rectangular box.  Positions
 * are r = L s (s scaled coordinates) and the integrator's velocities are
 * peculiar, u_a = L_a ds_a/dt; the extended energy
 *   H = sum m |u|^2 / 2 + U + P0 V + (W / 2) sum_a (dL_a/dt)^2
 * gives W d2L_a/dt2 = V (P_aa - P0) / L_a (P_aa = (mv2_a + virial_a) / V as
 * in membx_energy; x and y both driven by (P_xx + P_yy) / 2), and a move of
 * the box at fixed s scales r_a by L'_a / L_a and u_a by L_a / L'_a.  Box
 * mass W = 3 tau_p^2 L_max / (4 pi^2 compressibility), L_max the longest
 * edge at this call, fixed afterwards.  After every MD step whose index is
 * a multiple of nst (t = nst dt): dL_a/dt += t V (P_aa - P0) / (W L_a), then
 * L'_a = L_a + t dL_a/dt with coordinates and velocities scaled; the list is
 * rebuilt and the forces refreshed.  Without a thermostat (Langevin gamma =
 * 0) H is conserved to first order in t.  The box velocity starts at zero.
 * Replaces membx_set_barostat's coupling (and vice versa); nst <= 0: off.
 * Units and errors as membx_set_barostat; E_NONFINITE from membx_md_step if
 * the pressure or the new box is not finite and positive. */
int32_t membx_set_barostat_pr(membx_sys* sys, int32_t nst, double p_ref_bar,
                              double compressibility, double tau_p);

/* Parrinello-Rahman box state: if set_box_vel (host, [3] nm/ps) is not
 * NULL, the box velocity is replaced first (for a restart from membx_
 * get_state, membx_get_box and this call's output); box_vel (may be NULL)
 * receives the box velocity, h_box (may be NULL) the box's terms of the
 * conserved energy, P0 V + (W / 2) sum_a (dL_a/dt)^2 in kJ/mol.  E_INVAL,
 * E_NONFINITE (a non-finite set_box_vel, nothing changed). */
int32_t membx_barostat_state(membx_sys* sys, const double* set_box_vel, double* box_vel,
                             double* h_box);

/* Lambda path of MDAS cycles.  path 0 (default): linear in the end-state
 * energies, U(lambda) = (1 - lambda) U_A + lambda U_B (Eq. 2), forces from
 * one pass plus lambda (F_B - F_A).  path 1: the soft-core path of Eq. 4
 * (shift delta nm^2, e.g. 0.05 = the paper's 5 A^2): each pair with a
 * changed bead takes the A-state LJ at mu = 1 - lambda and the B-state LJ
 * at mu = lambda, mu (c12 / s^6 - c6 / s^3) with s = r^2 + delta (1 - mu),
 * shifted to zero at the cutoff, and the reaction field of the
 * interpolated charge product; the work sums U(lambda_k) - U(lambda_k-1)
 * of those pairs (float64).  The end states are the same on both paths.
 * Errors: E_INVAL (path, delta). */
int32_t membx_set_mdas_path(membx_sys* sys, int32_t path, double delta);

/* Current box lengths (nm), host box[3]. */
int32_t membx_get_box(membx_sys* sys, double* box);

/* Ensemble of the MD steps (membx_md_step and the steps of MDAS cycles).
 * ensemble 0 (default): Langevin BAOAB with the friction of the descriptor.
 * ensemble 1: the paper's thermostat (Methods), stochastic velocity
 * rescaling (Bussi, Donadio, Parrinello 2007): velocity Verlet, then per
 * coupling group the kinetic energy K takes one exact step of its stochastic
 * dynamics with c = exp(-dt / tau_t) (tau_t > 0 in ps; infinity leaves
 * velocity Verlet), target 3/2 N_g kT, and the group's velocities are
 * multiplied by +-sqrt(K' / K); random numbers from Philox stream 5 with the
 * step index as counter.  kind_group[n_kinds] (host, read during the call;
 * null: all 0) puts each molecule kind in group 0 or 1, so a molecule's
 * group follows exchanges of its kind.  Not fused with the force pass: four
 * launches per step instead of one.  Synchronizes.  E_INVAL (ensemble, tau_t or a
 * group out of range). */
int32_t membx_set_ensemble(membx_sys* sys, int32_t ensemble, double tau_t,
                           const int32_t* kind_group);

/* Enable (1) or disable (0) HIP-graph replay of step sequences (default 1). */
int32_t membx_set_graphs(membx_sys* sys, int32_t enable);

/* Kernel timing: when enabled, HIP events on the library stream bracket
 * every launch of the nonbonded force kernel; membx_kernel_time returns the
 * number of timed launches and their mean duration (ms).  Synchronizes. */
int32_t membx_kernel_timing(membx_sys* sys, int32_t enable);
int32_t membx_kernel_time(membx_sys* sys, int64_t* launches, double* mean_ms);

/* Mean duration (ms) of the force pass of the MD steps at the current
 * state (forces plus the next step's update; the inner-list walk when
 * pruning is on, else the Verlet-list walk): n_launch launches (1..4096)
 * captured back to back in one HIP graph, one replay to warm up, then HIP
 * events on the library stream around a second replay.  The update goes to
 * scratch buffers and the forces it rewrites are the ones it computed
 * already, so the state is unchanged.  Synchronizes.  E_INVAL, E_DEVICE. */
int32_t membx_kernel_bench(membx_sys* sys, int32_t n_launch, double* mean_ms);

/* Per-system message for the last error ("" if none). */
const char* membx_last_error(const membx_sys* sys);

/* Synchronize and report device-side flags (skin violation, list overflow). */
int32_t membx_status(membx_sys* sys);

/* Bandwidth calibration: copy `bytes` (multiple of 16) from src to dst on the
 * library's stream with a plain vector-load/store kernel. */
int32_t membx_calib_copy(membx_sys* sys, void* dst, const void* src, uint64_t bytes);

/* ---------------------------------------------------------------- serving
 * Many independent systems ("jobs") resident in one caller-owned device
 * arena, stepped concurrently.  A job is a system descriptor plus a request:
 * md_cycles cycles of md_steps MD steps each, then mdas_cycles MDAS cycles
 * (mdas_pairs pairs, mdas_k increments, mdas_m steps per increment) -- the
 * paper's MC-MD and MDAS protocols (Theory) run as a service.
 *
 * Admission: jobs are admitted first come, first served, when a block of
 * membx_sys_bytes() for the job fits in the arena (first fit, freed blocks
 * coalesced); a job that does not fit waits and blocks the queue behind it.
 * Each resident job runs on its own HIP stream (default priority) with at
 * most two cycles in flight; membx_server_poll advances every job without
 * blocking (it never waits for the GPU, except for the short energy query
 * that closes a job).  A job's results do not depend on the other jobs.
 * The server allocates no device memory besides the caller's arena. */
typedef struct membx_server membx_server;

typedef struct membx_request {
    int32_t minimize_iters;       /* steepest-descent steps at admission    */
                                  /* (membx_minimize, alpha 1e-4, step cap  */
                                  /* 0.01 nm); 0: none                      */
    int32_t md_cycles;            /* cycles of plain MD (>= 0)              */
    int32_t md_steps;             /* steps per MD cycle (>= 1)              */
    int32_t mdas_cycles;          /* MDAS cycles after the MD cycles (>= 0) */
    int32_t mdas_pairs;           /* pairs per MDAS cycle (1..max_pairs)    */
    int32_t mdas_k;               /* lambda increments per MDAS cycle       */
    int32_t mdas_m;               /* MD steps per increment                 */
    int32_t count_pairs;          /* 1: each cycle ends with an energy pass */
                                  /* (about one force pass) whose count of  */
                                  /* pairs within r_cut, times the cycle's  */
                                  /* MD steps, is the cycle's pair          */
                                  /* interactions; 0: not counted           */
} membx_request;

typedef struct membx_job_result {
    int64_t job_id;
    int32_t status;               /* MEMBX_OK or the job's first error      */
    int32_t n_cycles;             /* cycles completed                       */
    int32_t mdas_accepted;        /* MDAS cycles accepted                   */
    int32_t n_beads;
    double  submit_s, admit_s, finish_s;   /* server clock (s since create) */
    double  cycle_ms_p50, cycle_ms_p99, cycle_ms_max;  /* per-cycle device  */
                                  /* time, HIP events on the job's stream   */
    int64_t md_steps;             /* MD steps run (MDAS steps included)     */
    int64_t fe_count;             /* force evaluations                      */
    int64_t pairs_in_cutoff;      /* at the end of the job                  */
    double  potential;            /* final potential energy, kJ/mol         */
    int64_t pair_interactions;    /* sum over cycles of the pair count at   */
                                  /* the cycle's end times its MD steps     */
                                  /* (count_pairs), else -1                 */
} membx_job_result;

/* Create a server over a device arena of arena_bytes (owned by the caller,
 * used until membx_server_destroy).  E_INVAL. */
int32_t membx_server_create(void* dev_arena, uint64_t arena_bytes, membx_server** out);

/* Queue a job.  The descriptor is copied (read only during this call); the
 * device state is built when the job is admitted.  E_INVAL (bad descriptor
 * or request), E_NOMEM (the job can never fit in the arena). */
int32_t membx_server_submit(membx_server* srv, const membx_desc* desc, const membx_request* req,
                            int64_t* job_id);

/* Advance all jobs: collect finished cycles, close finished jobs (freeing
 * their blocks), admit waiting jobs, issue the next cycles.  Writes up to
 * cap results of jobs finished since the last call (the rest are kept for
 * the next call) and the numbers of resident and waiting jobs (nullable).
 * E_INVAL, E_DEVICE. */
int32_t membx_server_poll(membx_server* srv, membx_job_result* out, int32_t cap, int32_t* n_out,
                          int32_t* n_resident, int32_t* n_waiting);

/* Device times (ms) of every cycle completed since creation, in completion
 * order: up to cap values, *n = total count.  E_INVAL. */
int32_t membx_server_cycle_times(membx_server* srv, float* out, int64_t cap, int64_t* n);

/* Pair interactions of every cycle completed since creation (as
 * membx_job_result.pair_interactions; -1 for a job without count_pairs), in
 * the order of membx_server_cycle_times: up to cap values, *n = total count.
 * E_INVAL. */
int32_t membx_server_cycle_pairs(membx_server* srv, double* out, int64_t cap, int64_t* n);

/* Wait for and release every resident job (their results are dropped). */
int32_t membx_server_destroy(membx_server* srv);

const char* membx_server_last_error(const membx_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* MEMBX_H */
