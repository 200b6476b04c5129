/*
 * gcme.h -- C ABI of the MI355X (gfx950) engine for the GCMe nonbonded path:
 * Gaussian-core excluded volume plus Gaussian-smeared electrostatics with an
 * Ewald split (cell list -> cutoff pair kernels -> smooth PME).
 *
 * Model (reduced units, k_B T = 1; lengths in the bead diameter):
 *   u_ex(r)   = A_ij (3/(2 pi s_ij^2))^{3/2} exp(-3 r^2/(2 s_ij^2)),
 *               s_ij^2 = sigma_i^2 + sigma_j^2            (eq. u_ex)
 *   u_elec(r) = lB z_i z_j erf(sqrt(pi/2) r / a_ij) / r,
 *               a_ij^2 = a_i^2 + a_j^2                     (eq. u_elec)
 *   U_elec    = U_real + U_recip + U_corr + U_self         (eq. ewald)
 *     U_real  = lB sum_{i<j, r<rc} z_i z_j [erf(alpha_ij r) - erf(beta r)]/r,
 *               alpha_ij = sqrt(pi/2)/a_ij, beta = 1/(sqrt(2) G)
 *     U_recip = (2 pi lB/V) sum_{k!=0} exp(-k^2/(4 beta^2))/k^2 |S(k)|^2,
 *               evaluated by smooth particle-mesh Ewald (order p B-splines
 *               on a K0 x K1 x K2 mesh, tin-foil boundary: k = 0 dropped)
 *     U_corr  = -lB beta/sqrt(pi) sum z_i^2,  U_self = lB/2 sum z_i^2/a_i
 *   Forces F_i = -dE/dr_i.  Virial W_ab = sum_pairs r_ij,a f_ij,b plus the
 *   reciprocal-space tensor (its trace enters eq. pres_virial).
 *
 * Conventions for every call:
 *   - Arrays marked "device" are HIP device pointers on the context's device;
 *     the caller owns them, the library never frees or keeps them past the
 *     call.  Arrays marked "host" are read during the call only.
 *   - Per-bead arrays are replica-concatenated in n_beads order, original
 *     bead order within a replica.  Coordinates are SoA: [3][N_total]
 *     (all x, then all y, then all z), float64.
 *   - Device work is enqueued on the context's stream; outputs are valid
 *     once that stream has reached the call's end (gcme_sync waits for it).
 *   - Every call returns a gcme_status.  Validation errors leave all outputs
 *     and the context unchanged; gcme_last_error() gives a message.
 *     GCME_EDEVICE means the context is unusable and must be destroyed.
 *   - One context per host thread; calls on one context are not reentrant.
 */
#ifndef GCME_H
#define GCME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gcme_ctx* gcme_handle;

typedef enum {
    GCME_OK = 0,
    GCME_EINVAL = 1,        /* bad argument (NULL, size, range) */
    GCME_EUNSUPPORTED = 2,  /* grid not 2^a 3^b, order outside 3..8, too many types */
    GCME_EGEOMETRY = 3,     /* cutoff > L/2, non-positive box */
    GCME_ENONNEUTRAL = 4,   /* a replica's net charge is not zero */
    GCME_ESTATE = 5,        /* call order (e.g. forces before params/state) */
    GCME_EDEVICE = 6,       /* HIP runtime error */
    GCME_ENOMEM = 7,        /* device allocation failed */
    GCME_EOVERFLOW = 8      /* fixed-point force accumulator would overflow, or a
                               neighbour list is full.  The mixed-precision charge
                               mesh is not checked: a point holds +-128 unit
                               charges (32-bit integers at 2^-24), reached only
                               if several hundred unit charges of one sign
                               (300 at order 3, 600 at order 5) crowd into the
                               p^3 mesh cells around it */
} gcme_status;

typedef enum {
    GCME_FP64 = 0,  /* all pair, mesh and FFT arithmetic in float64 */
    GCME_MIXED = 1  /* pair + mesh + FFT in float32; forces summed in 64-bit
                       fixed point; energies and virial reduced in float64 */
} gcme_precision;

/* Energy terms, per replica, in this order (kT units). */
enum {
    GCME_E_EX = 0,      /* sum of u_ex over pairs within the cutoff */
    GCME_E_REAL = 1,    /* U_elec,real */
    GCME_E_RECIP = 2,   /* U_elec,recip (mesh) */
    GCME_E_CORR = 3,    /* U_elec,corr (constant) */
    GCME_E_SELF = 4,    /* U_elec,self (Born, constant) */
    GCME_E_POT = 5,     /* sum of the potential terms: 0..4, GCME_E_SLAB and
                           GCME_E_BOND */
    GCME_E_KIN = 6,     /* kinetic energy (gcme_step observations only, else 0) */
    GCME_E_SLAB = 7,    /* slab correction (GCME_FLAG_SLAB_CORRECTION, else 0) */
    GCME_E_BOND = 8,    /* harmonic bonds (gcme_set_bonds, else 0) */
    GCME_N_TERMS = 9
};

#define GCME_MAX_TYPES 4

typedef struct {
    int32_t n_replicas;       /* >= 1 independent periodic boxes */
    const int32_t* n_beads;   /* host [n_replicas], each >= 2 */
    int32_t precision;        /* gcme_precision */
    int32_t device;           /* HIP device ordinal */
    void* stream;             /* hipStream_t to enqueue on; NULL = a stream the
                                 library creates and owns */
    uint64_t seed;            /* Langevin noise seed */
} gcme_create_info;

typedef struct {
    double box[3];            /* orthorhombic box edges L0, L1, L2 (> 0) */
    double cutoff;            /* real-space cutoff rc, rc <= min(L)/2 */
    double beta;              /* Ewald splitting (erf(beta r)); beta = 1/(sqrt2 G) */
    int32_t grid[3];          /* mesh K0, K1, K2: each 2^a 3^b, 8 <= K <= 512
                                 (ignored when kmax > 0) */
    int32_t order;            /* B-spline order p, 3..8, p <= K/2; the same for
                                 every replica */
    double lB;                /* Bjerrum length */
    int32_t n_types;          /* 1..GCME_MAX_TYPES */
    const double* A;          /* host [n_types * n_types], symmetric, kT d^3 */
    const double* sigma;      /* host [n_types] mass smearing radius (> 0) */
    const double* a;          /* host [n_types] charge smearing radius (> 0) */
    const double* mass;       /* host [n_types] or NULL (all 1).  INFINITY holds
                                 the type's beads fixed (no kick, no noise, zero
                                 velocity, no kinetic energy): the electrode
                                 lattices of the slab systems (section on
                                 polyelectrolyte adsorption at electrodes) */
    double kT;                /* thermostat temperature */
    double dt;                /* time step */
    double gamma;             /* Langevin friction; 0 = velocity Verlet (NVE) */
    uint32_t flags;           /* GCME_FLAG_* */
    double kmax;              /* 0: the reciprocal term of eq. ewald by smooth PME
                                 on the mesh.  > 0: that term summed exactly over
                                 the wave vectors k = 2 pi (n0/L0, n1/L1, n2/L2),
                                 0 < |k| <= kmax (no mesh; for small replicas,
                                 where the sum is cheap and has no mesh error);
                                 kmax L / (2 pi) <= 64 on every axis */
    double bond_k;            /* harmonic bonds u = bond_k/2 (r - bond_b)^2 of the  */
    double bond_b;            /* pairs given to gcme_set_bonds (polyanion chains of
                                 the adsorption study: k = 100, b = 0.8); >= 0 */
} gcme_params;

/* Reject parameters that violate the paper's no-collapse condition
 * A_ij/(s_ij^3 kT) > 4 pi^{3/2} lB/(3^{3/2} a_ij) for some type pair
 * (Model and methods, after eq. u_elec).  Without the flag it is not checked. */
#define GCME_FLAG_STRICT_CONTACT 1u

/* All-reciprocal splitting: G = a/sqrt(pi), i.e. beta = alpha = sqrt(pi)/(2a),
 * the choice under which the real-space bracket of eq. ewald vanishes for
 * equal smearing radii (Model and methods, on the choice of G): the smeared
 * Coulomb interaction lies wholly in the reciprocal sum, whose Gaussian is
 * then the smearing itself.  Requires one charge radius a for every type
 * (GCME_EINVAL otherwise); `beta` is ignored and the real-space electrostatic
 * pairs are not evaluated (U_real = 0).  The reciprocal sum needs a mesh (or
 * kmax) fine enough for that beta.  dE/da is not provided for such a replica
 * (GCME_EUNSUPPORTED when requested), since beta then depends on a. */
#define GCME_FLAG_ALL_RECIPROCAL 2u

/* Slab correction for a slab that is periodic in x and y and separated from
 * its periodic images along z by a vacuum gap (the nonmetal-electrode
 * systems of the adsorption study, whose box is tripled along z; the
 * correction of Yeh and Berkowitz that the paper cites): adds
 * E = 2 pi lB M_z^2 / V, M_z = sum_i z_i zeta_i with zeta_i the z coordinate
 * in [0, L2), and its forces F_iz = -4 pi lB z_i M_z / V, to the tin-foil
 * sum of eq. ewald.  Virial diag(E, E, -E) (minus its derivative under
 * diagonal strains).  The beads must stay inside the slab (walls of fixed
 * beads, see gcme_params.mass): M_z uses the wrapped coordinate. */
#define GCME_FLAG_SLAB_CORRECTION 4u

typedef struct {
    const double* pos;   /* device [3][N_total] new positions, or NULL = keep state */
    double* force;       /* device [3][N_total] out, or NULL */
    double* energy;      /* device [n_replicas][GCME_N_TERMS] out, or NULL */
    double* virial;      /* device [n_replicas][6] out (xx,yy,zz,xy,xz,yz), or NULL */
    double* dE_dA;       /* device [n_replicas][MAX_TYPES*MAX_TYPES] out, or NULL:
                            entry (t,u) = dE/dA_tu of the symmetric parameter */
    double* dE_dsigma;   /* device [n_replicas][MAX_TYPES] out, or NULL */
    double* dE_da;       /* device [n_replicas][MAX_TYPES] out, or NULL */
    double* dE_dsigma_bead;  /* device [N_total] out, or NULL: per bead, the
                                derivative of E with respect to the bead's own
                                mass radius sigma_i (eq. u_ex), as if every bead
                                had its own radii, at the per-type values;
                                summed over a type it is dE_dsigma */
    double* dE_da_bead;      /* device [N_total] out, or NULL: the same for the
                                charge radius a_i (eq. u_elec through the
                                real-space term of eq. ewald, and eq.
                                self_energy; the reciprocal and correction
                                terms do not depend on a).  Original bead order.
                                gcme_forces_energy only (gcme_step with steps
                                to take: GCME_EINVAL) */
    const double* force_vjp; /* device [3][N_total] in, or NULL: a vector v per
                                bead.  When set, dE_dA, dE_dsigma and dE_da (at
                                least one required) receive the forces'
                                vector-Jacobian product sum_i v_i . dF_i/dtheta
                                instead of dE/dtheta: the gradient of a
                                force-matching loss L(F) with v = dL/dF.  Only
                                the pair terms depend on the parameters (eq.
                                u_ex, the real-space term of eq. ewald); the
                                entry for a type pair with A = 0 is 0.  Not
                                with the per-bead outputs (GCME_EINVAL);
                                gcme_forces_energy only */
} gcme_io;

/* Create a context for n_replicas independent periodic systems, each the
 * bead system of section "Gaussian core model" (N beads with positions,
 * types and charge numbers in an orthorhombic box; the batch of boxes is
 * this interface's own).  Allocates every device buffer whose size depends
 * only on bead counts.  *out is set only on GCME_OK; on an error nothing is
 * kept (GCME_EINVAL for a bad argument, GCME_EDEVICE when no device or
 * stream is available, GCME_ENOMEM when an allocation fails). */
gcme_status gcme_create(const gcme_create_info* info, gcme_handle* out);

/* Set force-field, mesh and integrator parameters of one replica
 * (replica = -1: all).  Validates geometry and sizes, builds the cell grid,
 * mesh plans, B-spline moduli and pair tables, and (re)allocates mesh and
 * cell buffers.  Synchronous with respect to the context's stream. */
gcme_status gcme_set_params(gcme_handle h, int32_t replica, const gcme_params* p);

/* Harmonic bonds (the chain connectivity of the adsorption study):
 * pairs is host [n_bonds][2] of concatenated bead indices, both beads of a
 * bond in the same replica, each bond u = bond_k/2 (r - bond_b)^2 with its
 * replica's bond_k and bond_b, over the minimum-image separation.  Bonded
 * beads keep their nonbonded terms.  Replaces the previous list
 * (n_bonds = 0 removes every bond); the pairs are copied.  GCME_EINVAL on an
 * index out of range, a bead bonded to itself or a bond across replicas.
 * The bond forces enter every later evaluation and step. */
gcme_status gcme_set_bonds(gcme_handle h, int64_t n_bonds, const int32_t* pairs);

/* Method of image charges for perfectly conducting electrodes (section
 * "Method of image charges"): the real system lies in 0 < z < L2/2 between
 * electrodes at z = 0 and z = L2/2, and each charged bead has an image bead,
 * its reflection (x, y, -z) across z = 0 with the opposite charge, in the
 * other half of the box (the reflection across z = 0 with the period L2 is
 * also the reflection across z = L2/2).  pairs is host [n_images][2] of
 * (image, source) concatenated bead indices in one replica; a bead is an
 * image at most once and never both an image and a source.  Image beads
 * must be of a type with infinite mass (gcme_params.mass) and, to carry no
 * excluded volume, zero A; their charge must be the opposite of their
 * source's (both checked at the next evaluation, GCME_EINVAL).  After every
 * binning (each evaluation and step) the images are moved to their sources'
 * reflections, exactly on the fixed-point lattice, so the forces on the real
 * beads include the images' field; the images' own forces are not used.
 * Energies and virial are those of the whole doubled box: the real system's
 * electrostatic energy is half of U_elec of the doubled box.  Replaces the
 * previous list (n_images = 0 removes them). */
gcme_status gcme_set_images(gcme_handle h, int64_t n_images, const int32_t* pairs);

/* Load the dynamic state of the bead system (section "Gaussian core
 * model": positions r_i, species, charge numbers z_i; the periodic images n
 * of eq. ewald make positions equivalent modulo the box): positions (device
 * [3][N] float64, any real coordinates; wrapped into the box and stored as
 * 32-bit fractions of each edge, i.e. rounded to the nearest multiple of
 * L/2^32), velocities (device [3][N] float64 or NULL = zero), types (device
 * int32 [N], 0..n_types-1) and charge numbers (device int32 [N],
 * |z| <= 127).  The arrays are copied; the caller keeps ownership.  Checks
 * types (GCME_EINVAL) and that every replica is neutral, as the Ewald sum
 * of eq. ewald with the tin-foil boundary requires (GCME_ENONNEUTRAL);
 * on an error the previous state is kept.  Resets the step counter.
 * Synchronous. */
gcme_status gcme_set_state(gcme_handle h, const double* pos, const double* vel,
                           const int32_t* type, const int32_t* z);

/* Copy the dynamic state (section "Gaussian core model": positions and
 * velocities of the beads) out in original bead order: positions wrapped
 * into [0, L) at the stored 2^-32 L resolution (device [3][N] or NULL),
 * velocities (device [3][N] or NULL), and the number of steps taken since
 * gcme_set_state (host, or NULL).  The caller owns the outputs.
 * GCME_ESTATE before any gcme_set_state.  Asynchronous for the device
 * arrays (valid after gcme_sync). */
gcme_status gcme_get_state(gcme_handle h, double* pos, double* vel, uint64_t* step);

/* One force/energy evaluation (paper: eqs. u_ex, u_elec, ewald) at the
 * state's positions, or at io->pos (which then become the state).
 * Asynchronous on the context's stream. */
gcme_status gcme_forces_energy(gcme_handle h, const gcme_io* io);

/* Advance n_steps >= 0 of molecular dynamics with the forces of eqs. u_ex,
 * u_elec and ewald: the Langevin equations of motion that the paper's MD
 * integrates each timestep (section "Method of image charges"; the timestep
 * sizes of sections "Performance" and "Image charge effects on
 * polyelectrolyte adsorption"), by BAOAB splitting with friction gamma at
 * temperature kT and Philox4x64-10 noise keyed by (seed, step, bead id,
 * replica); with gamma == 0, velocity Verlet (NVE).  Image beads follow
 * their sources after every update (gcme_set_images).  If observe != NULL
 * its outputs (caller-owned device arrays, as for gcme_forces_energy) are
 * filled at the final positions (energy includes GCME_E_KIN).  Steps are
 * replayed from captured HIP graphs, which the first run after a change of
 * parameters or tuning captures (n_steps == 0 without observe takes no step
 * and only captures them); the call allocates no device memory.
 * GCME_EINVAL for n_steps < 0, observe->pos set, or per-bead/force_vjp
 * outputs with steps to take; GCME_ESTATE before parameters and state.
 * Asynchronous; device errors surface at gcme_sync. */
gcme_status gcme_step(gcme_handle h, int32_t n_steps, const gcme_io* observe);

/* Wait for the context's stream and report device-side status: a force
 * that would overflow the 64-bit fixed-point accumulator of eq. ewald's
 * force sum, or a full neighbour list -> GCME_EOVERFLOW (the outputs of the calls since the last
 * gcme_sync are then invalid); runtime errors -> GCME_EDEVICE.  The status
 * is cleared once reported. */
gcme_status gcme_sync(gcme_handle h);

/* Message describing the last error on h (or on creation if h is NULL).
 * Valid until the next call on h. */
const char* gcme_last_error(gcme_handle h);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * evaluation of gcme_forces_energy for one periodic replica, with the
 * creation, parameters and state folded into the call and every device
 * buffer the evaluation needs (sorted state, cell lists, clusters, tables,
 * charge mesh, partial sums, status) carved from a static device array of
 * GCME_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds from
 * the library's load until the process ends.  The call makes no hipMalloc,
 * hipFree or other device allocation (its host-side planning uses ordinary
 * host memory); it runs on `stream` (NULL = the null stream) of the current
 * device and uses the default tuning, with the three parts of the
 * evaluation in sequence on that stream.
 *   p       host, as for gcme_set_params (bonds and images are not
 *           available here)
 *   n_beads >= 2; precision: gcme_precision
 *   pos     device [3][n_beads] float64, type and z device int32 [n_beads]
 *           (as for gcme_set_state)
 *   force   device [3][n_beads] out, energy device [GCME_N_TERMS] out,
 *           virial device [6] out; each may be NULL; caller-owned
 * Synchronous: returns after the outputs are written, with the device
 * status of gcme_sync (GCME_EOVERFLOW).  GCME_ENOMEM, before any kernel is
 * launched, when the system needs more scratch than
 * GCME_NOALLOC_SCRATCH_BYTES (about 140 bytes per bead plus the mesh and
 * cell tables: some 3e5 beads at a 64^3 mesh); validation errors as for the
 * calls it folds in.  gcme_last_error(NULL) gives the message.  Every call
 * on one GPU uses that GPU's one array and leaves its contents behind (the
 * call clears what it reads before writing it): calls that overlap on one
 * GPU, from several host threads or on several streams, race and must be
 * serialised by the caller. */
#define GCME_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
gcme_status gcme_forces_energy_noalloc(const gcme_params* p, int32_t n_beads, int32_t precision,
                                       const double* pos, const int32_t* type, const int32_t* z,
                                       double* force, double* energy, double* virial, void* stream);

/* Tuning knobs picked by the autotuner (exposed for benchmarks and tests).
 * Any field < 0 means "leave as is".  The pair kernels work on clusters of
 * consecutive cell-sorted beads, either with one neighbour list per cluster
 * (built each evaluation) or list-free (each cluster evaluates the beads of
 * its cell columns directly).  Both visit the same pairs with the same
 * cutoff test; they differ in the order of the per-bead sums. */
typedef struct {
    int32_t cells_per_cutoff;    /* cell edge ~ rc / n (1..4) */
    int32_t beads_per_cluster;   /* excluded-volume cluster size (2, 4, 8) */
    int32_t charges_per_cluster; /* real-space electrostatics cluster size (2, 4, 8) */
    int32_t list_slack_pct;      /* list capacity above the density estimate, % (0..1000) */
    int32_t direct_pairs;        /* list-free kernels: bit 0 excluded volume,
                                    bit 1 real-space electrostatics (0..3) */
    int32_t stream_layout;       /* how the three independent parts of a force
                                    evaluation (excluded-volume pairs, charged
                                    pairs, mesh chain) share streams (0..5):
                                    0: each on its own stream;
                                    1: the pairs on the context's stream, the
                                       mesh chain on a second one;
                                    2: the mesh chain on the context's stream,
                                       charged then excluded-volume pairs on a
                                       second one;
                                    3: as 2, excluded-volume pairs first;
                                    4: excluded-volume pairs on the context's
                                       stream, the mesh chain then the charged
                                       pairs on a second one;
                                    5: the mesh chain then the charged pairs on
                                       the context's stream, the
                                       excluded-volume pairs on a second one */
    int32_t mesh_tile_x;         /* z lines per mesh tile of the fused spread */
    int32_t mesh_tile_y;         /* pass along x and y (1..16; 0 = 4): a bead's
                                    B-splines are evaluated once per tile its
                                    stencil meets, so larger tiles evaluate them
                                    fewer times but hold more LDS, and fewer
                                    workgroups fit a compute unit (halved along
                                    the longer side until they fit) */
    int32_t gather_tile_x;       /* the same for the fused gather pass (0 = the */
    int32_t gather_tile_y;       /* spread's) */
    int32_t half_pairs;          /* column-cluster pair kernels, two bits per
                                    pair type: bits 0-1 excluded volume, bits
                                    2-3 real-space electrostatics; 0 = the
                                    kernels of direct_pairs, 1 = half shell,
                                    2 = both ends.  Clusters are then runs of
                                    consecutive beads of one cell column
                                    (beads_per_cluster / charges_per_cluster
                                    4 or 8; 2 is taken as 4), rebuilt after
                                    every sort.  Half shell: a cluster
                                    evaluates the beads of its own column
                                    that follow it and of the columns ahead
                                    of its own, each unordered pair once, and
                                    both beads of a pair receive its force.
                                    Both ends: every column within reach,
                                    each pair from both of its beads' clusters.
                                    Evaluations that ask for parameter
                                    derivatives, and pair counting, use the
                                    kernels of direct_pairs. */
} gcme_tuning;

gcme_status gcme_get_tuning(gcme_handle h, gcme_tuning* t);
gcme_status gcme_set_tuning(gcme_handle h, const gcme_tuning* t);

/* Time candidate tunings on the current state and keep the fastest: every
 * cluster size, cell size and list choice as a stream-launched evaluation,
 * then the charged-cluster sizes and stream layouts of the best few as
 * replays of the captured step graph (the form a run of steps takes), each
 * from the saved state.  The state (bead order, positions, velocities,
 * forces, step counter) is restored exactly afterwards.
 * Tunings change the order of the per-bead floating-point sums, so results
 * agree across tunings to rounding; for one tuning, reruns on the same
 * inputs are bit-identical.  Synchronous. */
gcme_status gcme_autotune(gcme_handle h);

/* Number of unordered pairs with r < rc (all replicas), counted by the pair
 * kernel's own cutoff test at the state's positions.  Synchronous. */
gcme_status gcme_count_pairs(gcme_handle h, uint64_t* n_pairs);

/* Device time of each stage of a step: the kernels of stage i are captured
 * n_reps >= 1 times back to back into a HIP graph, which is replayed between
 * two HIP events on the context's stream; ms[i] = elapsed / n_reps (host
 * array of at least GCME_N_STAGES entries).  The state, forces and mesh are
 * saved before and restored after, so the call leaves the simulation as it
 * found it.  Synchronous.  gcme_stage_name(i) names stage i (NULL if out of
 * range). */
#define GCME_N_STAGES 12
gcme_status gcme_profile_step(gcme_handle h, int32_t n_reps, double* ms);
const char* gcme_stage_name(int32_t i);

/* Device time of each stage's kernel inside real steps, as it runs in a
 * step's graph: n_steps >= 1 steps are taken (the state advances as with
 * gcme_step(n_steps)), each the first half on the stream followed by a
 * one-step graph (the step's own kernels, so they overlap as in gcme_step's
 * graphs).  In these launches the first lane of every wavefront records the
 * GPU's constant-rate real-time counter at the wavefront's start and end;
 * the host waits for each step and takes, per launch, the first start to
 * the last end: the launch's execution span.  ms[i] = the mean span of
 * stage i's kernel over the steps (host array of GCME_N_STAGES; 0 for a
 * stage this configuration does not launch, e.g. the list builds of
 * list-free pairs, and for the sort, which is several kernels; int_last is
 * the plain second half).  Synchronous. */
gcme_status gcme_time_stages(gcme_handle h, int32_t n_steps, double* ms);

/* Release all device memory and the owned stream. */
void gcme_destroy(gcme_handle h);

#ifdef __cplusplus
}
#endif

#endif /* GCME_H */
