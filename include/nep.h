/*
 * nep.h -- C-ABI of libnep: the neuroevolution-potential (NEP) energy, force
 * and virial evaluation and the MD step built on it, for AMD Instinct MI355X
 * (gfx950).
 *
 * The operation (paper Sec. II.A, Eqs. 2-8; Sec. II.C.1, Eqs. 15-16): given
 * bead positions, types, an orthorhombic box and NEP parameters, compute the
 * site energies
 *     U_i = sum_mu w1_mu tanh(sum_nu w0_mu,nu q^i_nu - b0_mu) - b1       (Eq. 2)
 * from the radial descriptor q_n = sum_j g_n(r_ij) (Eq. 3) and the 3-body
 * angular descriptor q_nl = sum_m (-1)^m A_nlm A_nl(-m),
 * A_nlm = sum_j g_n(r_ij) Y_lm(r_ij) (Eqs. 4-5), with Chebyshev radial
 * functions and a cosine cutoff (Eqs. 6-8); the forces
 *     F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji),  r_ij = r_j - r_i,
 * the per-site virial W_i = sum_j r_ij (x) dU_j/dr_ji (Eq. 15) and the totals
 * E = sum_i U_i, W = sum_i W_i (Eq. 16).
 *
 * Units: nm, eV, amu, fs.  Forces in eV/nm, virials and energies in eV.
 *
 * Conventions for every call:
 *  - Array pointers are DEVICE pointers owned by the caller unless a comment
 *    says "host".  The library never frees caller memory and allocates device
 *    memory only in nep_model_create.
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = default stream) and
 *    is asynchronous unless the call's comment says it synchronises.
 *  - Return value: NEP_OK (0) or a negative nep_status.  nep_last_error()
 *    returns a thread-local message describing the last failure.
 *  - Calls on distinct streams with distinct buffers may run concurrently.
 *
 * Supported hyperparameters: n_max_R = 8, n_max_A = 6, basis_R = basis_A = 8,
 * l_max = 4 (37 descriptor components; the 4- and 5-body terms are not part
 * of the descriptor), 1 <= n_hidden <= 64, 1 <= n_types <= 4,
 * rc_A <= rc_R elementwise.  Others return NEP_ERR_UNSUPPORTED.
 */
#ifndef NEP_H
#define NEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NEP_OK = 0,
    NEP_ERR_ARG = -1,                /* invalid argument (message says which) */
    NEP_ERR_HIP = -2,                /* a HIP runtime call failed */
    NEP_ERR_NEIGHBOR_OVERFLOW = -3,  /* list capacity too small; see status */
    NEP_ERR_SKIN_VIOLATION = -4,     /* beads moved far enough since the build that a pair may be missing */
    NEP_ERR_NONFINITE = -5,          /* NaN/Inf position */
    NEP_ERR_OVERLAP = -6,            /* two beads (or a bead and its image) at distance 0 */
    NEP_ERR_UNSUPPORTED = -7,        /* hyperparameters or box outside what is built */
    NEP_ERR_OUTSIDE_BOX = -8         /* periodic coordinate not in [0, L) at a build */
} nep_status;

/* Bits of status[0] (device word written by the kernels). */
#define NEP_FLAG_OVERFLOW_R   1
#define NEP_FLAG_OVERFLOW_A   2
#define NEP_FLAG_SKIN         4
#define NEP_FLAG_NONFINITE    8
#define NEP_FLAG_OUTSIDE_BOX 16
#define NEP_FLAG_OVERLAP     32
#define NEP_FLAG_IMAGE_RANGE 64
#define NEP_FLAG_BAD_TYPE   128

/* ------------------------------------------------------------------------ */
/* model                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n_types;        /* number of species (atom or bead types), Sec. II.A, II.C.2 */
    int n_max_R;        /* radial components are n = 0..n_max_R (Eq. 3) */
    int n_max_A;        /* angular n = 0..n_max_A (Eq. 5) */
    int basis_R;        /* N_bas^R: Chebyshev k = 0..basis_R (Eq. 6) */
    int basis_A;        /* N_bas^A */
    int l_max;          /* l = 1..l_max (Eq. 4) */
    int n_hidden;       /* N_neu, tanh neurons (Eq. 2) */
    const float *rc_R;  /* host [n_types*n_types] radial cutoff per ordered type pair, nm, symmetric */
    const float *rc_A;  /* host [n_types*n_types] angular cutoff, <= rc_R */
} nep_hyper;

typedef struct nep_model_t *nep_model;

/* Number of floats in the flat parameter vector:
 *   w0[t][mu][nu], b0[t][mu], w1[t][mu], b1, cR[ti][tj][n][k], cA[ti][tj][n][k]
 * with nu = n for radial components and nu = (n_max_R+1) + (l-1)(n_max_A+1) + n
 * for angular ones.  The coefficients c are indexed by the ordered type pair
 * (t_i, t_j) of centre and neighbour (the species encoding of Sec. II.A); the
 * network weights are per centre type, b1 is shared.  Returns 0 on bad input. */
size_t nep_param_count(const nep_hyper *hyper);

/* Copies the host parameter vector to the device (the only allocation the
 * library makes).  The model is immutable afterwards and may be shared by
 * concurrent calls.  Synchronous. */
int nep_model_create(const nep_hyper *hyper, const float *params_host, size_t n_params,
                     nep_model *out);
int nep_model_destroy(nep_model model);

/* Engine of the network (Eq. 2) in the single-system fused kernel
 * (nep_compute_efv, nep_compute_efv_noalloc, nep_md_step):
 *   NEP_NETWORK_VALU  (default) each lane contracts its bead's descriptor with
 *                     the weights on the vector ALUs;
 *   NEP_NETWORK_MFMA  the descriptor x hidden-layer product of the 64 beads of a
 *                     wavefront and its transpose (dU/dq) on the FP32 matrix
 *                     cores (16x16x4 MFMA), one bead type and a hidden width of
 *                     at most 64 only (NEP_ERR_UNSUPPORTED otherwise).
 * Both give the same results up to rounding (the sums over hidden units run in
 * another order).  The batched and served forms always use the vector ALUs.
 * Changes the model: not to be called while another call uses it. */
#define NEP_NETWORK_VALU 0
#define NEP_NETWORK_MFMA 1
int nep_model_set_network(nep_model model, int engine);

/* ------------------------------------------------------------------------ */
/* system and neighbour lists                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;                /* number of beads */
    float *x, *y, *z;     /* device [n] each (SoA).  On periodic dimensions a build
                             needs 0 <= x < L; an MD step wraps them at rebuilds. */
    const uint8_t *type;  /* device [n], values < n_types */
    float box[3];         /* box lengths, nm.  On open dimensions box[d] sets the
                             extent [0, box[d]) of the cell grid. */
    int pbc[3];           /* 1 = periodic */
} nep_system;

/* Neighbour lists within r_c + skin (Sec. II.A "local environment within a
 * cutoff"), one row per bead, stored slot-major so that lanes of a wavefront
 * read consecutive beads:
 *   nbr[p*n + i], p < cnt[i]        entry p of bead i, packed as
 *                                    j | (code << 25), code = (nx+2) + 5(ny+2) + 25(nz+2)
 *                                    for the periodic image r_j + (nx Lx, ny Ly, nz Lz)
 *   the first cnt[n+i] entries      are the angular candidates (within r_c^A + skin),
 *                                    the rest the radial-only ones
 *   rev[p*n + i], p < cnt[n+i]      flat index q*n + j of the reverse entry (i in row j),
 *                                    or -1 when rounding left it out of row j
 *   order[t], t < n                 bead evaluated by thread t of the fused kernel (beads of
 *                                    similar row cost side by side within blocks of 256); the
 *                                    build writes it with the rows, so it always belongs to them
 * Rows are in a fixed order (neighbour cells, then index), so every later sum
 * has one canonical order.  The pair predicate is exact in float32:
 * s = fl(n*L); dx = fl(fl(x_j + s) - x_i); d2 = fl(fl(fl(dx dx) + fl(dy dy)) + fl(dz dz));
 * keep iff d2 < fl32((r_c(t_i,t_j) + skin)^2).                                      */
typedef struct {
    int cap;             /* slots per row (all entries) */
    int cap_A;           /* slots per row for the angular prefix (<= cap) */
    uint32_t *nbr;       /* device [cap][n] */
    int32_t *rev;        /* device [cap_A][n] */
    int32_t *cnt;        /* device [2][n]: cnt[i] all entries, cnt[n+i] angular prefix */
    float *ref;          /* device [3][n]: positions at the last build (completeness test) */
    float skin;          /* nm */
    int32_t *status;     /* device [4]: flags, max row length seen, max angular length, and the
                            float bits of the compression factor sigma accumulated since the
                            build (1.0 after a build; see nep_md_step) */
    int32_t *order;      /* device [n] or NULL: processing order written by the build (NULL: the
                            build writes none and the kernels take beads in index order) */
} nep_neighbors;

/* Device workspace needed by the calls below for n beads and capacities cap,
 * cap_A.  Contents are scratch; nothing persists between calls (a list build
 * and the evaluations that use its lists may each take a different workspace). */
size_t nep_workspace_bytes(nep_model model, int n, int cap, int cap_A);

/* Builds the lists for the current positions (cell lists with cells no smaller
 * than half of r_c + skin; images enumerated for boxes smaller than a few
 * cells).  wrap = 1 first wraps every periodic coordinate into [0, L) in place
 * (the lists then refer to the wrapped positions); wrap = 0 requires them to be
 * there already and reports NEP_ERR_OUTSIDE_BOX otherwise.
 * Synchronises the stream to read the status word: returns
 * NEP_ERR_NEIGHBOR_OVERFLOW when a row did not fit (status[1], status[2] hold
 * the required cap and cap_A; grow the buffers and call again),
 * NEP_ERR_NONFINITE, NEP_ERR_OUTSIDE_BOX, NEP_ERR_OVERLAP, NEP_ERR_ARG for a
 * type value >= n_types, or NEP_ERR_UNSUPPORTED when an image beyond +-2 boxes
 * would be needed. */
int nep_build_neighbors(nep_model model, nep_system *sys, nep_neighbors *nbrs, int wrap,
                        void *ws, size_t ws_bytes, void *stream);

/* Data layout only (no quantity of the paper changes: E, F and W are
 * invariant under a permutation of the beads, Sec. II.A).
 * Reorders the beads of a system in place into the cell order of the
 * neighbour build, so that beads near in space are near in memory again after
 * they have diffused (the lists, the fused kernel and the gather all read
 * neighbours' data by index).  x, y, z and type are permuted together with v,
 * F and U (device arrays as in nep_md_step, each may be NULL) and with perm
 * (device int32 [n] or NULL): new position s receives the bead that was at
 * position src(s), and perm[s] keeps naming that bead's index in the
 * caller's original numbering.  sys->type is written (it must be writable).
 * Periodic coordinates are wrapped first; the lists are rebuilt for the new
 * order.  Returns like nep_build_neighbors (synchronises the stream). */
int nep_sort_system(nep_model model, nep_system *sys, float *v, float *F, float *U, int32_t *perm,
                    nep_neighbors *nbrs, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* energy / force / virial (Eqs. 2-8, 15-16)                                 */
/* ------------------------------------------------------------------------ */
/* U: device [n] site energies or NULL.  F: device [3][n] (Fx, Fy, Fz planes).
 * W: device [9][n] per-site virial W_i[a][b] (plane 3a+b) or NULL.
 * E_tot: device double[1] or NULL.  W_tot: device double[9] or NULL.
 * Totals are reduced in a fixed order in FP64.  Lists must come from
 * nep_build_neighbors with the same model and skin.  Asynchronous.  A pair's
 * distance changes by at most the sum of its two beads' displacements since
 * the build, so the lists hold every pair within the cutoffs while the two
 * largest displacements of the system add up to less than the skin.  Once they
 * add up to 0.99 skin or more (the margin covers the rounding of the list
 * predicate), NEP_FLAG_SKIN is set in the status word (the results may then be
 * incomplete), which nep_check_status reports as NEP_ERR_SKIN_VIOLATION. */
int nep_compute_efv(nep_model model, const nep_system *sys, const nep_neighbors *nbrs,
                    float *U, float *F, float *W, double *E_tot, double *W_tot,
                    void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as nep_compute_efv, with the same arguments and results (bit for
 * bit), but no workspace argument.  Its scratch is a static device array of
 * NEP_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; the call itself allocates nothing.  An evaluation
 * needs about n (64 + 48 n_types + 16 cap_A) bytes of it (n = 16,384 beads
 * with cap_A = 64 fit); a larger one returns NEP_ERR_ARG with the size it
 * needs.  Nothing in the array must start at zero, and it keeps the last
 * call's contents.  Every call on one GPU shares its array: calls that
 * overlap on one GPU (other streams or threads) race and must be serialised
 * by the caller. */
#define NEP_NOALLOC_SCRATCH_BYTES (64u << 20)
int nep_compute_efv_noalloc(nep_model model, const nep_system *sys, const nep_neighbors *nbrs,
                            float *U, float *F, float *W, double *E_tot, double *W_tot, void *stream);

/* ------------------------------------------------------------------------ */
/* velocity-Verlet MD                                                        */
/* ------------------------------------------------------------------------ */
/* Constrained bead centres of mass, for generating coarse-grained training
 * labels (Sec. II.C.1): every bead I is a contiguous range of atoms whose
 * centre of mass R_I = sum_i C_Ii r_i (Eq. 9, mass weights) is held fixed by
 * the constraint force -(m_i/M_I) sum_{k in I} f_k on its atoms (applied to
 * the incoming force at the start of a call, and after every force
 * evaluation; it does no work, so the run is NVE).  After every step the
 * library adds the bead's total atomic force sum_{i in I} f_i (the mean force
 * of Eq. 12 once divided by the step count) and its virial sum_{i in I} W_i
 * (Eq. 14) to double accumulators.  The virial correction of Eq. 17 is the
 * caller's: it adds (N_AA - N_CG) k_B T to the diagonal of the total. */
typedef struct {
    int n_groups;                 /* N_CG */
    const int32_t *group_start;   /* device [n_groups + 1]: bead I holds atoms group_start[I] ..
                                     group_start[I+1] - 1 (ascending, covering 0 .. n) */
    double *F_sum;                /* device [3][n_groups]: += sum_{i in I} f_i after every step */
    double *W_sum;                /* device [9][n_groups]: += sum_{i in I} W_i after every step */
} nep_constraint;

typedef struct {
    float dt_fs;              /* time step */
    int n_steps;              /* steps in this call */
    int rebuild_every;        /* lists are rebuilt after the drift of step s when (s+1) % rebuild_every == 0,
                                 and whenever after a drift the two largest displacements since the build
                                 add up to more than 0.99 skin, unless the pair test (plain_skin_test)
                                 then finds every pair inside the cutoffs still listed; where the pair test
                                 runs, once the call has built lists the schedule instead rebuilds lists that
                                 have served rebuild_every steps */
    int force_rebuild;        /* in: rebuild after the first drift whatever the displacement (after the
                                 caller has regrown the lists of a call stopped by an overflow) */
    float mass[4];            /* amu per type */
    double strain_rate[3];    /* engineering strain per step: L_d(s) = box0_d (1 + rate_d s) */
    double box0[3];           /* reference box of the strain */
    int64_t step;             /* global step counter s; advanced per completed step (in/out) */
    int n_rebuilds;           /* out: list rebuilds done by this call */
    double *pair_counts;      /* device double[2] or NULL: += sum_i N_R(i), sum_i N_A(i) over every
                                 force evaluation (pairs inside the interaction cutoffs) */
    double *W_trace;          /* device double [n_steps][9] or NULL: total virial W = sum_i W_i
                                 (Eq. 16) at the end of every step, W[a][b] at 9k + 3a + b */
    float *W;                 /* device [9][n] or NULL: per-bead virial W_i (Eq. 15) at the final
                                 positions, plane 3a + b */
    /* Ensembles.  The paper equilibrates in NVT and NPT (Sec. III.A.1, III.C.3)
     * and runs HNEMD (Sec. III.B.3) in an external engine without naming the
     * algorithms; these are the published methods taken here (all off when zero). */
    int thermostat;           /* 0 none (NVE), 1 Berendsen, 2 Bussi stochastic velocity rescaling;
                                 applied after the second half-kick of every step */
    float T_target;           /* K */
    float tau_T;              /* coupling time, fs */
    const double *noise;      /* device [n_steps][2] (thermostat 2): per step a standard normal R and a
                                 chi-square draw S with 3n - 4 degrees of freedom */
    int barostat;             /* 0 none, 1 Berendsen per periodic axis: every step of the call scales
                                 positions and box by mu_d = cbrt(1 - beta dt/tau_P (P_target_d - P_in_d)),
                                 clamped to [0.99, 1.01]; not with strain on the same axis */
    double P_target[3];       /* eV/nm^3 (1 GPa = 6.2415 eV/nm^3) */
    double tau_P;             /* fs */
    double beta;              /* compressibility, 1/(eV/nm^3) */
    double P_in[3];           /* pressure that sets this call's factor (the previous call's P_out);
                                 a non-finite entry leaves that axis unscaled */
    double P_out[3];          /* out: mean diagonal pressure (2 K_dd + W_dd)/V over the completed steps */
    float Fe[3];              /* HNEMD driving force parameter, 1/nm (zero: off): the force of every
                                 step gains W_i^T F_e minus its mean over the beads */
    double *J_trace;          /* device [n_steps][3] or NULL: potential heat current sum_i W_i v_i
                                 after every step (eV nm/fs; with a thermostat, after its scaling) */
    const nep_constraint *constraint;  /* host struct or NULL: constrained bead centres of mass */
    int plain_skin_test;      /* 0: when the two-largest test fires, the pair test decides: every pair
                                 with a bead that moved at least half of 0.99 skin since the build and
                                 now inside an interaction cutoff must have been inside the list cutoff
                                 at the build (any other pair moved less than 0.99 skin); found through
                                 the build's cells, so used only after a rebuild within this call, in a
                                 fully periodic box with every side at least 3 (r_c + skin), without
                                 strain or barostat.  1: the two-largest test alone and the schedule
                                 by step number */
} nep_md_params;

/* Advances sys by n_steps of velocity Verlet (the paper's MD runs in an
 * external engine and states no integrator; this is plain NVE):
 *   v' = v + dt/2 a(F);  x += dt v';  affine strain;  [wrap + rebuild];
 *   F = F(x), U, W (Eqs. 2-8, 15-16);  v = v' + dt/2 a(F),
 * with a = 9.648533212e-5 F/m (nm/fs^2 from eV/nm and amu).  Every step
 * evaluates the site energies, the forces and the per-bead and total virial.
 * On entry F (device [3][n]) must hold the forces at the current positions,
 * and the lists must come from nep_build_neighbors for this system (built at
 * any earlier positions: the rebuild test rebuilds them when they no longer
 * cover the pairs), or force_rebuild must be set.  On exit x, v, F and the
 * lists hold for the final positions.  v: device [3][n] nm/fs.  U: device [n]
 * or NULL (site energies at the last step).  E_pot / E_kin: device double
 * [n_steps] traces or NULL; params->W_trace and params->W as above.
 *
 * Ensembles (thermostat, barostat, F_e or a constraint set): each step runs the gather
 * without the fused kick, then four small kernels (sums, drive without its
 * mean and second half-kick, thermostat factor, velocity scaling).  The
 * force F passed in is used as is for the first half-kick (the plain
 * potential force from nep_compute_efv, or the previous call's F, which holds
 * the drive); F on exit holds the total force with the drive.  The barostat
 * factor is fixed for the call, so the caller runs NPT as a sequence of calls
 * (of, say, 10 steps) passing P_out back as P_in.
 *
 * Strain: the constant engineering strain-rate loading of the nanowire
 * (Sec. III.C.5), L_d(s) = box0_d (1 + rate_d s) with positions scaled
 * affinely about the origin each step; rates of either sign are accepted as
 * long as 1 + rate_d s stays above 0.05 over the call (NEP_ERR_ARG otherwise).
 *
 * Rebuild decisions are taken on the device, with no host synchronisation
 * inside the call.  A pair's separation changes since the build by its affine
 * part, which under compression shrinks it by at most (1 - sigma)(r_c + skin)
 * (sigma = product over the steps since the build of the smallest per-step
 * scale factor, capped at 1; kept in status[3]), plus the non-affine
 * displacements of its two beads.  The lists are rebuilt after a drift when
 * the two largest non-affine displacements plus (1 - sigma)(r_c + skin) exceed
 * 0.99 skin, or when the schedule (s + 1) % rebuild_every == 0 asks for one;
 * the build kernels queued in every step do nothing while the gate is off.
 * The lists used by a force evaluation therefore always hold every pair
 * within the cutoffs.  params->n_rebuilds returns the number of rebuilds.
 *
 * The new positions and velocities of a step are written to sys and v only
 * when its forces are done.  A rebuild that overflows (or finds a bad
 * position) therefore stops the run with x, v and F of the last completed
 * step: the call returns the error with params->step advanced by the completed
 * steps, and the caller regrows the lists (status[1], status[2]) and repeats
 * the call for the remaining steps with force_rebuild set, which continues the
 * same trajectory.  sys->box follows the strain of the completed steps.  The
 * call synchronises the stream before it returns. */
int nep_md_step(nep_model model, nep_system *sys, float *v, nep_md_params *params,
                nep_neighbors *nbrs, float *F, float *U, double *E_pot, double *E_kin,
                void *ws, size_t ws_bytes, void *stream);

/* Reads the status word (synchronises the stream) and maps it to a status. */
int nep_check_status(const nep_neighbors *nbrs, int32_t host_status_out[4], void *stream);

/* ------------------------------------------------------------------------ */
/* many independent replicas, one MD step each (served form)                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    nep_system *sys;         /* positions (device [n] each), types, box, pbc */
    float *v;                /* device [3][n] nm/fs */
    float *F;                /* device [3][n]: forces at the current positions (in/out) */
    float *U;                /* device [n] or NULL */
    nep_neighbors *nbrs;     /* the replica's lists, from nep_build_neighbors */
    void *ws;                /* the replica's own workspace (nep_workspace_bytes) */
    size_t ws_bytes;
    int64_t step;            /* in/out: the replica's step counter (advanced when the step completed) */
    int rebuilt;             /* out: 1 when this step rebuilt the lists */
    int status;              /* out: NEP_OK, or the error that stopped this replica's step */
} nep_replica;

/* Workspace of nep_md_step_batch for up to max_active replicas per call. */
size_t nep_md_batch_workspace_bytes(int max_active);

/* The served form of the MD step: continuous batching of independent
 * replicas, each advanced by the integrator of nep_md_step (Eqs. 2-8 for the
 * forces).  One velocity-Verlet step (as nep_md_step, no strain) for each of n_active
 * replicas that share one model, batched: one drift launch over the tiles of
 * every replica, the builds of the replicas that fail the rebuild test of
 * nep_md_step (their two largest displacements add up to more than 0.99 skin;
 * no pair test, as nep_md_step with plain_skin_test = 1, whose results it
 * equals bit for bit) or whose schedule asks for one
 * ((step + 1) % rebuild_every == 0), one fused-
 * kernel launch, one gather launch and one launch of per-replica energy sums.
 * A replica's results depend only on its own state: alone or in any mix they
 * are the same.  E_pot / E_kin: device double [n_active] or NULL.  A replica
 * whose rebuild fails keeps x, v and F of its last step (status set, step not
 * advanced); the others are unaffected.  The call reads the rebuild gates back
 * to the host once and synchronises the stream before it returns; it returns
 * NEP_OK unless an argument is invalid or HIP fails (per-replica errors are in
 * the status fields). */
int nep_md_step_batch(nep_model model, nep_replica *replicas, int n_active, float dt_fs, const float mass[4],
                      int rebuild_every, double *E_pot, double *E_kin, void *ws, size_t ws_bytes,
                      void *stream);

/* ------------------------------------------------------------------------ */
/* batched evaluation for the fitness loop (Sec. II.A: candidates of the      */
/* evolution strategy scored by the RMSE of energies and virials per bead and */
/* of forces per component)                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int block;       /* threads per workgroup: 64, 128 or 256 (0 = 256) */
    int order;       /* structures by index (0) or largest first (1) */
    int wg_per_cu;   /* resident workgroups per compute unit (0 = as many as fit) */
    int schedule;    /* the order in which workgroups take the (candidate, structure) items:
                        0 the given work order (largest structures first when order = 1),
                        1 structure-major (every candidate of a structure together: its
                          positions and lists stay in cache), 2 candidate-major (every structure
                          of a candidate together: its tables stay in cache), 3 blocked (groups of
                          8 candidates, structure-major inside a group) */
} nep_batch_config;

/* Number of configurations nep_batch_autotune tries. */
#define NEP_BATCH_TUNE_CONFIGS 36

typedef struct {
    const double *E; /* device [n_systems]: reference energy of each structure (eV) */
    const double *F; /* device [sum_s n_s][3]: reference forces, structures in order (eV/nm) */
    const double *W; /* device [n_systems][9]: reference total virial W[a][b] at 3a+b (eV) */
} nep_labels;

/* Workspace for nep_compute_efv_batch with this configuration (cfg NULL: the
 * largest over every configuration nep_batch_autotune tries).  0 on bad
 * arguments (nep_last_error). */
size_t nep_batch_workspace_bytes(const nep_model *models, int n_models, const nep_system *systems,
                                 const nep_neighbors *lists, int n_systems, int n_items,
                                 const nep_batch_config *cfg);

/* Evaluates n_items (candidate, structure) pairs in one persistent launch.
 * The batched kernel is built for n_types <= 2 (the one-type water-like and
 * the two-type C60-like families); models with more types return
 * NEP_ERR_UNSUPPORTED here and in the two calls around it.
 * models: host array of n_models handles that share n_types, n_hidden and
 * cutoffs (the candidates of one model family).  systems / lists: host arrays
 * of n_systems structures and their lists from nep_build_neighbors (skin 0 is
 * fine for a single evaluation; positions must not have moved since).  work:
 * host [n_items][2] = (model index, system index).  Workgroups take items from
 * a device work queue, each item being evaluated whole by one workgroup; every
 * reduction has a fixed order, so results do not depend on the schedule.
 * Outputs (device, each may be NULL):
 *   rmse     [n_models][3]: RMSE_E (eV/bead), RMSE_F (eV/nm per component),
 *            RMSE_W (eV/bead over xx yy zz xy yz xz) over the model's items,
 *            against labels (labels required when rmse is given);
 *   item_out [n_items][10]: E and total W[9] of every item, in work order;
 *   F_out    [sum over items of n][3]: forces of every item, in work order.
 * cfg NULL: defaults.  Synchronises the stream before it returns. */
int nep_compute_efv_batch(const nep_model *models, int n_models, const nep_system *systems,
                          const nep_neighbors *lists, int n_systems, const int32_t *work, int n_items,
                          const nep_labels *labels, double *rmse, double *item_out, float *F_out,
                          const nep_batch_config *cfg, void *ws, size_t ws_bytes, void *stream);

/* Times every configuration of its search space on the given work and returns
 * the fastest in best: schedule 1..3 x order 0/1 x wg_per_cu (0, 2) x block
 * (64, 128, 256), NEP_BATCH_TUNE_CONFIGS points, each timed as the median of
 * three runs after a warm-up run.  tried: host [NEP_BATCH_TUNE_CONFIGS] or
 * NULL, the configurations in the order of ms: host [NEP_BATCH_TUNE_CONFIGS] or
 * NULL, the measured times (ms).  The result is kept in-process under the
 * device and a signature of the workload (sizes, list capacities, work list);
 * a later call with the same signature returns it without timing
 * (*from_cache = 1; from_cache may be NULL).  The workspace must hold
 * nep_batch_workspace_bytes(..., NULL).  Synchronises the stream. */
int nep_batch_autotune(const nep_model *models, int n_models, const nep_system *systems,
                       const nep_neighbors *lists, int n_systems, const int32_t *work, int n_items,
                       void *ws, size_t ws_bytes, void *stream, nep_batch_config *best, float *ms,
                       nep_batch_config *tried, int *from_cache);

/* ------------------------------------------------------------------------ */
/* the training loop: SNES over the batched fitness evaluation (Sec. II.A)    */
/* ------------------------------------------------------------------------ */
/* The paper optimises the parameters with the separable natural evolution
 * strategy (SNES, Schaul et al. 2011) on a loss of energy, force and virial
 * RMSEs (per bead, per component, per bead) plus L1 and L2 regularisation
 * with weights lambda_e, lambda_f, lambda_v, lambda_1, lambda_2.  A generation
 * on the device: nep_snes_sample, nep_models_load_params (candidates become
 * the parameters of existing models), nep_compute_efv_batch (their RMSEs), and
 * nep_snes_update.  All three calls are asynchronous on the stream. */
typedef struct {
    double lambda_e, lambda_f, lambda_v;   /* weights of RMSE_E (eV/bead), RMSE_F (eV/nm), RMSE_W (eV/bead) */
    double lambda_1, lambda_2;             /* weights of mean |z| and sqrt(mean z^2) over the parameters */
    double eta_mu, eta_sigma;              /* learning rates (SNES defaults: 1 and (3 + ln d)/(5 sqrt d)) */
} nep_snes_params;

/* Replaces the parameters of n_models existing models by the rows of params
 * (device [n_models][nep_param_count] floats, the flat layout above): the
 * flat copy and the derived tables are rewritten on the device with the
 * arithmetic of nep_model_create, so the result equals a model created from
 * the same vector.  The models must share n_types and n_hidden.  Calls that
 * use the models must follow on the same stream (the models change in stream
 * order).  Non-finite parameters are not checked here. */
int nep_models_load_params(nep_model *models, int n_models, const float *params, void *stream);

/* z[k][p] = mu[p] + sigma[p] s[k][p] for k < pop (device arrays; s holds
 * standard normal draws, an input so that any caller can reproduce them). */
int nep_snes_sample(int pop, size_t dim, const float *mu, const float *sigma, const float *s, float *z,
                    void *stream);

/* One SNES update.  loss (device double [pop]) receives
 *   L_k = lambda_e rmse[k][0] + lambda_f rmse[k][1] + lambda_v rmse[k][2]
 *         + lambda_1 mean_p |z[k][p]| + lambda_2 sqrt(mean_p z[k][p]^2),
 * order (device int32 [pop] or NULL) the candidates from best to worst
 * (lower loss first, ties by index, non-finite losses last); then with the
 * utilities u_r = max(0, ln(pop/2 + 1) - ln r) / sum_j max(0, ...) - 1/pop
 * of the ranks r = 1..pop,
 *   mu    += eta_mu sigma sum_r u_r s_(r),
 *   sigma *= exp(eta_sigma/2 sum_r u_r (s_(r)^2 - 1)).
 * 2 <= pop <= 1024. */
int nep_snes_update(int pop, size_t dim, const float *s, const float *z, const double *rmse,
                    const nep_snes_params *h, float *mu, float *sigma, double *loss, int32_t *order,
                    void *stream);

/* ------------------------------------------------------------------------ */
/* kernel timing (benchmark support)                                         */
/* ------------------------------------------------------------------------ */
/* While enabled, the library records a HIP event pair on the launching stream
 * around every launch of its kernels, by class: 0 = fused descriptor /
 * network / angular-force kernel, 1 = gather (forces, virial, half-kick),
 * 2 = neighbour build (all of its kernels), 3 = first half-kick + drift
 * (with the rebuild test and, in MD, the previous step's energy reduction).
 * nep_timing_begin(max_launches, class_mask) creates the event pool
 * (host-side objects only) and enables recording, for the classes whose bit
 * is set in class_mask (bit c for class c), in the calling process; launches
 * beyond the pool are not timed.  Every event pair adds a little time on the
 * device, so a throughput measurement times only the class it needs.
 * nep_timing_end synchronises on the recorded events, writes the summed
 * milliseconds and launch counts per class into ms[4] and
 * launches[4] (host), destroys the pool and disables recording.  Not
 * thread-safe: meant for a single benchmarking thread. */
int nep_timing_begin(int max_launches, unsigned class_mask);
int nep_timing_end(double ms[4], int launches[4]);

const char *nep_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NEP_H */
