/*
 * qnep.h -- C ABI of the MI355X (gfx950) qNEP force-evaluation library.
 *
 * qNEP (arXiv:2601.19034): a neuroevolution potential whose network has two
 * outputs per atom, a site energy and a partial charge (Sec. 2.1 Eq. 1, Sec. 2.2),
 * with long-range electrostatics on the corrected charges by Ewald summation
 * (Sec. 2.2.1-2.2.3, Eqs. 6-10) or PPPM (Sec. 2.6, Eqs. 34-38).  One call
 * evaluates, for one periodic structure,
 *   E       total energy U_NEP + U_ES                       (Eqs. 2-4)
 *   F       forces with static and dynamic-charge terms     (Sec. 2.3, Eqs. 11-23)
 *   W       virial, W_ab = -dE/d(strain_ab)                 (Eqs. 12, 20-22)
 *   q       screened corrected charges q' and naked q~'     (Eqs. 24, 33)
 *   Z*      Born effective charges, periodic form           (Sec. 2.4 Eq. 28)
 *   P       polarization sum_i q~'_i r_i                    (Eq. 26)
 *
 * Conventions
 *   Units: eV, Angstrom, elementary charge.  k_e = e^2/(4 pi eps0) = 14.399645 eV*A.
 *   Charges: q~ = s q with s = sqrt(eps_inf) (Eq. 24); the neutrality correction
 *   q~' = q~ + (Q - sum_j q~_j)/N (Eq. 33, sign read so that sum q~' = Q); U_ES
 *   uses q' = q~'/s, P and Z* use q~'.  The chain rule through the correction is
 *   exact (dE/dq_i = phi_i - mean(phi)).
 *
 * Memory and streams
 *   Every array argument marked "device" lives in device memory of the current
 *   HIP device; the caller owns all of them, including the workspace.  The library
 *   does not allocate device memory, does not free anything it did not create, and
 *   never synchronizes the stream inside qnep_compute / qnep_backward: all work is
 *   enqueued on the caller's stream and the outputs are valid once that stream
 *   has reached the end of the call.  Functions are thread-compatible: one model
 *   handle may be used from one thread at a time; concurrent calls must use
 *   distinct workspaces.
 *
 * Errors
 *   Arguments are validated on the host before any launch; a failing call returns
 *   a negative status and enqueues nothing.  Conditions that can only be detected
 *   on the device (a neighbour list longer than its capacity, a species index out
 *   of range) raise bits in the workspace's status word, read by qnep_check_status.
 *   qnep_last_error() returns a thread-local message describing the last failure.
 */
#ifndef QNEP_H
#define QNEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QNEP_OK = 0,
    QNEP_E_INVALID_ARG = -1,  /* null pointer, bad size, singular cell, bad species count */
    QNEP_E_UNSUPPORTED = -2,  /* hyper-parameters or mesh not compiled into this library */
    QNEP_E_WORKSPACE = -3,    /* workspace smaller than qnep_workspace_size() */
    QNEP_E_DEVICE = -4,       /* a HIP runtime call failed */
    QNEP_E_INTERNAL = -5,
    QNEP_E_CAPACITY = -6      /* a device-side capacity was exceeded (see qnep_check_status) */
} qnep_status;

/* device status bits (qnep_check_status) */
#define QNEP_FLAG_RADIAL_OVERFLOW 1
#define QNEP_FLAG_ANGULAR_OVERFLOW 2
#define QNEP_FLAG_COULOMB_OVERFLOW 4
#define QNEP_FLAG_BAD_SPECIES 8
#define QNEP_FLAG_INTERNAL 16  /* an atom fell outside its charge-assignment tile (should not happen) */
#define QNEP_FLAG_OUTSIDE 32   /* isolated system: an atom lies outside the bounding box */
#define QNEP_FLAG_IMAGE 64     /* isolated system: a periodic image of the bounding box is within a cutoff */

/* MLP arithmetic */
#define QNEP_MLP_FP32 0   /* FP32 vector ALU */
/* The BF16 forms run both products of the network on the matrix cores (BF16 inputs,
   FP32 accumulation) with FP32 operands split as hi + lo BF16 parts:
   QNEP_MLP_BF16    forward D W0^T with both operands split (three products), backward
                    G W0 with the split weights against the activation gradient rounded
                    once to BF16 (two products); forces within 5 meV/A of FP64 on the test
                    workloads (a single rounding of every operand is not: about 1e-2)
   QNEP_MLP_BF16X3  both products with both operands split (about 16 mantissa bits) */
#define QNEP_MLP_BF16 1
#define QNEP_MLP_BF16X3 2

/* NEP hyper-parameters (Sec. 2.1; the descriptor definitions are the published
   NEP3/NEP4 ones the paper refers to):
     radial   q_n  = sum_j g^R_n(r_ij),          n = 0..n_max_R
     angular  q_nl = sum_m (sum_j g^A_n(r_ij) Yhat_lm(r_ij))^2,  n = 0..n_max_A, l = 1..l_max
     g_n(r) = sum_k c^{t_i t_j}_{nk} f_k(r),  f_k = (T_k(2(r/rc-1)^2-1)+1)/2 * (1+cos(pi r/rc))/2
   with k = 0..basis_R (or basis_A) and Yhat_lm real spherical harmonics normalized so that
   sum_m Yhat_lm(u) Yhat_lm(v) = P_l(u.v).  Descriptor order: radial, then angular l-major. */
typedef struct {
    int32_t n_types;   /* number of species T (1..4) */
    int32_t n_max_R, n_max_A;
    int32_t basis_R, basis_A;
    int32_t l_max;     /* 4 */
    int32_t n_neu;     /* hidden units (<= 64) */
    double rc_R, rc_A; /* cutoffs, Angstrom, rc_A <= rc_R */
} qnep_hparams;

#define QNEP_ES_EWALD 0
#define QNEP_ES_PPPM 1
#define QNEP_ES_DIRECT 2

/* electrostatics (Sec. 2.2 and 2.6) */
typedef struct {
    int32_t mode;           /* 1: real + reciprocal + self (Eq. 3); 2: reciprocal only (Eq. 5) */
    int32_t method;         /* 0: direct Ewald; 1: PPPM (periodic systems); 2 (QNEP_ES_DIRECT): the
                               plain Coulomb sum over all pairs of an isolated system (mode ignored) */
    double alpha;           /* Ewald splitting parameter, 1/Angstrom */
    double rc_coul;         /* real-space cutoff (mode 1), Angstrom */
    double kmax;            /* Ewald: wave vectors with |k| < kmax (Eq. 7) */
    int32_t kmax_inclusive; /* 1: |k| <= kmax.  Ties resolved with a 1e-9 relative tolerance on k^2 */
    int32_t mesh[3];        /* PPPM mesh along a, b, c: each a product of 2, 3, 5, at most 1024 */
    int32_t order;          /* PPPM assignment order, 5 */
    double q_total;         /* target total charge Q of Eq. 33 */
    double efield[3];       /* external electric field E (V/Angstrom): adds F_i[b] += sum_a E_a Z_i[a][b]
                               to the forces (Sec. 2.4 Eq. 29); the energy and virial carry no field
                               term (the paper gives the force only).  Zero = no field */
} qnep_es_params;

/* one structure */
typedef struct {
    int64_t n_atoms;      /* N >= 0, N < 2^23 */
    const float *pos;     /* device, SoA [3][N]: x[0..N), y[0..N), z[0..N), Angstrom, any image */
    const int32_t *type;  /* device, [N], species in [0, n_types) */
    double cell[9];       /* host, row-major, rows are the cell vectors a, b, c (right-handed) */
    int32_t pbc[3];       /* periodicity along a, b, c: {1, 1, 1} periodic; {0, 0, 0} an isolated
                             system (cluster, molecule) whose cell is a bounding box: every atom
                             inside it (QNEP_FLAG_OUTSIDE otherwise) and no atom within a cutoff of
                             another atom's periodic image (QNEP_FLAG_IMAGE otherwise); isolated
                             systems take es->method = QNEP_ES_DIRECT and their Born charges are the
                             derivative of P with absolute positions (Sec. 2.4 Eq. 27).  Mixed
                             periodicity is not supported (QNEP_E_UNSUPPORTED). */
} qnep_system;

/* outputs; any pointer may be NULL to skip that output (all device) */
typedef struct {
    double *energy;        /* [1] E */
    float *forces;         /* SoA [3][N] */
    double *virial;        /* [9] W[a][b] */
    float *charges;        /* [N] screened corrected charges q' (enter U_ES) */
    float *charges_naked;  /* [N] naked corrected charges q~' = s q' (enter P, Z*) */
    float *bec;            /* [9][N]: Z_i[a][b] stored at bec[(3a+b)*N + i] */
    double *polarization;  /* [3] */
    double *energy_terms;  /* [8]: U_NEP, U_r, U_k, U_s, U_bg, sum q_raw, mean phi, number of k vectors */
    float *virial_atom;    /* [9][N]: per-atom virial W_i[a][b] at virial_atom[(3a+b)*N + i] (Sec. 2.3
                              Eq. 12, W_i = sum_j r_ij (x) F_ji over every partial force; reciprocal part
                              per atom by Eq. 20 (Ewald) or Eq. 39 (PPPM, six more inverse transforms);
                              the static real-space pair virial shared equally by the two atoms; the
                              background virial U_bg I split evenly).  sum_i W_i = W.  NULL = skip (the
                              extra work is only done when requested) */
} qnep_outputs;

/* number of entries of the flat FP32 parameter vector theta, laid out as
     cR[ti][tj][n][k], cA[ti][tj][n][k],
     per species t: W0[mu][nu] (n_neu x N_des), b0[mu], w1E[mu], w1q[mu], b1q,
     then b1E (shared output bias of Eq. 1) and s = sqrt(eps_inf) (Eq. 24).
   Returns -1 for invalid hyper-parameters. */
int64_t qnep_param_count(const qnep_hparams *hp);

/* creates a host-side model handle (hyper-parameters, MLP precision, plans).
   mlp_precision: QNEP_MLP_FP32, QNEP_MLP_BF16 or QNEP_MLP_BF16X3. */
qnep_status qnep_model_create(const qnep_hparams *hp, int32_t mlp_precision, void **model);
qnep_status qnep_model_destroy(void *model);

/* neighbour-list capacity = factor * (density * 4/3 pi rc^3) + 32 entries per atom
   (default factor 1.6).  Overflow is reported by qnep_check_status. */
qnep_status qnep_model_set_capacity_factor(void *model, double factor);

/* bytes of device workspace qnep_compute needs for this structure size, cell and
   electrostatics setup (no device work). */
qnep_status qnep_workspace_size(const void *model, const qnep_es_params *es, const qnep_system *sys,
                                size_t *bytes);

/* full evaluation (E, F, W, q, Z*, P) of one structure.
   theta: device FP32 [qnep_param_count].  ws: device, ws_bytes >= qnep_workspace_size.
   stream: a hipStream_t (NULL = default stream).  Asynchronous: see the header notes. */
qnep_status qnep_compute(void *model, const float *theta, const qnep_es_params *es, const qnep_system *sys,
                         const qnep_outputs *out, void *ws, size_t ws_bytes, void *stream);

/* Allocation-free evaluation, for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   qnep_compute with the workspace taken from a fixed device array that the library
   holds, one per GPU, from the first call on that GPU until the process ends.
     limit      structures whose qnep_workspace_size() exceeds QNEP_STATIC_WORKSPACE_BYTES
                (64 MiB: about 12,000 water-like atoms with Ewald or PPPM) are rejected
                with QNEP_E_WORKSPACE before anything is enqueued
     flags_out  device int32 [1] or NULL: receives the device status bits of this call
                (those qnep_check_status reports) at the end of the enqueued work
   The call enqueues kernel launches only (no allocation, no memset, no event record, no
   synchronization; per-stage timing is not recorded).  Its first call on a device
   resolves the array's address (hipGetSymbolAddress), so make one call before
   capturing.  Every call on one GPU shares that GPU's array and the array keeps the
   last call's contents (every value read is first written by the same call): calls that
   overlap on one GPU, on different streams or threads, race and give undefined results. */
#define QNEP_STATIC_WORKSPACE_BYTES (64u * 1024u * 1024u)
qnep_status qnep_compute_static(void *model, const float *theta, const qnep_es_params *es, const qnep_system *sys,
                                const qnep_outputs *out, int32_t *flags_out, void *stream);

/* Reverse mode for L = gE * E + gP . P (the adjoint of qnep_compute), recomputing the
   forward pass (descriptors are not kept between calls).  Writes, when non-NULL:
     d_pos   device FP32 SoA [3][N]  dL/dr_i = -gE F_i + sum_a gP_a Z_i[a][:]
             (the polarization term uses the periodic Born charges of Eq. 28)
     d_cell  device FP64 [9]         dE/dh for the row-major cell at fixed Cartesian
             positions, gE h^{-T} (sum_i F_i (x) r_i - W)^T.  The energy term only: the
             cell derivative of P (through the image shifts that enter the charges) is
             not formed, so a call with d_cell != NULL and a non-zero gP is rejected
             with QNEP_E_UNSUPPORTED before anything is enqueued
     d_theta device FP32 [n_theta]   exact dL/dtheta in the parameter layout above
   gP may be NULL (zero).  es->efield must be zero (the adjoint is of the field-free
   energy; QNEP_E_UNSUPPORTED otherwise).  ws must hold qnep_backward_workspace_size() bytes. */
qnep_status qnep_backward_workspace_size(const void *model, const qnep_es_params *es, const qnep_system *sys,
                                         size_t *bytes);
qnep_status qnep_backward(void *model, const float *theta, const qnep_es_params *es, const qnep_system *sys,
                          double gE, const double *gP, float *d_pos, double *d_cell, float *d_theta, void *ws,
                          size_t ws_bytes, void *stream);

/* Molecular dynamics in the microcanonical ensemble (velocity Verlet), the workload the
   paper's speed figures refer to (Sec. 3.1), with the time series of the polarization
   current P_dot_a = sum_i sum_b Z_i[a][b] v_i[b] (Sec. 2.4 Eq. 30).  Every step runs one
   full evaluation (neighbour lists rebuilt from the sorted bins each step).
     md->dt        time step, fs;  md->n_steps  number of steps (>= 0)
     md->masses    host, [n_types], atomic mass units
     type          device, [N];  cell: host [9] as in qnep_system
     pos, vel      device FP32 SoA [3][N], Angstrom and Angstrom/fs, updated in place
                   (positions are not wrapped back into the cell)
     series        device FP64 [n_steps + 1][8]: E_pot, E_kin, P_dot (3, e*Angstrom/fs),
                   P (3, e*Angstrom); row 0 is the initial state, row s the state after
                   step s.  With an external field (es->efield) the forces include the
                   field force and E_pot excludes the field's work.
   ws must hold qnep_md_workspace_size() bytes; the device status word is at its start
   (qnep_check_status).  Asynchronous; nothing is allocated. */
typedef struct {
    double dt;
    int32_t n_steps;
    const double *masses;
} qnep_md_params;
qnep_status qnep_md_workspace_size(const void *model, const qnep_es_params *es, int64_t n_atoms,
                                   const double *cell, size_t *bytes);
qnep_status qnep_md_nve(void *model, const float *theta, const qnep_es_params *es, const qnep_md_params *md,
                        int64_t n_atoms, const int32_t *type, const double *cell, float *pos, float *vel,
                        double *series, void *ws, size_t ws_bytes, void *stream);

/* synchronizes `stream` and returns the device status bits of the last call that
   used this workspace (0 = no device-side condition). */
qnep_status qnep_check_status(const void *ws, void *stream, int32_t *flags);

/* Per-stage timing with HIP events recorded on the caller's stream (for profiling;
   adds one event record per stage).  enable = 0 turns it off.  read_timing
   synchronizes the recorded events and returns, for each stage, the total
   milliseconds and the number of kernel launches since the previous read
   (arrays of length QNEP_N_STAGES), then resets the totals. */
#define QNEP_N_STAGES 19
qnep_status qnep_model_enable_timing(void *model, int32_t enable);
qnep_status qnep_model_read_timing(void *model, double *ms, int64_t *launches, int32_t *calls);
const char *qnep_stage_name(int32_t stage);

/* ------------------------------------------------------------------------------
 * Batched evaluation for training (Sec. 2.5): many small periodic structures, each
 * under many candidate parameter vectors (a population, as evaluated by the
 * evolution strategy the paper trains with), in one persistent launch.  Ewald
 * electrostatics only (Sec. 2.2); the per-structure Ewald sum is set up once as a
 * pair kernel (the parameters do not enter it) and contracted with the charges of
 * every candidate.
 *
 * Sequence: qnep_batch_workspace_size -> allocate -> qnep_batch_prepare (builds the
 * parameter-independent geometry into the workspace) -> any number of
 * qnep_batch_compute calls with the same workspace.  The model handle keeps the
 * host-side plan of the last prepared batch; a later prepare replaces it.
 * qnep_batch_tune times tile choices on the prepared batch and keeps the fastest.
 * Species must be in [0, n_types); all structures share the model's species set.
 * Limits: at most 2048 atoms per structure; parameters per candidate at most 12288;
 * l_max = 4, basis_R = basis_A = 8, (n_max_R, n_max_A) = (4, 4) or (8, 6).
 * ------------------------------------------------------------------------------ */
#define QNEP_BATCH_VIRIAL 1   /* also form the per-(structure, candidate) virial */
#define QNEP_BATCH_GRADIENT 2 /* reserve the buffers of qnep_batch_gradient */

typedef struct {
    int32_t n_structures;   /* S >= 1 */
    int32_t flags;          /* QNEP_BATCH_VIRIAL or 0 */
    const int64_t *offsets; /* host, [S + 1], offsets[0] = 0; atoms of structure s are
                               offsets[s] .. offsets[s+1]-1 of the packed arrays */
    const double *cells;    /* host, [S][9], rows a, b, c (Angstrom), right-handed */
    const float *pos;       /* device, SoA [3][n_total] (Angstrom), read by prepare only */
    const int32_t *type;    /* device, [n_total], read by prepare only */
} qnep_batch;

typedef struct {
    const double *energy;   /* device, [S] reference energies (eV) */
    const float *forces;    /* device, SoA [3][n_total] reference forces (eV/Angstrom) */
    double lambda_e, lambda_f, lambda_q; /* weights of the three RMSE terms */
    double lambda_1, lambda_2;           /* weights of |theta|_1 and |theta|_2^2 */
} qnep_batch_targets;

typedef struct {
    float *losses;   /* device, [S][C][3]: |E - E_ref|/N, RMS over the 3N force components
                        of F - F_ref, |sum_i q~_i - Q| (scaled charges before the
                        correction, Q = es.q_total); required */
    double *loss;    /* device, [C]: lambda_e sqrt(mean_s (dE/N)^2) + lambda_f RMSE of all
                        force components + lambda_q sqrt(mean_s dQ^2) + lambda_1 |theta|_1
                        + lambda_2 |theta|_2^2; NULL = skip */
    double *energy;  /* device, [S][C]; NULL = skip */
    double *virial;  /* device, [S][C][9]; needs QNEP_BATCH_VIRIAL at prepare; NULL = skip */
    float *forces;   /* device, [C][3][n_total]; NULL = skip */
    float *charges;  /* device, [C][n_total], corrected scaled charges q~'; NULL = skip */
} qnep_batch_outputs;

/* bytes of device workspace for the batch and up to max_candidates candidates */
qnep_status qnep_batch_workspace_size(const void *model, const qnep_es_params *es, const qnep_batch *batch,
                                      int32_t max_candidates, size_t *bytes);
/* enqueues the parameter-independent setup (lists, k-sets, Ewald pair matrices).
   es->efield must be zero (QNEP_E_UNSUPPORTED otherwise).
   Raises QNEP_FLAG_RADIAL_OVERFLOW / QNEP_FLAG_BAD_SPECIES in the status word. */
qnep_status qnep_batch_prepare(void *model, const qnep_es_params *es, const qnep_batch *batch,
                               int32_t max_candidates, void *ws, size_t ws_bytes, void *stream);
/* thetas: device, [C][n_theta] (layout of qnep_param_count), 1 <= C <= max_candidates.
   Enqueues one persistent launch (plus one small launch for outputs->loss). */
qnep_status qnep_batch_compute(void *model, const float *thetas, int32_t n_candidates,
                               const qnep_batch_targets *targets, const qnep_batch_outputs *outputs, void *ws,
                               size_t ws_bytes, void *stream);
/* Gradient of each candidate's total loss (outputs->loss, Sec. 2.5) with respect to
   all of its parameters: d_thetas, device, [C][n_theta].  Runs the forward launch
   (filling the requested outputs), the loss reduction and a second persistent launch
   that differentiates the energy, force and total-charge terms in reverse mode, the
   force term through the descriptor tangents and the network's second derivatives
   (exact up to rounding; FP32 network arithmetic in the adjoint whatever the forward
   precision).  Where an RMSE term is zero its gradient is taken as zero.  Needs
   QNEP_BATCH_GRADIENT at prepare. */
qnep_status qnep_batch_gradient(void *model, const float *thetas, int32_t n_candidates,
                                const qnep_batch_targets *targets, const qnep_batch_outputs *outputs,
                                float *d_thetas, void *ws, size_t ws_bytes, void *stream);
/* One generation of the separable natural evolution strategy the paper trains with
   (Sec. 2.5; Schaul, Glasmachers and Schmidhuber 2011) on the prepared batch:
     1. population   thetas[k] = mu + sigma * noise[k]   (k = 0..C-1)
     2. fitness      qnep_batch_compute on the population; outputs->loss[k] (required)
                     receives each member's loss (the other outputs as in that call)
     3. update       members ranked by loss (ties by index), rank utilities
                     u_r = max(0, ln(C/2+1) - ln r) / sum_j max(0, ln(C/2+1) - ln j) - 1/C,
                     mu += eta_mu sigma sum_k u_k noise[k],
                     sigma *= exp(eta_sigma / 2 sum_k u_k (noise[k]^2 - 1))
   mu, sigma: device FP32 [n_theta], updated in place.  noise: device FP32 [C][n_theta],
   standard-normal draws chosen by the caller (the library draws no random numbers).
   thetas: device FP32 [C][n_theta], receives the population.  2 <= C <= min(1024,
   max_candidates of the prepare call).  eta_sigma <= 0 selects the published default
   (3 + ln d) / (5 sqrt d), d = n_theta.  Asynchronous like qnep_batch_compute. */
qnep_status qnep_snes_generation(void *model, float *mu, float *sigma, const float *noise, int32_t n_candidates,
                                 double eta_mu, double eta_sigma, const qnep_batch_targets *targets,
                                 const qnep_batch_outputs *outputs, float *thetas, void *ws, size_t ws_bytes,
                                 void *stream);

/* Autotuner: times the lanes-per-atom choice for each structure-size class (fewer
   than 48, 48-127, 128-383, 384 or more atoms) over {1, 2, 4, 8, 16} and then the
   number of resident workgroups per compute unit over {1, 2, 3, 4}, on the prepared
   batch; keeps the fastest choice in the model.  Synchronizes the stream; the
   outputs hold the result of the last timed run.  choice (may be NULL) receives
   {lanes class 0..3, workgroups per compute unit}. */
qnep_status qnep_batch_tune(void *model, const float *thetas, int32_t n_candidates,
                            const qnep_batch_targets *targets, const qnep_batch_outputs *outputs, void *ws,
                            size_t ws_bytes, void *stream, int32_t *choice);

const char *qnep_status_string(qnep_status s);
const char *qnep_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QNEP_H */
