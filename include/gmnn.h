/*
 * gmnn.h -- C ABI of the MI355X (gfx950) Gaussian Moment Neural Network
 * energy/force library.
 *
 * The method is the Gaussian Moment Neural Network potential of the Apax
 * paper (arXiv 2505.22168):
 *   Section 2.1, eq. (energy_sum):   E = sum_i E_i(G_i)
 *   Section 2.1, eq. (basis_fn):     Psi_{i,L,s} = sum_{j != i} R_{Zi,Zj,s}(r_ij) rhat_ij^{(x)L}
 *                                    with R built from equidistant Gaussians
 *                                    mixed by species-pair coefficients beta
 *   Section 2.1, eq. (contraction):  G_i = full tensor contractions of Psi, L <= 3
 *   Section 2.1, eq. (scale_shift):  E_i = sigma_{Z_i} NN(G_i) + mu_{Z_i}
 *   Section 3.3:                     forces and virials are gradients of E
 *                                    w.r.t. positions and strain
 *   Section 2.2, eq. (uncertainty), eq. (jacobian): shallow ensembles share
 *                                    everything but the last layer
 *   Section 3.5:                     periodic cells narrower than twice the
 *                                    cutoff need several images per neighbour
 *
 * Conventions
 *   Units: Angstrom, eV, eV/A, eV/A^3.  F = -dE/dx.  stress = (1/V) dE/dstrain.
 *   All array pointers in the structs below are DEVICE pointers unless the
 *   field name ends in _host.  Every buffer is owned by the caller; the
 *   library never allocates or frees device memory and keeps no global state.
 *   Work is enqueued on the given HIP stream (NULL = default stream) and is
 *   complete in stream order; argument and shape checks are synchronous and
 *   return a negative status without enqueuing anything.  Device-side
 *   conditions (list capacity overflow, non-finite input, coincident atoms)
 *   are OR-ed into a device status word (GMNN_FLAG_*), never trapped.
 */
#ifndef GMNN_H_
#define GMNN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gmnn_status;
#define GMNN_OK 0
#define GMNN_ERR_INVALID_ARG -1   /* null pointer, bad size, bad flag */
#define GMNN_ERR_CAPACITY -2      /* neighbour capacity too small (SYNC mode) */
#define GMNN_ERR_UNSUPPORTED -3   /* shape/model outside what the kernels handle */
#define GMNN_ERR_HIP -4           /* a HIP runtime call failed */
#define GMNN_ERR_DEVICE_FLAG -5   /* a device status flag was raised (SYNC mode) */
#define GMNN_ERR_WORKSPACE -6     /* workspace smaller than gmnn_workspace_bytes() */
#define GMNN_ERR_SCRATCH_LIMIT -7 /* input too large for gmnn_energy_forces_noalloc's fixed scratch */

/* bits of the device status word */
#define GMNN_FLAG_CAPACITY 1u      /* more pairs than nl->capacity */
#define GMNN_FLAG_NONFINITE 2u     /* a non-finite position */
#define GMNN_FLAG_COINCIDENT 4u    /* two atoms (or images) at zero distance */
#define GMNN_FLAG_ROW_TOO_LONG 8u  /* an atom with more than GMNN_MAX_ROW neighbours */
#define GMNN_FLAG_SHIFT_RANGE 16u  /* an image vector outside [-127, 127] */

#define GMNN_MAX_ROW 1024          /* neighbours per atom handled by the list build */

/* flags of gmnn_energy_forces / gmnn_backward */
#define GMNN_PREC_FP32 0u          /* network products in FP32 (MFMA f32) */
#define GMNN_PREC_BF16 1u          /* network products in BF16 on MFMA, FP32 accumulate */
#define GMNN_WANT_STRESS 2u        /* fill outputs->stress */
#define GMNN_WANT_FORCE_VAR 4u     /* fill outputs->force_var (one backward per head) */
#define GMNN_SYNC 8u               /* synchronise and turn device flags into a status */
#define GMNN_BACKWARD_LANES16 16u  /* gmnn_backward: 16 lanes per atom row in its pair kernels whatever
                                      the atom count (built-in: 64 below 8192 atoms, 16 from there) */
#define GMNN_BACKWARD_PER_HEAD 32u /* gmnn_backward: per-head upstream gradients (shallow-ensemble losses) */

/* A ragged batch of B structures with N atoms in total (Section 2.1: a
 * configuration is positions R and atomic numbers Z; Section 3.5: with a
 * periodic cell).  Structure b owns atoms atom_ptr[b] .. atom_ptr[b+1]-1. */
typedef struct gmnn_system {
  int32_t n_structs;            /* B >= 1 */
  int32_t n_atoms;              /* N >= 0 */
  const int64_t* atom_ptr;      /* [B+1] device, atom_ptr[0] = 0, non-decreasing */
  const int64_t* atom_ptr_host; /* [B+1] host mirror (sizes the launches) */
  const float* pos;             /* [N,3] device, Cartesian positions; need not lie in the cell */
  const int32_t* species;       /* [N] device, species index in [0, n_species) */
  const double* cell;           /* [B,3,3] device, lattice vectors as rows */
  const double* cell_host;      /* [B,3,3] host mirror (sizes the cell grids) */
  const uint8_t* pbc;           /* [B,3] device, 1 = periodic along that axis */
  const uint8_t* pbc_host;      /* [B,3] host mirror */
} gmnn_system;

/* Neighbour list in CSR form, canonical order: rows by centre atom i, inside a
 * row by (j, Sx, Sy, Sz) ascending.  A pair p = (i, j, S) means the neighbour
 * x_j + S . h_b of x_i.  All arrays device, caller-allocated. */
typedef struct gmnn_neighbors {
  int64_t capacity;       /* length of j, shift, rev */
  int64_t* row_ptr;       /* [N+1] */
  int32_t* j;             /* [capacity] neighbour atom (global index) */
  int32_t* shift;         /* [capacity] S packed as int8 x3: Sx | Sy<<8 | Sz<<16 */
  int32_t* rev;           /* [capacity] index of the reverse pair (j, i, -S) */
  int32_t* atom_struct;   /* [N] structure of every atom */
  int64_t* n_pairs;       /* [1] total pairs (written even when above capacity) */
  uint32_t* status;       /* [1] GMNN_FLAG_* bits, OR-ed; clear before a build */
  float cutoff;           /* list cutoff the list was built with (r_cut + skin) */
} gmnn_neighbors;

/* Model hyperparameters and parameters (Section 2.1).  Device arrays in FP32.
 * F = number of invariants = S + 3 S(S+1)/2 + S(S+1)(S+2)/6 + S^2(S+1) + S^3
 * (360 for S = 5); the kernels support S = 5, K <= 8, H1, H2 multiples of 64
 * up to 512, n_heads <= 16, n_species <= 16. */
typedef struct gmnn_model {
  int32_t n_species;
  int32_t n_radial;       /* S */
  int32_t n_basis;        /* K */
  int32_t hidden1;        /* H1 */
  int32_t hidden2;        /* H2 */
  int32_t n_heads;        /* shallow-ensemble heads (Section 2.2) */
  float r_min;            /* first Gaussian centre */
  float r_cut;            /* cutoff radius */
  float gamma;            /* Gaussian width: g_k = exp(-gamma (r - mu_k)^2) */
  float psi_scale;        /* prefactor of the moment sums; the Gaussian centres
                             are mu_k = r_min + k (r_cut - r_min)/(K - 1) */
  const float* beta;      /* [n_species, n_species, S, K] */
  const float* W1;        /* [F, H1] */
  const float* b1;        /* [H1] */
  const float* W2;        /* [H1, H2] */
  const float* b2;        /* [H2] */
  const float* W3;        /* [H2, n_heads] */
  const float* b3;        /* [n_heads] */
  const float* scale;     /* [n_species] sigma_Z */
  const float* shift;     /* [n_species] mu_Z */
  void* packed;           /* device buffer of gmnn_model_packed_bytes() bytes,
                             filled by gmnn_model_prepare(): MFMA-ordered FP32
                             and BF16 copies of W1, W2 and their transposes */
  int32_t basis;          /* radial basis functions g_k (Section 2.1 names both):
                             GMNN_BASIS_GAUSSIAN: equidistant Gaussians (r_min,
                             gamma as above); GMNN_BASIS_BESSEL: Bessel-like
                             g_n = a_n [sinc((n+1) x) + sinc((n+2) x)],
                             x = pi r / r_cut, sinc(y) = sin(y)/y,
                             a_n = (-1)^n sqrt(2) pi r_cut^(-3/2) (n+1)(n+2) /
                             sqrt((n+1)^2 + (n+2)^2) (r_min, gamma unused).
                             Both are multiplied by the cosine cutoff. */
} gmnn_model;
#define GMNN_BASIS_GAUSSIAN 0
#define GMNN_BASIS_BESSEL 1

/* Parameter gradients: FP32 device arrays with the shapes of the matching
 * gmnn_model fields; overwritten by gmnn_backward. */
typedef struct gmnn_param_grads {
  float* beta;
  float* W1;
  float* b1;
  float* W2;
  float* b2;
  float* W3;
  float* b3;
  float* scale;
  float* shift;
} gmnn_param_grads;

/* Results.  energy[b, m] is the total energy of structure b under head m
 * (eq. energy_sum, summed in FP64).  forces are -d(mean over heads of E)/dx
 * (eq. jacobian).  Optional fields may be NULL unless requested. */
typedef struct gmnn_outputs {
  double* energy;         /* [B, n_heads] */
  float* forces;          /* [N, 3] */
  double* stress;         /* [B, 3, 3], with GMNN_WANT_STRESS */
  double* energy_var;     /* [B] population variance over heads, may be NULL */
  float* force_var;       /* [N] (1/M) sum_m |F_i^m - Fbar_i|^2, with GMNN_WANT_FORCE_VAR */
  float* atomic_energy;   /* [N, n_heads] E_i^m, may be NULL */
  double* energy_mean;    /* [B] mean over heads of energy (eq. uncertainty), may be NULL */
  uint32_t* status;       /* [1] device status word, may be NULL: GMNN_FLAG_COINCIDENT for a
                           * listed pair at zero distance, GMNN_FLAG_NONFINITE for a non-finite
                           * separation, energy or force.  Bits are OR-ed and kept until the
                           * caller clears the word; with GMNN_SYNC a raised bit turns into
                           * GMNN_ERR_DEVICE_FLAG. */
  float* forces_heads;    /* [n_heads, N, 3] per-head forces F^m = -dE^m/dx (eq. jacobian), with
                           * GMNN_WANT_FORCE_VAR, may be NULL */
} gmnn_outputs;

/* ---------------------------------------------------------------------- */

/* Human-readable name of a status code (static string). */
const char* gmnn_status_string(gmnn_status s);

/* Number of invariants F for S radial channels (Section 2.1, eq. contraction;
 * eight contraction families, see gmnn_energy_forces). */
int32_t gmnn_num_features(int32_t n_radial);

/* Bytes of model->packed needed for this model's shapes. */
size_t gmnn_model_packed_bytes(const gmnn_model* m);

/* Fill model->packed from the FP32 weights (enqueued on `stream`).  Call again
 * whenever W1 or W2 change (for example after an optimiser step). */
gmnn_status gmnn_model_prepare(gmnn_model* m, void* stream);

/* Workspace bytes for op = GMNN_OP_ENERGY_FORCES / GMNN_OP_BACKWARD (sized by
 * sys->n_atoms, nl->capacity and the model).  GMNN_OP_NEIGHBORS takes the list
 * cutoff from nl->cutoff (= cutoff + skin) and ignores `m`.  Returns 0 on
 * invalid arguments. */
#define GMNN_OP_NEIGHBORS 0
#define GMNN_OP_ENERGY_FORCES 1
#define GMNN_OP_BACKWARD 2
#define GMNN_OP_FEATURES 3
size_t gmnn_workspace_bytes(int32_t op, const gmnn_model* m, const gmnn_system* sys,
                            const gmnn_neighbors* nl, uint32_t flags);

/* Workspace bytes of gmnn_build_neighbors for this system and list cutoff
 * (cell grids sized from sys->cell_host). */
size_t gmnn_neighbors_workspace_bytes(const gmnn_system* sys, float cutoff, float skin);

/* Build the periodic neighbour list (Section 3.5: cell list with as many
 * periodic images as the cell width requires; Section 2.1: all j != i within
 * the cutoff).  A pair (i, j, S) is listed iff its separation
 *   d = x_j - x_i + S . h,   computed in FP64 from the FP32 positions as
 *   dx = (x_j - x_i) + ((Sx h00 + Sy h10) + Sz h20)   (each op rounded once)
 *   d2 = (dx dx + dy dy) + dz dz
 * satisfies 0 < d2 < (cutoff + skin)^2, except (i, i, 0).  Coincident pairs
 * (d2 == 0) are left out and raise GMNN_FLAG_COINCIDENT.  Non-periodic axes
 * take S = 0.  If the pair count exceeds nl->capacity, *nl->n_pairs still
 * holds the required size and GMNN_FLAG_CAPACITY is raised; the pair arrays
 * are then not filled.  With GMNN_SYNC in `flags` the call synchronises and
 * returns GMNN_ERR_CAPACITY / GMNN_ERR_DEVICE_FLAG accordingly.
 * The workspace must hold gmnn_workspace_bytes(GMNN_OP_NEIGHBORS, ...). */
gmnn_status gmnn_build_neighbors(const gmnn_system* sys, float cutoff, float skin,
                                 gmnn_neighbors* nl, uint32_t flags,
                                 void* workspace, size_t workspace_bytes, void* stream);

/* Energies, forces and (optionally) stress, energy variance and force
 * variance of every structure.  Pairs of the list with r >= model->r_cut
 * contribute nothing (a list built with a skin can be reused).  Steps:
 *   pair geometry, Gaussian basis x cosine cutoff, species-pair mixing and
 *   moment sums (eq. basis_fn) -> invariants (eq. contraction; families
 *   Psi0 | Psi1.Psi1 | Psi2:Psi2 | Psi3:Psi3 | tr(Psi2 Psi2 Psi2) |
 *   Psi1 Psi1 Psi2 | Psi2 Psi3 Psi3 | Psi1 Psi3 Psi2) -> network and
 *   scale/shift (eq. scale_shift) -> exact gradient back to the pairs ->
 *   scatter-free force gather over the reverse pair index -> FP64
 *   per-structure sums of energy and virial.
 * GMNN_PREC_BF16 rounds the inputs of the two hidden-layer products (and of
 * their backward products) to BF16 and accumulates in FP32; everything else
 * is FP32 with FP64 per-structure sums.  The workspace must hold
 * gmnn_workspace_bytes(GMNN_OP_ENERGY_FORCES, ...). */
gmnn_status gmnn_energy_forces(const gmnn_model* m, const gmnn_system* sys,
                               const gmnn_neighbors* nl, uint32_t flags, gmnn_outputs* out,
                               void* workspace, size_t workspace_bytes, void* stream);

/* gmnn_energy_forces for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same evaluation under the built-in plan, with the workspace
 * taken from a fixed scratch array compiled into the library instead of a
 * caller buffer.  The caller still passes the model, system, list and
 * outputs.  Limit: gmnn_workspace_bytes(GMNN_OP_ENERGY_FORCES, ...) must not
 * exceed GMNN_NOALLOC_SCRATCH_BYTES (64 MiB: for example about 15,000 atoms
 * with 60 neighbours each), else GMNN_ERR_SCRATCH_LIMIT and nothing runs.
 * The call allocates nothing: each GPU holds its own copy of the array
 * (looked up on the first call on that device, with the stream's device
 * current) until the process ends.  Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU (other streams, other host
 * threads) race; calls ordered on one stream do not.  Other behaviour,
 * arguments and errors as gmnn_energy_forces. */
#define GMNN_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
gmnn_status gmnn_energy_forces_noalloc(const gmnn_model* m, const gmnn_system* sys,
                                       const gmnn_neighbors* nl, uint32_t flags, gmnn_outputs* out,
                                       void* stream);

/* ---------------------------------------------------------------------- */
/* Execution plans.  Every plan computes the same quantities (up to FP32
 * summation order); they differ in how the work is cut into kernels:
 *   FUSED  one tile kernel computes the moments, the readout and the pair
 *          backward of a tile of tile_atoms atoms (16, or 8: twice the
 *          blocks, each with half the pair and invariant work and the same
 *          network products), then one kernel gathers the forces and sums
 *          per structure (latency-bound small systems; needs <= 8 species,
 *          no force variance, every structure <= 16384 atoms);
 *   SPLIT  pair moments -> readout -> pair backward -> gather/sums, with the
 *          readout (invariants, network, their backward) either
 *            TILE    one kernel per 16 atoms, or
 *            STREAM  three kernels: invariants of 16 atoms -> network on
 *                    row tiles of 32 to 64 atoms -> invariant backward; G
 *                    and dE/dG pass through the workspace (the head-mean
 *                    backward only: not with GMNN_WANT_FORCE_VAR).
 * lanes_per_atom (8, 16, 32 or 64) is the number of lanes that share one atom's
 * neighbour row in the pair and gather kernels.  Zero fields mean "built-in
 * choice": FUSED with 64 lanes below 16384 atoms where it is allowed (else
 * SPLIT, with 64 lanes below 8192 atoms and 16 beyond), SPLIT with 16 lanes
 * and the STREAM readout from 16384 atoms on (TILE where STREAM is not
 * allowed), 8-atom fused tiles while 16-atom ones would number fewer than
 * 256 (the compute units of one MI355X). */
#define GMNN_SCHEDULE_AUTO 0
#define GMNN_SCHEDULE_FUSED 1
#define GMNN_SCHEDULE_SPLIT 2
#define GMNN_READOUT_AUTO 0
#define GMNN_READOUT_TILE 1
#define GMNN_READOUT_STREAM 2
typedef struct gmnn_plan {
  int32_t schedule;        /* GMNN_SCHEDULE_* */
  int32_t lanes_per_atom;  /* 0, 8, 16, 32 or 64 */
  int32_t readout;         /* GMNN_READOUT_* (SPLIT schedule) */
  int32_t tile_atoms;      /* FUSED schedule: atoms per tile, 0 (auto), 8 or 16;
                              must be 0 when the plan resolves to SPLIT */
} gmnn_plan;

/* Resolve the zero fields of `plan` (NULL: all zero) for these shapes and
 * flags into `resolved` (may be NULL).  GMNN_ERR_UNSUPPORTED if the plan
 * cannot run them, GMNN_ERR_INVALID_ARG for an unknown field value.  Host only. */
gmnn_status gmnn_resolve_plan(const gmnn_model* m, const gmnn_system* sys, uint32_t flags,
                              const gmnn_plan* plan, gmnn_plan* resolved);

/* 1 if the built-in plan for these shapes and flags is FUSED, 0 if SPLIT,
 * -1 on invalid arguments.  Host only. */
int32_t gmnn_uses_fused_path(const gmnn_model* m, const gmnn_system* sys, uint32_t flags);

/* gmnn_energy_forces under an explicit plan (NULL: the built-in one). */
gmnn_status gmnn_energy_forces_plan(const gmnn_model* m, const gmnn_system* sys,
                                    const gmnn_neighbors* nl, uint32_t flags, const gmnn_plan* plan,
                                    gmnn_outputs* out, void* workspace, size_t workspace_bytes,
                                    void* stream);

/* Uncertainty-driven bias (Section 2.3, eq. udd) on the shallow ensemble's
 * energy variance: per structure b with N_b atoms, M heads and population
 * variance var_b of the head energies,
 *   E_bias,b = A [exp(-var_b / (M N_b B^2)) - 1],
 * and the forces (and stress) become those of Ebar + E_bias:
 *   F = -sum_m c_m dE^m/dx,  c_m = 1/M + dE_bias/dvar * 2 (E^m - Ebar) / M.
 * The evaluation runs the split schedule in two passes: the energies of every
 * head first (readout forward only, FP64 sums per structure), then the
 * backward with the weights c_m (one weighted backward; with
 * GMNN_WANT_FORCE_VAR the per-head backwards, whose forces give both the
 * variance of the unbiased head forces and sum_m c_m F^m).  out->energy,
 * energy_mean and energy_var stay unbiased. */
typedef struct gmnn_udd {
  float A;               /* bias strength, eV (finite) */
  float B;               /* bias width, eV (> 0) */
  double* bias_energy;   /* [B] E_bias per structure (device), may be NULL */
} gmnn_udd;

/* gmnn_energy_forces with the uncertainty-driven bias (needs n_heads >= 2;
 * same workspace, flags and outputs).  plan: NULL for the built-in split
 * plan, else a SPLIT (or AUTO) plan whose other fields are honoured; FUSED
 * gives GMNN_ERR_UNSUPPORTED. */
gmnn_status gmnn_energy_forces_udd(const gmnn_model* m, const gmnn_system* sys,
                                   const gmnn_neighbors* nl, uint32_t flags, const gmnn_plan* plan,
                                   const gmnn_udd* udd, gmnn_outputs* out, void* workspace,
                                   size_t workspace_bytes, void* stream);

/* gmnn_energy_forces_plan with a hipEvent_t recorded on `stream` right before
 * and right after each kernel stage, for profiling: stage_events[2k] /
 * [2k+1] bracket stage k =
 *   0 pair moments (FUSED: the tile kernel, which also covers stages 1-4)
 *   1 invariants (streamed readout; the tile readout's one kernel covers 1-3)
 *   2 network forward and backward (streamed readout)
 *   3 invariant backward (streamed readout)
 *   4 pair backward
 *   5 force gather + per-structure reductions
 * (GMNN_TIMED_EVENTS = 12 events, created by the caller with hipEventCreate;
 * NULL: none).  A stage a plan does not run gets two adjacent events. */
#define GMNN_TIMED_STAGES 6
#define GMNN_TIMED_EVENTS (2 * GMNN_TIMED_STAGES)
gmnn_status gmnn_energy_forces_timed(const gmnn_model* m, const gmnn_system* sys,
                                     const gmnn_neighbors* nl, uint32_t flags, const gmnn_plan* plan,
                                     gmnn_outputs* out, void* workspace, size_t workspace_bytes,
                                     void* stream, void* const* stage_events);

/* Autotuner: runs gmnn_energy_forces under every plan these shapes support
 * (2 warm-up calls, then `reps` calls each bracketed by hipEvents on
 * `stream`), and returns in *best the plan of least median time.  The
 * candidates and their median / minimum times in microseconds go to
 * entries[0 .. min(max_entries, *n_entries)) (entries may be NULL when
 * max_entries is 0).  Synchronises `stream`; `out` ends holding the results
 * of the chosen plan.  Same workspace as gmnn_energy_forces.  The choice
 * depends on the shapes (atom count, structure sizes, neighbours per atom,
 * model widths, flags), not on positions: callers may cache it per shape. */
typedef struct gmnn_tune_entry {
  gmnn_plan plan;
  float median_us;
  float min_us;
} gmnn_tune_entry;
gmnn_status gmnn_autotune(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                          uint32_t flags, gmnn_outputs* out, void* workspace, size_t workspace_bytes,
                          void* stream, int32_t reps, gmnn_plan* best, gmnn_tune_entry* entries,
                          int32_t max_entries, int32_t* n_entries);

/* Gradients of a scalar loss L(E, F) w.r.t. the model parameters and,
 * optionally, the positions, given the upstream gradients dL/dE (per
 * structure, w.r.t. the head-mean energy) and dL/dF [N,3] (Section 3.4:
 * energy + force losses; Section 3.3: forces are -dE/dx, so the force term
 * needs the mixed second derivative).  Every array of `grads` is
 * overwritten.  dL_dpos (device [N,3], may be NULL) receives
 *   dL/dx = sum_b dL/dE_b dE_b/dx + sum_k dL/dF_k . dF_k/dx,
 * the second term a Hessian-vector product of the energy along dL/dF,
 * evaluated per pair in dual numbers and gathered like the forces.  With
 * GMNN_PREC_BF16 the network products of the
 * forward and reverse passes (primal and tangent rows) run in BF16 on MFMA
 * with FP32 accumulation, the operands rounded as in gmnn_energy_forces; the
 * products that form the weight gradients split each FP32 operand into a
 * BF16 high and low part and add the three products hi.hi + hi.lo + lo.hi
 * (about 16 significant bits per product).  Without it everything is FP32.
 *
 * With GMNN_BACKWARD_PER_HEAD the upstream gradients are per head, as a loss
 * over the members of a shallow ensemble needs (Section 2.2, eq. nll):
 * dL_dE is [B, n_heads] (dL/dE_b^m) and dL_dF [n_heads, N, 3] (dL/dF^m with
 * F^m = -dE^m/dx, eq. jacobian).  The call runs one double backward per
 * head; the gradients of the shared parameters (beta, W1, b1, W2, b2, scale,
 * shift) and of the positions are added over the heads in head order,
 * W3[:, m] and b3[m] take head m's alone.
 *
 * The workspace must hold gmnn_workspace_bytes(GMNN_OP_BACKWARD, ..., flags)
 * for the same flags.  Recomputes the forward pass itself. */
gmnn_status gmnn_backward(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                          const double* dL_dE, const float* dL_dF, uint32_t flags,
                          gmnn_param_grads* grads, float* dL_dpos,
                          void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Shallow-ensemble training step (Section 2.2, eq. nll; Section 3.4).
 *
 * Loss terms over the M heads' predictions.  The energy term scores x_b^m =
 * E_b^m (or E_b^m / N_b with energy_per_atom) against x_b^ref, the force
 * term every Cartesian component F_ia^m of the per-head forces
 * (outputs->forces_heads) against F_ia^ref, through
 *   GMNN_LOSS_MSE   (xbar - x_ref)^2
 *   GMNN_LOSS_NLL   (1/2) [(xbar - x_ref)^2 / s2 + log(2 pi s2)]
 *   GMNN_LOSS_CRPS  s [z (2 Phi(z) - 1) + 2 phi(z) - 1/sqrt(pi)],  z = |xbar - x_ref| / s
 * where xbar is the mean over the heads and s2 = s^2 their population
 * variance (1/M) plus var_floor;
 *   L = w_energy (1/B) sum_b l_b + w_force (1/(3N)) sum_{i,a} l_ia
 * (with energy_per_atom a structure without atoms adds nothing to the
 * energy term and gets zero gradients; B still counts it).
 * gmnn_ensemble_loss writes loss[0] (energy term) and loss[1] (force term)
 * (device FP64, fixed-order sums) and the per-head gradients dL_dE [B, M]
 * (FP64) and dL_dF [M, N, 3] (FP32) that gmnn_backward takes with
 * GMNN_BACKWARD_PER_HEAD; dL_dE or dL_dF may be NULL.  All arrays device.
 * energy [B, M] FP64 and forces_heads [M, N, 3] FP32 as gmnn_energy_forces
 * writes them; energy_ref [B] FP64, forces_ref [N, 3] FP32.  Workspace:
 * gmnn_loss_workspace_bytes(sys).  Non-finite inputs propagate into the
 * outputs (no device flag). */
#define GMNN_LOSS_MSE 0
#define GMNN_LOSS_NLL 1
#define GMNN_LOSS_CRPS 2
typedef struct gmnn_loss {
  int32_t energy_kind;      /* GMNN_LOSS_* */
  int32_t force_kind;       /* GMNN_LOSS_* */
  int32_t energy_per_atom;  /* 1: the energy term scores E_b / N_b */
  int32_t reserved;
  double w_energy;          /* weight of the energy term (0 drops it) */
  double w_force;           /* weight of the force term (0 drops it) */
  double var_floor;         /* added to every variance (units of x^2); NLL and CRPS need
                               s2 > 0, which equal heads break without it; with one head a
                               weighted NLL or CRPS term and var_floor 0 is INVALID_ARG */
} gmnn_loss;
size_t gmnn_loss_workspace_bytes(const gmnn_system* sys);
gmnn_status gmnn_ensemble_loss(const gmnn_loss* spec, const gmnn_system* sys, int32_t n_heads,
                               const double* energy, const float* forces_heads, const double* energy_ref,
                               const float* forces_ref, double* loss, double* dL_dE, float* dL_dF,
                               void* workspace, size_t workspace_bytes, void* stream);

/* One Adam update (Kingma & Ba, Algorithm 1) of every parameter array of m,
 * in place, with one learning rate per parameter group (Section 3.4:
 * separate rates for the embedding, the neural network, the scales and the
 * shifts; a rate of 0 freezes its group):
 *   m1 = beta1 m1 + (1 - beta1) g;  m2 = beta2 m2 + (1 - beta2) g^2;
 *   theta -= lr_group (m1 / (1 - beta1^t)) / (sqrt(m2 / (1 - beta2^t)) + eps).
 * grads, m1, m2: device FP32 arrays shaped like the parameters (m1 and m2
 * zero before the first step, updated in place).  The arrays m points to
 * must be writable.  The packed copies (m->packed) are rebuilt afterwards,
 * as gmnn_model_prepare does, so the next evaluation sees the new weights.
 * FP32 arithmetic; the bias corrections are formed on the host in FP64. */
#define GMNN_GROUP_EMBEDDING 0  /* beta */
#define GMNN_GROUP_NN 1         /* W1, b1, W2, b2, W3, b3 */
#define GMNN_GROUP_SCALE 2      /* scale */
#define GMNN_GROUP_SHIFT 3      /* shift */
typedef struct gmnn_adam {
  double lr[4];             /* learning rate per GMNN_GROUP_* */
  double beta1, beta2, eps;
  int64_t step;             /* t >= 1, the index of this update */
} gmnn_adam;
gmnn_status gmnn_adam_step(gmnn_model* m, const gmnn_param_grads* grads, gmnn_param_grads* m1,
                           gmnn_param_grads* m2, const gmnn_adam* opt, void* stream);

/* Learning-rate schedules (Section 3.4): the factor every group's base rate
 * is multiplied by at a (0-based) step.
 *   GMNN_LR_CONSTANT  1
 *   GMNN_LR_LINEAR    1 + (end_factor - 1) min(step, total_steps) / total_steps
 *   GMNN_LR_COSINE    cyclic cosine: decay_factor^c (1 + cos(pi r / period)) / 2
 *                     with c, r = step div/mod period
 * Host function; NaN for an invalid schedule. */
#define GMNN_LR_CONSTANT 0
#define GMNN_LR_LINEAR 1
#define GMNN_LR_COSINE 2
typedef struct gmnn_lr_schedule {
  int32_t kind;
  int32_t reserved;
  int64_t total_steps;      /* GMNN_LR_LINEAR, >= 1 */
  double end_factor;        /* GMNN_LR_LINEAR */
  int64_t period;           /* GMNN_LR_COSINE, >= 1 */
  double decay_factor;      /* GMNN_LR_COSINE */
} gmnn_lr_schedule;
double gmnn_lr_factor(const gmnn_lr_schedule* s, int64_t step);

/* ---------------------------------------------------------------------- */
/* Batch active learning (Section 2.4).
 *
 * Last-layer gradient features (eq. lastlayer): phi[b] = the gradient of
 * structure b's head-mean energy w.r.t. one head's last-layer weights and
 * bias,
 *   phi[b] = (1/M) [ sum_{i in b} sigma_Zi h2_i ,  sum_{i in b} sigma_Zi ],
 * H2 + 1 values per structure (FP64, summed in atom order), h2_i the second
 * hidden layer's activations of atom i (the network as in
 * gmnn_energy_forces, GMNN_PREC_BF16 honoured).  The full gradient repeats
 * this block once per head, which scales every distance by sqrt(M) and
 * leaves the selection below unchanged.  phi: device [B][H2 + 1].
 * Workspace: gmnn_workspace_bytes(GMNN_OP_FEATURES, ...).  Runs the readout
 * forward only (split schedule). */
gmnn_status gmnn_last_layer_features(const gmnn_model* m, const gmnn_system* sys,
                                     const gmnn_neighbors* nl, uint32_t flags, double* phi,
                                     void* workspace, size_t workspace_bytes, void* stream);

/* Greedy maximum-distance selection (eq. maxdist): n_select indices of
 * pool[n_pool][dim] (device, FP64), each the pool entry (not yet selected)
 * whose smallest Euclidean distance to the training entries train[n_train]
 * [dim] and to the entries selected before it is largest; ties go to the
 * smaller index.  With no training entries the first pick is the entry of
 * largest norm (reading: the paper's minimum runs over an empty set there).
 * selected: device [n_select] int32, in selection order.  Distances in FP64.
 * Workspace: gmnn_select_workspace_bytes(n_pool).  3 n_select + 1 launches,
 * no host synchronisation. */
size_t gmnn_select_workspace_bytes(int64_t n_pool);
gmnn_status gmnn_select_max_distance(const double* pool, int64_t n_pool, int32_t dim, const double* train,
                                     int64_t n_train, int32_t n_select, int32_t* selected,
                                     void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Molecular dynamics on the device (Section 3.5: the whole simulation loop
 * runs on the GPU; the neighbour list carries a skin).  NVE velocity Verlet:
 *   v += dt/2 k_u F/m;  x += dt v;  rebuild the list if some atom moved more
 *   than skin/2 since the last build (decided on the device);  F = forces(x);
 *   v += dt/2 k_u F/m,     k_u = 9.648533e-3 A/fs^2 per eV/(A amu).
 * The steps write the positions sys->pos in place.  All arrays device. */
typedef struct gmnn_md {
  float dt;               /* time step, fs */
  float skin;             /* list skin, A (the list cutoff is r_cut + skin) */
  const float* inv_mass;  /* [N] 1/mass, 1/amu */
  float* vel;             /* [N,3] velocities, A/fs (updated) */
  float* forces;          /* [N,3] forces at the current positions, eV/A (updated) */
  double* energy;         /* [B, n_heads] potential energies at the current positions */
  float* ref_pos;         /* [N,3] positions at the last list build */
  uint32_t* disp;         /* [1] largest squared displacement of the step (scratch word) */
  /* shallow-ensemble options (Section 2.3, Section 3.5); all zero: off */
  const gmnn_udd* udd;    /* uncertainty-driven bias on the forces (gmnn_energy_forces_udd), may be NULL */
  int32_t var_every;      /* with GMNN_WANT_FORCE_VAR in flags: the per-head force variance on every
                             var_every-th step of a call (or of a captured graph) only, the cheap
                             head-mean forces on the others (mode switching at a dump interval) */
  float* force_var;       /* [N] written on those steps */
  double* energy_var;     /* [B] energy variance over heads at every step, may be NULL */
} gmnn_md;

/* Workspace of gmnn_md_init / _steps / _graph_create (list build and
 * energy/forces); nl->cutoff must already hold r_cut + skin.  flags: the
 * precision bit and GMNN_WANT_FORCE_VAR (with md->var_every > 0).  Returns 0
 * on invalid arguments. */
size_t gmnn_md_workspace_bytes(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                               uint32_t flags);

/* Build the list (recording ref_pos), compute forces and energies at the
 * current positions, clear md->disp.  Call before the first step and before
 * capturing a graph. */
gmnn_status gmnn_md_init(const gmnn_model* m, const gmnn_system* sys, gmnn_neighbors* nl, const gmnn_md* md,
                         uint32_t flags, void* workspace, size_t workspace_bytes, void* stream);

/* n_steps steps enqueued on `stream` (no host synchronisation).  A list that
 * outgrows nl->capacity during a rebuild raises GMNN_FLAG_CAPACITY in
 * nl->status and is left empty; the caller checks the status between calls,
 * re-sizes and restarts from saved state. */
gmnn_status gmnn_md_steps(const gmnn_model* m, const gmnn_system* sys, gmnn_neighbors* nl, const gmnn_md* md,
                          uint32_t flags, int32_t n_steps, void* workspace, size_t workspace_bytes,
                          void* stream);

/* Capture n_steps steps into a HIP graph (on an internal stream; every
 * pointer of the arguments is baked in); replay with gmnn_md_graph_launch on
 * any stream; release with gmnn_md_graph_destroy.  The graph handle is host
 * memory owned by the caller. */
gmnn_status gmnn_md_graph_create(const gmnn_model* m, const gmnn_system* sys, gmnn_neighbors* nl,
                                 const gmnn_md* md, uint32_t flags, int32_t n_steps, void* workspace,
                                 size_t workspace_bytes, void** graph_out);
gmnn_status gmnn_md_graph_launch(void* graph, void* stream);
void gmnn_md_graph_destroy(void* graph);

/* HIP graph of n_evals back-to-back evaluations (gmnn_energy_forces_plan
 * with these arguments), for callers that evaluate the same buffers over
 * and over (serving loops over fixed-size batches whose positions are
 * rewritten in place): one graph launch replaces n_evals x (2 to 6) kernel
 * launches.  The graph reads every buffer when it runs (new contents of
 * sys->pos or the parameters are used; their addresses are baked in).  Runs
 * one eager evaluation on an internal stream first (argument checks; it does
 * not wait for other streams: the inputs must be ready), then captures;
 * GMNN_SYNC is not allowed.  Replay with gmnn_graph_launch on
 * any stream; release with gmnn_graph_destroy (host memory of the handle and
 * the graph).  The MD graphs of gmnn_md_graph_create take the same two calls. */
gmnn_status gmnn_energy_forces_graph_create(const gmnn_model* m, const gmnn_system* sys,
                                            const gmnn_neighbors* nl, uint32_t flags, const gmnn_plan* plan,
                                            gmnn_outputs* out, void* workspace, size_t workspace_bytes,
                                            int32_t n_evals, void** graph);
gmnn_status gmnn_graph_launch(void* graph, void* stream);
void gmnn_graph_destroy(void* graph);

#ifdef __cplusplus
}
#endif

#endif /* GMNN_H_ */
