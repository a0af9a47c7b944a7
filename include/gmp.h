/*
 * gmp.h -- C ABI of the MI355X (gfx950) Gaussian Multipole feature library.
 *
 * The method is the one GMP-Featurizer computes (arXiv 2303.12980): for every
 * centre atom i, every probe (angular order l of a solid Maxwell-Cartesian
 * spherical harmonic, Gaussian radial width sigma) and every neighbour j
 * within the sigma-dependent cutoff (periodic images included), the
 * closed-form overlap of the probe with each Gaussian primitive
 * B_k exp(-beta_k |r - R_j|^2) of the neighbour's density is accumulated into
 * multipole components mu_{i,l,sigma,abc}; the feature is the weighted
 * root-sum-square F_{i,l,sigma} = sqrt(sum_abc l!/(a!b!c!) mu^2)
 * ("Examples": probe set = Cartesian product of orders and sigmas, order-major;
 * cutoff inferred from the overlap threshold; derivatives with respect to the
 * atom positions on request).  Order -1 is the local density at the centre,
 * rho_i = sum_j sum_k B_k exp(-beta_k |d|^2) ("Examples": it takes no sigma
 * and gives one feature), the sigma -> 0 limit of the order-0 probe; its
 * feature is |rho_i|.
 *
 * Cutoff slots: every sigma has its own cutoff, and order -1 adds one more
 * slot after the sigmas, rc_{-1}^2 = max_{e,k} ln(|B|/tau)/beta (the
 * sigma -> 0 limit of the per-sigma rule).  n_slots = n_sigmas, plus 1 when
 * order -1 is requested; per-sigma arrays below are per slot.
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers owned by the caller unless marked [host].
 *  - Nothing is allocated on the device by any entry point; scratch memory
 *    is the caller's workspace `ws` of `ws_bytes` bytes (see
 *    gmp_workspace_size).  The plan owns small constant tables that it
 *    allocates once in gmp_plan_create.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *    Entry points return after enqueueing, except where a host-visible
 *    result is requested (n_pairs of gmp_build_neighbors).
 *  - Errors are reported by status codes only; nothing aborts or prints.
 *    gmp_last_error() returns a thread-local message for the last non-OK
 *    status.  Device-side conditions (non-finite coordinates, image shifts
 *    out of range, list overflow in no-sync mode) are recorded in a status
 *    word inside `ws` and reported by gmp_build_neighbors when it syncs, or
 *    by gmp_check_status.
 */
#ifndef GMP_H
#define GMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GMP_OK = 0,
  GMP_E_INVALID = 1,      /* bad argument: null pointer, order outside -1..4, sigma <= 0, beta <= 0, ... */
  GMP_E_UNSUPPORTED = 2,  /* valid but outside what the kernels handle (documented limits) */
  GMP_E_CELL = 3,         /* singular lattice for a structure with a periodic axis */
  GMP_E_CAPACITY = 4,     /* neighbour capacity too small; required count returned */
  GMP_E_NONFINITE = 5,    /* non-finite coordinate or lattice entry */
  GMP_E_HIP = 6,          /* a HIP runtime call failed */
  GMP_E_NOMEM = 7,        /* host allocation or workspace too small */
  GMP_E_STALE = 8,        /* a no-sync rebuild met a single (shell, species) bucket longer than the
                             largest in-LDS sort (the device's workgroup LDS): that centre holds
                             placeholder entries; a synchronous build reports such a list as
                             GMP_E_UNSUPPORTED */
} gmp_status;

/* Arithmetic of the overlap kernels.
 *  GMP_FP64:              every step in FP64 (exp in FP64).
 *  GMP_FP32_COMPENSATED:  pair terms (displacement, monomials, exponentials,
 *                         radial sums, products) in FP32; per-lane component
 *                         accumulation as an FP32 (hi, lo) pair updated with
 *                         an error-free two-sum; cross-lane reduction, the
 *                         moment-to-component map and the norm in FP64.
 *  GMP_FP32_WIDE:         exponentials and radial sums in FP32; monomials of
 *                         the FP64 displacement and the per-lane accumulation
 *                         in FP64 (one FP64 fma per term: on gfx950 FP64 FMA
 *                         issues at the non-packed FP32 rate, so widening is
 *                         cheaper than a two-sum and loses nothing).
 * In every mode the lattice wrap, image shifts and distances are FP64.
 * Features are float for both FP32 modes and double for GMP_FP64; the
 * adjoint of both FP32 modes evaluates its pair terms in FP32. */
typedef enum { GMP_FP64 = 0, GMP_FP32_COMPENSATED = 1, GMP_FP32_WIDE = 2 } gmp_precision;

typedef struct gmp_plan gmp_plan; /* opaque, immutable after creation */

/* [host] probe set and density primitives; mirrors the featurizer's
 * hyper-parameter dictionary ("Examples": orders, sigmas, pseudopotential
 * primitives, overlap_threshold).  Copied by gmp_plan_create. */
typedef struct {
  int32_t n_orders;              /* 1..6 */
  const int32_t *orders;         /* distinct, each in -1..4 (-1: local density); output order as given */
  int32_t n_sigmas;              /* 1..16 (1..15 with order -1: at most 16 cutoff slots) */
  const double *sigmas;          /* Angstrom, > 0; output order as given */
  int32_t n_elements;            /* 1..64 */
  const int32_t *prim_offsets;   /* [n_elements+1], ascending, prim_offsets[0] = 0; <= 16 per element */
  const double *B;               /* [prim_offsets[n_elements]] primitive weights (any sign) */
  const double *beta;            /* [prim_offsets[n_elements]] exponents, > 0 (1/Angstrom^2) */
  double overlap_threshold;      /* tau > 0: rc(sigma)^2 = max_{e,k} ln(|A0|/tau)/gamma */
  int32_t screening;             /* 0: every primitive of a neighbour inside the slot cutoff contributes.
                                    1: per-primitive screening, a faster variant of the truncation:
                                    primitive k of element e contributes to slot s only where its own
                                    l = 0 overlap reaches tau, (float)q <= (float)(ln(|A0|/tau)/gamma)
                                    (never when |A0| <= tau; density slot: A0 = B, gamma = beta); each
                                    skipped radial term is below tau */
  int32_t radial_intervals;      /* 0: the radial factors c_{l,s,e}(q) = sum_k A exp(-gamma q) are
                                    evaluated exactly.  16..65536 (FP32 precisions, no screening):
                                    a faster variant for elements with many primitives, the
                                    forward reads c from a table instead: per (slot, element,
                                    order) a cubic Hermite interpolant of c in r = sqrt(q) on
                                    radial_intervals equal intervals of [0, rc(slot)], whose
                                    error is at most h^4/32 sum_k gamma_k^2 |A_k| (h the interval
                                    width; the fourth r-derivative of exp(-gamma r^2) is at most
                                    12 gamma^2); the adjoint and the Jacobian keep the exact
                                    factors */
} gmp_probe_desc;

/* A packed batch of structures (CSR over atoms); mirrors the featurizer's
 * native structure dictionary (lattice vectors, positions, atom types). */
typedef struct {
  int32_t n_structs;
  int64_t n_atoms;
  const int64_t *atom_offsets;   /* [n_structs+1]; structure s owns atoms [off[s], off[s+1]) */
  const double *x, *y, *z;       /* [n_atoms] Cartesian coordinates, Angstrom (SoA) */
  const int32_t *species;        /* [n_atoms] element index 0..n_elements-1 */
  const double *cell;            /* [n_structs*9]; row m (entries 3m..3m+2) is lattice vector a_m */
  const uint8_t *pbc;            /* [n_structs]; bit k set = periodic along a_k; 0 = isolated
                                    (then the cell is ignored and may be zero) */
  const double *occupancy;       /* [n_atoms] fractional site occupancies, or NULL (all 1):
                                    disordered structures ("Overview"); atom j's density is
                                    scaled by occupancy[j], a site shared by several species is
                                    one entry per species at the same position; cutoffs and
                                    neighbour lists do not depend on it; must be finite */
  /* Reference points ("Overview": features at any set of positions inside
   * each structure instead of at its atoms).  point_offsets == NULL: the
   * centres are the atoms.  Otherwise the centres are the n_points points
   * (points of structure s: [point_offsets[s], point_offsets[s+1])), every
   * per-centre array below is per point, the neighbours are the atoms, a
   * point has no self term of its own, and the backward differentiates
   * with respect to atoms and points. */
  int64_t n_points;
  const int64_t *point_offsets;  /* [n_structs+1] or NULL */
  const double *px, *py, *pz;    /* [n_points] Cartesian coordinates, Angstrom (SoA) */
} gmp_batch;

/* Neighbour lists in canonical order; n_centres = n_atoms, or n_points
 * with reference points, and n_total = n_atoms (+ n_points).  The lists are
 * stored in list-slot order: slot k holds the list of centre order[k] and
 * slot[i] is the slot of centre i.  Atom centres are ordered by the cell list
 * (by spatial bin, by atom index within a bin), so the lists of atoms that
 * are near in space are near in memory; reference points keep their own
 * order.  The list of centre i, entries [offsets[k], offsets[k+1]) with
 * k = slot[i], is sorted by (shell, species of j, j, n1, n2, n3) where
 * shell(q) = number of cutoff slots with rc^2 < q, so the pairs each cutoff
 * slot uses (q <= its rc^2) are a prefix of the list.  Bucket
 * b = shell * n_elements + species holds the entries of one (shell, species).
 * Neighbour indices j, wrap and rw are by atom (and point) index. */
typedef struct {
  int64_t capacity;              /* [host] entries allocated in j, shift, reverse */
  int64_t n_pairs;               /* [host] total pairs, set by a synchronous build; a no-sync build sets
                                    it to 0 (unknown on the host): every call then bounds its pair
                                    range by the capacity and the list ends on the device.  Callers
                                    that copy this struct must not pass a count from an earlier
                                    build after a no-sync rebuild */
  int64_t *offsets;              /* [n_centres+1] per list slot */
  int32_t *j;                    /* [capacity] neighbour atom (global index) */
  int32_t *shift;                /* [capacity] bytes (n1, n2, n3, species_j), n_k signed, little endian;
                                    d = (Rw_j - Rw_i) + n1 a1 + n2 a2 + n3 a3 with wrapped positions */
  int32_t *bucket_start;         /* [n_centres*(n_slots*n_elements+1)] per list slot k: bucket starts,
                                    local to offsets[k]; the last entry is the list length */
  int32_t *sigma_end;            /* [n_centres*n_slots] per list slot: length of the prefix cutoff
                                    slot s uses, local */
  int32_t *wrap;                 /* [n_total*3] m_i: Rw_i = R_i - (m1 a1 + m2 a2 + m3 a3); atoms, then
                                    points */
  double *rw;                    /* [3*n_total] wrapped positions, SoA (x block, y block, z block) */
  int32_t *reverse;              /* [capacity] or NULL; required by gmp_features_backward.  Atoms as
                                    centres: pair index (into j / shift) of the mirror (j, i, -n);
                                    capacity must then stay below 2^31.  Reference
                                    points: the pair indices ordered by neighbour atom (stable), the
                                    order in which the backward gathers each atom's pairs */
  int64_t max_list;              /* [host] longest list of the last synchronous build (set by it); a
                                    no-sync build sizes its short-list sort for this many entries plus
                                    1/8 (0: 8,192 entries); lists that outgrow it are filled by the
                                    long-list kernel, whose sort takes the device's workgroup LDS */
  int32_t *order;                /* [n_centres] centre whose list list-slot k holds (set by the build) */
  int32_t *slot;                 /* [n_centres] list slot of centre i (set by the build) */
} gmp_neighbors;

/* Plan: validates the probe set, infers rc(sigma)^2 from the overlap
 * threshold ("Examples": the local cutoff is inferred from
 * overlap_threshold), and uploads the per (sigma, element, primitive)
 * coefficient tables.  Allocates a few KB of device memory once. */
gmp_status gmp_plan_create(const gmp_probe_desc *desc, gmp_precision precision, gmp_plan **out);
void gmp_plan_destroy(gmp_plan *plan);

/* [host] rc^2 of every cutoff slot of a probe set, without creating a
 * plan (host only, no device needed): for sigma, the squared distance beyond
 * which every primitive's l = 0 overlap |B| (alpha/lambda)^(3/2) exp(-gamma q)
 * falls below overlap_threshold ("Examples": the cutoff is inferred from the
 * threshold); for the density slot, the distance beyond which every
 * primitive's |B| exp(-beta q) does.  rc2: [n_slots]. */
gmp_status gmp_probe_cutoffs(const gmp_probe_desc *desc, double *rc2);

/* [host] outputs (each may be NULL): n_features = sum over orders of
 * n_sigmas (1 for order -1); n_components = sum over orders of
 * n_sigmas (l+1)(l+2)/2 (1 for order -1); n_slots; rc2 [n_slots]. */
gmp_status gmp_plan_info(const gmp_plan *plan, int32_t *n_features, int32_t *n_components,
                         int32_t *n_slots, double *rc2);

/* Tuning knobs (autotuned by the caller or left at defaults).
 *  chunk_pairs:   a centre's list is processed in work items of this many
 *                 pairs (0 = never split).  Item boundaries depend only on
 *                 that centre's own list, so a structure's features are
 *                 bitwise the same alone or inside a batch, for one tuning.
 *  bin_divisor:   cell-list bin edge is about rc_max / bin_divisor (1..4).
 *  blocks_per_cu: workgroups per compute unit of the persistent kernels
 *                 (0 = as many as fit).
 *  adj_items:     work items per centre of the adjoint and Jacobian pair
 *                 kernels (equal pieces of the list; 0 = automatic: about
 *                 8,192 items over the batch, none shorter than chunk_pairs).
 *  sigma_groups:  each forward work item (a chunk of a list) is split into
 *                 this many work items, each taking one group of the cutoff
 *                 slots in cutoff order (1..16, capped at the slot count;
 *                 0 = 1); finer items for the persistent grid, the same
 *                 features bit for bit.
 * The workspace size depends on the tuning.  Changing the tuning is not
 * thread-safe with concurrent calls on the plan. */
typedef struct {
  int32_t chunk_pairs;
  int32_t bin_divisor;
  int32_t blocks_per_cu;
  int32_t adj_items;             /* 0..64 */
  int32_t sigma_groups;          /* 0..16 */
} gmp_tuning;
gmp_status gmp_plan_get_tuning(const gmp_plan *plan, gmp_tuning *out);
gmp_status gmp_plan_set_tuning(gmp_plan *plan, const gmp_tuning *t);

/* [host] bytes of workspace needed by every entry point for a batch of this
 * size (n_points: reference points, 0 without) and a neighbour capacity. */
gmp_status gmp_workspace_size(const gmp_plan *plan, int32_t n_structs, int64_t n_atoms,
                              int64_t n_points, int64_t capacity, size_t *bytes);

/* Lattice wrap, cell-list binning, neighbour count, fill and canonical
 * sort; also the reverse-pair index when nbrs->reverse is not NULL.
 * Every (shell, species) bucket of a list is sorted in LDS.  Lists of up to
 * 8,192 entries are filled by a workgroup per centre with a sort sized for
 * the longest list; longer ones by a second, persistent kernel whose sort
 * takes the workgroup LDS of the device (160 KB on gfx950, about 18,900
 * entries): a list longer than that is filled one range of buckets at a
 * time, and a single bucket longer than that returns GMP_E_UNSUPPORTED.
 * Sync mode (n_pairs != NULL): syncs `stream` once after counting; if the
 * count exceeds nbrs->capacity it returns GMP_E_CAPACITY with *n_pairs set
 * to the required count (offsets are valid; call again with a larger
 * capacity).  No-sync mode (n_pairs == NULL, usable under graph capture):
 * never syncs; an overflow is flagged in the workspace status word (see
 * gmp_check_status): lists that would end past the capacity are not written
 * and gmp_features / gmp_features_backward treat them as empty (zero
 * features and gradients for those centres), and a list with a bucket
 * longer than the long-list sort is replaced by placeholder entries
 * (GMP_E_STALE); every kernel stays inside the caller's arrays. */
gmp_status gmp_build_neighbors(const gmp_plan *plan, const gmp_batch *batch, gmp_neighbors *nbrs,
                               int64_t *n_pairs, void *ws, size_t ws_bytes, void *stream);

/* gmp_build_neighbors without the reverse-pair search: when nbrs->reverse
 * is not NULL its entries are set to -1 and the search keys are kept in
 * `ws`; gmp_build_reverse then completes the index.  gmp_features does not
 * read the reverse index, so the search may run on a second stream (one
 * that waits for this build) while the forward runs; it must have finished
 * before gmp_features_backward.  Same modes, capacity and status rules as
 * gmp_build_neighbors. */
gmp_status gmp_build_lists(const gmp_plan *plan, const gmp_batch *batch, gmp_neighbors *nbrs,
                           int64_t *n_pairs, void *ws, size_t ws_bytes, void *stream);

/* The reverse-pair index (nbrs->reverse) of the lists most recently built
 * by gmp_build_lists into `ws`; reads the search keys that build left in
 * `ws` and nothing that gmp_features writes, so it may run concurrently
 * with gmp_features on the same workspace, but not with another build.
 * Uses nbrs->n_pairs when set (sync mode), else nbrs->capacity, as the
 * bound of the pair range. */
gmp_status gmp_build_reverse(const gmp_plan *plan, const gmp_batch *batch, gmp_neighbors *nbrs, void *ws,
                             size_t ws_bytes, void *stream);

/* Features [n_centres * n_features] (float for the FP32 modes, double for
 * GMP_FP64), order-major: features[i*n_features + f_o + s] with
 * f_o = sum over the orders before o of n_sigmas (1 for order -1), and the
 * single feature of order -1 at f_o.
 * The pair set is the one in nbrs; displacements are evaluated at the
 * batch's current coordinates and lattice with the wrap indices of the
 * build (d = R_j - R_i + (n - m_j + m_i) . cell), so moving atoms or the
 * cell after the build gives the features of the same pairs at the new
 * geometry (bitwise the build's geometry when nothing moved).
 * components (optional, FP64) [n_centres * n_components] laid out
 * (order, sigma, component) with components of order l in the order
 * (a descending, then b descending), and the signed density rho_i as the
 * one component of order -1; required later by the backward. */
gmp_status gmp_features(const gmp_plan *plan, const gmp_batch *batch, const gmp_neighbors *nbrs,
                        void *features, double *components, void *ws, size_t ws_bytes,
                        void *stream);

/* gmp_features without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the forward's scratch (partial moments
 * per work item, chunk offsets, packed positions, the work-item counter) is
 * a fixed array of GMP_NOALLOC_SCRATCH_BYTES in device memory that the
 * library holds on every GPU it runs on until the process ends.  Same
 * arguments, results (bitwise) and status codes as gmp_features, plus
 * GMP_E_NOMEM when the batch needs more scratch than the array holds
 * (about 8 S (l_max+1)(l_max+2)(l_max+3)/6 bytes per work item, i.e. per
 * centre and per chunk_pairs pairs, plus ~100 bytes per atom; the message
 * names both sizes).  Nothing is allocated.  Every call on one GPU shares
 * that GPU's array: calls that overlap in time on one GPU (concurrent
 * streams, several host threads) race and must be serialized by the
 * caller. */
#define GMP_NOALLOC_SCRATCH_BYTES (64u << 20)
gmp_status gmp_features_noalloc(const gmp_plan *plan, const gmp_batch *batch, const gmp_neighbors *nbrs,
                                void *features, double *components, void *stream);

/* Adjoint: given G = dL/dF [n_centres * n_features] (same type as features),
 * writes grad_pos [3 * n_total] (FP64, SoA: x block, y block, z block; each
 * block the atoms, then the reference points) and, when grad_cell is not
 * NULL, grad_cell [n_structs * 9] (FP64, row m = dL/da_m), with Cartesian
 * input positions held fixed and the pair set held fixed.  Needs the
 * components and features of the forward and nbrs->reverse. */
gmp_status gmp_features_backward(const gmp_plan *plan, const gmp_batch *batch,
                                 const gmp_neighbors *nbrs, const double *components,
                                 const void *features, const void *grad_features,
                                 double *grad_pos, double *grad_cell, void *ws, size_t ws_bytes,
                                 void *stream);

/* Full per-pair feature Jacobian ("Examples": feature derivatives with
 * respect to the atom positions), without contraction: for centre i and pair
 * p = (j, n) of its list (global index p, as in j / shift),
 *   jac[(f * 3 + k) * ld + p] = dF_{i,f} / d d_{p,k},  d_p = R_j + n.cell - R_i,
 * so dF_{i,f}/dR_j = sum of the pairs of i with neighbour j, dF_{i,f}/dR_i (or
 * the reference point) = minus the sum over i's list, and dF_{i,f}/da_m =
 * sum_p (n_m - m_j,m + m_i,m) J_p.  Pairs outside a slot's cutoff have zero
 * entries for its features; entries of pairs past the lists are not written.
 * jac: [n_features * 3 * ld], float for the FP32 modes, double for GMP_FP64;
 * ld >= n_pairs (>= capacity when n_pairs is not known, e.g. after a no-sync
 * build).  Needs the components of the forward; the reverse index is not
 * used. */
gmp_status gmp_feature_jacobian(const gmp_plan *plan, const gmp_batch *batch, const gmp_neighbors *nbrs,
                                const double *components, void *jac, int64_t ld, void *ws, size_t ws_bytes,
                                void *stream);

/* Syncs `stream` and reports (and clears) the device status word in ws. */
gmp_status gmp_check_status(void *ws, size_t ws_bytes, void *stream);

/* Per-kernel timing with HIP events on the launch stream.  Between
 * gmp_profile_begin and gmp_profile_end every kernel the library launches is
 * bracketed by events; gmp_profile_end syncs and returns, per kernel name,
 * the number of launches and the summed milliseconds.  names: [host]
 * buffer of max_kernels*64 chars. */
gmp_status gmp_profile_begin(void);
gmp_status gmp_profile_end(int32_t max_kernels, int32_t *n_kernels, char *names,
                           int32_t *launches, double *ms);

const char *gmp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GMP_H */
