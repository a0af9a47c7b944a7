// Internal declarations of the gfx950 GMP feature library.
//
// Every translation unit is compiled with -ffp-contract=off: the lattice
// wrap, image shifts and squared distances must round identically wherever
// they are evaluated (neighbour build, overlap, adjoint), and the two-sum of
// the compensated accumulation must not be fused.  Multiply-adds that may
// round once are written as explicit fma()/fmaf().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/gmp.h"

namespace gmp {

constexpr int kMaxOrders = 6;    // -1 (local density) and 0..4
constexpr int kMaxSigmas = 16;   // cutoff slots: the sigmas plus the density slot of order -1
constexpr int kMaxElements = 64;
constexpr int kMaxL = 4;
constexpr int kCoefStride = 8;    // per (slot, element, primitive): -g', A0..A4, -gamma, screening radius^2
constexpr int kMaxPrims = 16;
constexpr int kWave = 64;

// status-word bits (device side)
enum : uint32_t {
  ST_NONFINITE = 1u,
  ST_CELL = 2u,
  ST_SHIFT_RANGE = 4u,
  ST_OVERFLOW = 8u,
  ST_SORT_SIZE = 16u,
  ST_INTERNAL = 32u,
  ST_BIN_RANGE = 64u,
  ST_SPECIES = 128u,
};

__host__ __device__ constexpr int ncomp(int l) { return (l + 1) * (l + 2) / 2; }
// number of monomials of degree <= d
__host__ __device__ constexpr int nmono(int d) { return d < 0 ? 0 : (d + 1) * (d + 2) * (d + 3) / 6; }
// offset of degree d's block in the monomial array
__host__ __device__ constexpr int doff(int d) { return nmono(d - 1); }
// index of (a, b, c=d-a-b) inside degree d, components ordered a desc then b desc
__host__ __device__ constexpr int midx(int d, int a, int b) { return (d - a) * (d - a + 1) / 2 + (d - a - b); }

// Monomial recursion table: monomial t (global index, degree >= 1) equals
// variable var[t] (0=x, 1=y, 2=z) times monomial parent[t].
struct MonoTable {
  int parent[35];
  int var[35];
  int deg[35];
  int ea[35], eb[35], ec[35];
};

__host__ __device__ constexpr MonoTable make_mono_table() {
  MonoTable t{};
  for (int d = 0; d <= 4; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        int c = d - a - b;
        int g = doff(d) + midx(d, a, b);
        t.deg[g] = d; t.ea[g] = a; t.eb[g] = b; t.ec[g] = c;
        if (d == 0) { t.parent[g] = -1; t.var[g] = -1; continue; }
        if (a > 0) { t.parent[g] = doff(d - 1) + midx(d - 1, a - 1, b); t.var[g] = 0; }
        else if (b > 0) { t.parent[g] = doff(d - 1) + midx(d - 1, 0, b - 1); t.var[g] = 1; }
        else { t.parent[g] = doff(d - 1) + midx(d - 1, 0, 0); t.var[g] = 2; }
      }
  return t;
}

// Adjoint coefficient block per (centre, slot): the monomial coefficients M
// [nmono(L)] of the upstream-weighted polynomial, padded to a multiple of 4
// entries so the pair kernels' wavefront-uniform LDS reads can be 16-byte
// vector reads.  The pair kernels take the gradient of the polynomial from
// the same coefficients (exponents are compile-time constants).
// entries of the moment -> component maps of orders 0..kMaxL (ncomp(l)^2 each)
__host__ __device__ constexpr int tmat_size() {
  int n = 0;
  for (int l = 0; l <= kMaxL; ++l) n += ncomp(l) * ncomp(l);
  return n;
}
constexpr int kTmat = tmat_size();
__host__ __device__ constexpr int round4(int n) { return (n + 3) & ~3; }
__host__ __device__ constexpr int coef_m(int lmax) { return round4(nmono(lmax)); }
__host__ __device__ constexpr int coef_block(int lmax) { return coef_m(lmax); }

struct StructInfo {
  double b[9];        // reciprocal rows
  double reach[3];    // fractional reach rc_max/h_k (periodic axes)
  int nb[3];          // bins per axis
  int pbc;
  int64_t bin_base;   // first bin slot of this structure
  double lam_lo;      // lower bound of the smallest eigenvalue of the lattice metric (0: no bin culling)
  double inv_nb[3];   // 1 / nb[k] (bin-image culling bounds)
};

// Device view of a plan (passed by value to kernels).  S counts cutoff
// slots: the n_sig sigmas, then (dens_slot = n_sig) the local density of
// order -1 when requested (dens_slot = -1 otherwise).  The density slot's
// coefficient rows hold -beta (scaled), A_0 = B, A_1..A_4 = 0, -beta.
struct PlanDev {
  int S, E, n_orders, lmax, order_mask, kmax, kb, nf, ncomp_total;  // kb: primitive stride of the tables (4/8/16)
  int n_sig, dens_slot, dens_order;  // sigmas, density slot, index of order -1 in orders (-1: none)
  int screen;                        // per-primitive screening (radius^2 in column 7 of the tables, FP32 value)
  int tab_n;                         // tabulated radial factors: intervals per (slot, element) (0: exact)
  float tab_inv_h[kMaxSigmas];       // 1 / interval width (in r = sqrt(q)) of every slot's table
  const float4 *rtab;                // [S][E][tab_n][5]: cubic coefficients in t of c_l, l = 0..4
  int orders[kMaxOrders];
  int comp_off[kMaxOrders];       // offset of order o's (sigma, component) block in one centre's components
  int feat_off[kMaxOrders];       // first feature of order o (n_sig features per order, 1 for order -1)
  int order_idx[kMaxL + 1];       // index o of angular order l in orders (-1: not requested)
  int sig_order[kMaxSigmas];      // slots sorted by rc^2 ascending (stable)
  int rank_lt[kMaxSigmas];        // #{s': rc2[s'] < rc2[s]}
  double rc2[kMaxSigmas];
  double rcmax2;
  const float *coef32;            // [S][E][kb][kCoefStride]: -gamma*log2(e), A_0..A_4, -gamma, r^2 (zero rows past K_e)
  const double *coef64;           // [S][E][kb][kCoefStride]: -gamma, A_0..A_4, -gamma, r^2
  const int *kcount;              // [E]
  const double *T;                // moment->component maps, per order l: ncomp(l)^2 at toff[l]
  int toff[kMaxL + 1];
  double weight[35];              // l!/(a!b!c!) by global monomial index (same (a,b,c) ordering)
};

// Atoms and (optional) reference points share one index space g: atoms
// 0..N-1, then points N..N+M-1.  The centres are the atoms (centre c is g = c)
// or, with reference points, the points (centre c is g = N + c); neighbours
// are always atoms.
struct BatchDev {
  int n_structs;
  int64_t n_atoms;
  const int64_t *atom_offsets;
  const double *x, *y, *z;
  const int32_t *species;
  const double *cell;
  const uint8_t *pbc;
  const double *occ;       // [n_atoms] occupancies or null (all 1)
  int64_t n_points;        // reference points (0 without)
  const int64_t *point_offsets;  // [n_structs+1], null: the centres are the atoms
  const double *px, *py, *pz;
};

__host__ __device__ inline bool point_mode(const BatchDev &b) { return b.point_offsets != nullptr; }
__host__ __device__ inline int64_t n_points_of(const BatchDev &b) { return point_mode(b) ? b.n_points : 0; }
__host__ __device__ inline int64_t n_total(const BatchDev &b) { return b.n_atoms + n_points_of(b); }
__host__ __device__ inline int64_t n_centres(const BatchDev &b) { return point_mode(b) ? b.n_points : b.n_atoms; }
__host__ __device__ inline int64_t centre_base(const BatchDev &b) { return point_mode(b) ? b.n_atoms : 0; }

// Lists are stored per slot: slot k holds the list of centre order[k], and
// slot[i] is the slot of centre i (atoms: cell-list order, points: their own).
struct NbrDev {
  int64_t capacity;
  int64_t *offsets;        // [N+1] per slot
  int32_t *j;
  int32_t *shift;
  int32_t *bucket_start;   // [N][S*E+1] per slot: local starts of buckets (shell h, species e) = h*E + e
  int32_t *sigma_end;      // [N][S] per slot: end of each cutoff slot's prefix
  int32_t *wrap;
  double *rw;
  int32_t *reverse;
  int32_t *order;          // [N] centre of every slot
  int32_t *slot;           // [N] slot of every centre
};

// ---------------------------------------------------------------- device helpers
// Workgroup index -> position in a sequence, such that the workgroups the
// dispatcher places on one XCD (every eighth) take one contiguous range.
__device__ inline int64_t xcd_contiguous(int64_t b, int64_t nblk) {
  const int64_t x = b & 7, per = nblk >> 3, rem = nblk & 7;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

// LDS writes of one wavefront become visible to its other lanes.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The value of lane 0 as a wavefront-uniform (scalar) value.
__device__ inline int64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Next work item of a persistent kernel (one atomic per wavefront).
__device__ inline int64_t next_item(unsigned long long *counter) {
  unsigned long long it = 0;
  if ((threadIdx.x & 63) == 0) it = atomicAdd(counter, 1ull);
  return uniform64(__shfl(it, 0, 64));
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline int struct_of_atom(const int64_t *off, int n_structs, int64_t i) {
  int lo = 0, hi = n_structs;  // find s with off[s] <= i < off[s+1]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Image shift s(n) = (n1 a1 + n2 a2) + n3 a3, FP64, fixed operation order.
__device__ inline void image_shift(const double *cell, int n1, int n2, int n3, double &sx, double &sy,
                                   double &sz) {
  double t;
  t = (double)n1 * cell[0] + (double)n2 * cell[3]; sx = t + (double)n3 * cell[6];
  t = (double)n1 * cell[1] + (double)n2 * cell[4]; sy = t + (double)n3 * cell[7];
  t = (double)n1 * cell[2] + (double)n2 * cell[5]; sz = t + (double)n3 * cell[8];
}

// Lattice rows held in registers for the duration of a work item.
struct Cell9 {
  double a[9];
};
__device__ inline Cell9 load_cell(const double *cell) {
  Cell9 c;
#pragma unroll
  for (int k = 0; k < 9; ++k) c.a[k] = cell[k];
  return c;
}
__device__ inline void image_shift(const Cell9 &c, int n1, int n2, int n3, double &sx, double &sy, double &sz) {
  image_shift(c.a, n1, n2, n3, sx, sy, sz);
}

// Structure of index g (atom or reference point).
__device__ inline int struct_of_index(const BatchDev &bt, int64_t g) {
  return g < bt.n_atoms ? struct_of_atom(bt.atom_offsets, bt.n_structs, g)
                        : struct_of_atom(bt.point_offsets, bt.n_structs, g - bt.n_atoms);
}

// Wrapped position Rw_i = R_i - ((m1 a1 + m2 a2) + m3 a3) of index i (atom or
// reference point) from the current positions and lattice and the wrap
// indices of the neighbour build; the same operation order as the build, so
// unchanged inputs give the same bits.  The fourth component carries the
// atom's occupancy (1 when none is given, and for points).
__device__ inline double4 wrapped_position(const BatchDev &bt, const NbrDev &nb, int64_t i, int s) {
  const bool atom = i < bt.n_atoms;
  const int64_t k = atom ? i : i - bt.n_atoms;
  const double *X = atom ? bt.x : bt.px, *Y = atom ? bt.y : bt.py, *Z = atom ? bt.z : bt.pz;
  double r[3] = {X[k], Y[k], Z[k]};
  if (bt.pbc[s] & 7) {
    const double *a = bt.cell + 9 * (int64_t)s;
    const double m0 = (double)nb.wrap[3 * i], m1 = (double)nb.wrap[3 * i + 1], m2 = (double)nb.wrap[3 * i + 2];
    for (int c = 0; c < 3; ++c) {
      double t = m0 * a[c] + m1 * a[3 + c];
      t = t + m2 * a[6 + c];
      r[c] = r[c] - t;
    }
  }
  return make_double4(r[0], r[1], r[2], (atom && bt.occ) ? bt.occ[i] : 1.0);
}

__device__ inline int shift_n(int32_t w, int k) { return (int)(int8_t)((uint32_t)w >> (8 * k)); }
__device__ inline int shift_species(int32_t w) { return (int)((uint32_t)w >> 24); }

}  // namespace gmp

// ---------------------------------------------------------------- host side
struct gmp_plan {
  gmp_precision prec;
  gmp::PlanDev dev;
  int S, E, n_orders;  // S: cutoff slots (sigmas, plus the density slot of order -1)
  int orders[gmp::kMaxOrders];
  double sigmas[gmp::kMaxSigmas];
  double rc2[gmp::kMaxSigmas];
  gmp_tuning tuning;
  void *dmem;  // single device allocation holding the tables
};

namespace gmp {
gmp_status set_error(gmp_status st, const std::string &msg);
gmp_status hip_error(hipError_t e, const char *where);

// kernel launch bookkeeping for the optional per-kernel event timing
void prof_before(const char *name, hipStream_t s);
void prof_after(hipStream_t s);

// workspace carving
struct Carver {
  char *base;
  size_t off, cap;
  bool dry;
  explicit Carver(void *p, size_t c) : base((char *)p), off(0), cap(c), dry(p == nullptr) {}
  template <typename T> T *take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T *p = dry ? nullptr : (T *)(base + off);
    off += n * sizeof(T);
    return p;
  }
};

struct WsLayout {
  uint32_t *status;       // [64] words: [0] flags, [2..3] total pairs, [4] longest list, [5] longest bucket,
                          // [6] long-list queue length, [7] next queue entry
  StructInfo *sinfo;
  int32_t *bin_of;
  int32_t *astruct;       // [N] structure of every atom (written by the per-atom kernel of each stage)
  int32_t *bin_count;
  int64_t *bin_start;
  int32_t *bin_fill;
  double *fw;             // [3][N]
  double *sx, *sy, *sz;   // bin-sorted wrapped positions
  int32_t *sid, *ssp;     // bin-sorted atom index and species
  int32_t *cnt;           // [N][S][E] neighbours per bucket (shell, species)
  int64_t *ptotal;        // [N]
  int32_t *long_q;        // [N] slots whose lists the long-list fill kernel writes
  int32_t *sid_tmp;       // [N] atoms placed in their bins in arrival order (before the in-bin ordering)
  int64_t *scan_aux;      // scan block sums
  double *partial;        // overlap partial moments [chunk][sigma][monomial]
  int64_t *nch;           // [N] chunks per centre
  int64_t *chunk_off;     // [N+1] first chunk of each centre
  unsigned long long *counter;  // work-item counter of the persistent kernels
  double4 *rw4;           // [N] AoS copy of the wrapped positions
  uint64_t *pair_key;     // [capacity] packed (j, n) of every pair (reverse search)
  int32_t *pair_centre;   // [capacity] centre of every pair (reverse search)
  uint64_t *pair_sum;     // [capacity/16 + 1] every 16th packed key (first level of the reverse search)
  int64_t *abs_bstart;    // [N][S*E+1] bucket starts as global pair indices, a row per atom (reverse search)
  // reference points: pairs sorted by neighbour atom (adjoint gather order)
  uint32_t *tr_key_in, *tr_key_out, *tr_val_in, *tr_val_out;  // [capacity] radix-sort ping-pong buffers
  int32_t *tr_hist;       // [256 * tiles] per-tile digit counts
  int64_t *tr_off;        // [256 * tiles + 1] their exclusive scan
  int64_t *tr_start;      // [n_atoms + 1] first sorted pair of every atom
  void *bcoef;            // adjoint per-centre polynomial coefficients
  void *vbuf;             // adjoint per-pair vectors [capacity][4]
  double *cellpart;       // [N][9]
  size_t bytes;
};
WsLayout carve(const gmp_plan *p, int n_structs, int64_t n_atoms, int64_t n_points, int64_t capacity, void *ws,
               size_t ws_bytes);
int64_t transpose_tiles(int64_t n);  // tiles of the by-neighbour sort of n pairs
int64_t partial_slots(const gmp_plan *p, int64_t n_atoms, int64_t capacity);

// device scans (exclusive, writes n+1 outputs)
void scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *aux, hipStream_t s);
void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *aux, hipStream_t s);
int64_t scan_aux_size(int64_t n);
void fill_zero(void *p, size_t bytes, hipStream_t s);
}  // namespace gmp

// Launch with optional event timing.  `label` names the kernel in the
// per-kernel timing report; `kernel` may be a function-pointer variable.
#define GMP_LAUNCH(label, kernel, grid, block, smem, stream, ...)              \
  do {                                                                         \
    gmp::prof_before(label, stream);                                           \
    hipLaunchKernelGGL(kernel, grid, block, smem, stream, __VA_ARGS__);        \
    gmp::prof_after(stream);                                                   \
  } while (0)
