// Overlap kernel (multipole moments) and norm kernel.
//
// Closed form of one pair's contribution (derived from the Gaussian product
// theorem and the mean-value property of harmonic polynomials; the paper
// defines the probe as an MCSH angular probe times a Gaussian radial probe
// and the density as per-element Gaussian primitives):
//   mu_{i,l,s,abc} += c_{l,s,e_j}(q) P_abc(d),
//   c_{l,s,e}(q) = sum_k A_{l,s,e,k} exp(-gamma_{s,e,k} q),
// each pair term scaled by the neighbour's occupancy (disordered structures;
// 1 when none is given), which rides in the fourth component of its packed
// wrapped position and multiplies the monomial recursion's seed.
// P_abc is a homogeneous polynomial of degree l, so the kernel accumulates
// the Cartesian moments  M_{i,s,m} = sum_j c_{deg m,s,e_j}(q_j) x^a y^b z^c
// of every monomial m of each requested degree, and the norm kernel maps
// moments to components with the plan's exact integer matrices (FP64).
//
// Work decomposition: persistent wavefronts pull work items (a chunk of one
// centre's list) from a global counter; lanes take consecutive pairs.  The
// list is ordered by cutoff shell first, so the pairs a sigma uses form a
// prefix and each sigma is one pass over its own prefix, without testing q.
// Lanes read the coefficient row of their own neighbour's species from the
// LDS copy of the plan table.  The local density of order -1 is one more
// cutoff slot whose pass accumulates only the degree-0 moment
// rho = sum_j sum_k B exp(-beta q).
//
// Precision policies (template MODE):
//   FP32 compensated: displacement rounded to FP32; monomials, exp2, radial
//              sums and products in FP32; per-lane accumulation as FP32
//              (hi, lo) two-sum pairs; cross-lane reduction in FP64.
//   FP32 wide: FP32 exp2 and radial sums, FP64 monomials and accumulation.
//   FP64:      everything FP64 (exp in FP64), plain accumulation.
#include <map>
#include <mutex>
#include <type_traits>

#include "gmp_internal.h"

namespace gmp {
namespace {

constexpr MonoTable kMT = make_mono_table();

__device__ inline float exp_scaled(float a, float q) { return __builtin_amdgcn_exp2f(a * q); }
__device__ inline double exp_scaled(double a, double q) { return exp(a * q); }
__device__ inline float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fma_(double a, double b, double c) { return fma(a, b, c); }

// Chunks of one centre's list: fixed-size pieces of kc pairs (kc = 0: whole
// list), so the decomposition of a centre depends on its own list only and
// a batched launch sums in the same order as a launch over one structure.
// Per list slot: the number of work items of its list (fixed-size pieces
// of kc pairs, kc = 0: whole list, each split into ng groups of cutoff
// slots, so the decomposition of a centre depends on its own list only and
// a batched launch sums in the same order as a launch over one structure),
// its structure, and its wrapped position as an AoS double4 (one 32-byte
// gather per neighbour).  The first thread also clears the work-item counter.
// Indices g < n_total get their structure and packed position; centres
// c < n_centres their chunk count.
__global__ void k_overlap_prep(BatchDev bt, NbrDev nb, int kc, int ng, int64_t *nch, double4 *rw4,
                               int32_t *astruct, unsigned long long *counter) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *counter = 0ull;
  if (i < n_centres(bt)) {
    const int64_t cnt = nb.offsets[i + 1] - nb.offsets[i];
    // a list that ends past the capacity was not written (overflowed no-sync
    // build, reported in the status word): no work items, zero moments
    nch[i] = nb.offsets[i + 1] > nb.capacity ? 0 : ng * (kc > 0 ? (cnt > kc ? (cnt + kc - 1) / kc : 1) : 1);
  }
  if (i < n_total(bt)) {
    const int st = struct_of_index(bt, i);
    astruct[i] = st;
    rw4[i] = wrapped_position(bt, nb, i, st);
  }
}

__device__ inline int64_t centre_of_chunk(const int64_t *chunk_off, int64_t N, int64_t q) {
  int64_t lo = 0, hi = N;  // chunk_off[lo] <= q < chunk_off[lo+1]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= q) lo = mid; else hi = mid;
  }
  return lo;
}

// Accumulation policies of the overlap kernel.
enum AccMode { ACC_F64 = 0, ACC_TWOSUM = 1, ACC_WIDE = 2 };

// Per-lane accumulator of one sigma's moments.
template <int MODE, int NM> struct Acc;
// FP32 (hi, lo) pairs updated with an error-free sum: Dekker's Fast2Sum
// on the two addends ordered by magnitude (exact when the first is the
// larger).  It yields the same exact rounding error, hence the same (hi,
// lo), as Knuth's branch-free two-sum, in as many operations (a compare on
// magnitudes, two selects, three additions), but reads the old sum only
// before the new one is formed, so the new sum takes its register without a
// copy back.
template <int NM> struct Acc<ACC_TWOSUM, NM> {
  float hi[NM], lo[NM];
  __device__ void zero() {
#pragma unroll
    for (int m = 0; m < NM; ++m) { hi[m] = 0.f; lo[m] = 0.f; }
  }
  __device__ void add(int m, float p) {
    const bool ge = __builtin_fabsf(hi[m]) >= __builtin_fabsf(p);
    const float big = ge ? hi[m] : p, small = ge ? p : hi[m];
    const float s = big + small;
    lo[m] += small - (s - big);
    hi[m] = s;
  }
  __device__ double value(int m) const { return (double)hi[m] + (double)lo[m]; }
};
// FP64 accumulators (FP64 path and the wide FP32 path).
template <int NM> struct Acc<ACC_F64, NM> {
  double v[NM];
  __device__ void zero() {
#pragma unroll
    for (int m = 0; m < NM; ++m) v[m] = 0.0;
  }
  __device__ double value(int m) const { return v[m]; }
};
template <int NM> struct Acc<ACC_WIDE, NM> : Acc<ACC_F64, NM> {};

// Fixed-order cross-lane sum of NV per-lane doubles, written to dst[0..NV):
// rounds of 8 columns are transposed through LDS (each lane sums 8 rows of
// one column), then the 8 row-group partials are combined with xor shuffles.
// Every lane of a column group computes the same bits; lanes 0..7 store.
template <int NV>
__device__ inline void wave_reduce_store(const double (&v)[NV], double *dst, double *lds) {
  const int lane = lane_id();
  const int col = lane & 7, grp = lane >> 3;
#pragma unroll
  for (int base = 0; base < NV; base += 8) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (base + c < NV) lds[lane * 9 + c] = v[base + c];
    wave_lds_sync();
    double s = 0.0;
    if (base + col < NV) {
#pragma unroll
      for (int r = 0; r < 8; ++r) s += lds[(grp * 8 + r) * 9 + col];
    }
    s += __shfl_xor(s, 8, kWave);
    s += __shfl_xor(s, 16, kWave);
    s += __shfl_xor(s, 32, kWave);
    if (lane < 8 && base + lane < NV) dst[base + lane] = s;
    wave_lds_sync();
  }
}

template <int MODE, int NM> __device__ inline double acc_value(const Acc<MODE, NM> &a, int m) { return a.value(m); }

// Overlap kernel, persistent: every wavefront pulls work items (one chunk
// of one centre's list) from a global counter until none are left, and
// walks the sigmas of the item one after another in cutoff order, each over
// its own prefix of the chunk.  The loads of pair data (j, shift) run two
// steps ahead and the gathers of the neighbours' wrapped positions one step
// ahead, continuously across the sigma passes.  Every monomial of degree
// <= LMAX is accumulated (moments of orders that were not requested are
// simply not read back).
//
// The coefficient table [sigma][element][KB][8] (exponent scale, A_0..A_4,
// -gamma) is copied into LDS once per workgroup when it fits; lanes read
// the row of their own neighbour's species.
// Radial factors c_0..c_L of slot s and element e at squared distance q from
// the plan's table: cubic in t = r/h - k on interval k of r = sqrt(q).
template <int L>
__device__ inline void radial_from_table(const PlanDev &P, int s, int e, float q, float (&cl)[L + 1]) {
  const float x = __builtin_sqrtf(q) * P.tab_inv_h[s];
  int k = (int)x;
  k = k < P.tab_n - 1 ? k : P.tab_n - 1;
  const float t = x - (float)k;
  const float4 *c = P.rtab + (((size_t)s * P.E + e) * P.tab_n + k) * 5;
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    const float4 a = c[l];
    cl[l] = fmaf(fmaf(fmaf(a.w, t, a.z), t, a.y), t, a.x);
  }
}

// The wide mode's 35 FP64 accumulators and FP64 monomials fit three
// wavefronts per SIMD (<= 168 VGPRs) once each monomial is accumulated as it
// is formed; the bound keeps the compiler at that occupancy.
template <int LMAX, int KB, int MODE, bool LDS, bool DENS, bool SCREEN, bool TAB = false>
__global__ __launch_bounds__(256, MODE == ACC_WIDE ? 3 : 1) void k_overlap(PlanDev P, BatchDev bt, NbrDev nb, const double4 *rw4,
                                                 const int32_t *astruct, double *partial, const int64_t *chunk_off,
                                                 int kc, int ng, unsigned long long *counter,
                                                 const void *tab_global) {
  constexpr bool F64 = MODE == ACC_F64;
  using TR = typename std::conditional<F64, double, float>::type;                 // radial arithmetic
  using TM = typename std::conditional<MODE == ACC_TWOSUM, float, double>::type;  // monomials
  constexpr int NM = nmono(LMAX);
  extern __shared__ __align__(16) double lds_dyn[];
  __shared__ double lds_red[4][64 * 9];
  __shared__ int lds_k[kMaxElements];
  const int S = P.S, E = P.E;
  const TR *__restrict__ tabg = (const TR *)tab_global;
  TR *tabl = (TR *)lds_dyn;
  if (LDS) {
    const int n = S * E * KB * kCoefStride;
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) tabl[idx] = tabg[idx];
  }
  for (int e = threadIdx.x; e < E; e += blockDim.x) lds_k[e] = P.kcount[e];
  __syncthreads();

  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  const int64_t N = n_centres(bt), cb = centre_base(bt);
  const int64_t n_items = chunk_off[N];
  for (;;) {
    const int64_t qc = next_item(counter);
    if (qc >= n_items) break;
    const int64_t k = centre_of_chunk(chunk_off, N, qc);  // list slot
    const int64_t i = nb.order[k];                         // its centre
    // item = (chunk c of the list, group g of the cutoff slots in cutoff
    // order: passes [t0, t1)); every item writes all slots' moments, zero
    // for the slots outside its group, so a centre's sum is the same for any ng
    const int cg = (int)(qc - chunk_off[k]);
    const int c = cg / ng, g = cg - c * ng;
    const int t0 = g * S / ng, t1 = (g + 1) * S / ng;
    const int st = astruct[cb + i];
    const Cell9 cell = load_cell(bt.cell + 9 * (int64_t)st);
    const int pbc = bt.pbc[st] & 7;
    const double4 ri4 = rw4[cb + i];
    const double rix = ri4.x, riy = ri4.y, riz = ri4.z;
    const int64_t base = nb.offsets[k];
    const int cnt = (int)(nb.offsets[k + 1] - base);
    const int clo = kc > 0 ? c * kc : 0;
    const int chi = kc > 0 ? (clo + kc < cnt ? clo + kc : cnt) : cnt;
    // per-item pass ends and sigma order, one per lane (lane t <-> t-th sigma by cutoff)
    int end_lane = clo, so_lane = 0;
    if (lane < S) {
      so_lane = P.sig_order[lane];
      const int en = nb.sigma_end[k * S + so_lane];
      end_lane = en < chi ? en : chi;
    }
    auto uni = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
    auto pass_end = [&](int t) { return __builtin_amdgcn_readlane(end_lane, t); };
    double *dst_item = partial + (size_t)qc * S * NM;
    // sigmas outside the item's group, or whose prefix misses this chunk,
    // contribute zero moments
    for (int t = 0; t < S; ++t)
      if (t < t0 || t >= t1 || pass_end(t) <= clo)
        for (int m = lane; m < NM; m += kWave)
          dst_item[(size_t)__builtin_amdgcn_readlane(so_lane, t) * NM + m] = 0.0;
    // step iterator over (sigma pass t, pair block p0); pass ends are non-decreasing in t
    int tb = t0, pb = clo;
    while (tb < t1 && pass_end(tb) <= clo) ++tb;
    if (tb >= t1) continue;
    int tc = tb, pc = pb;
    auto advance = [&](int &t, int &p) {
      p += kWave;
      if (p >= pass_end(t)) {
        ++t;
        p = clo;
        while (t < t1 && pass_end(t) <= clo) ++t;
      }
      t = uni(t);
      p = uni(p);
    };
    advance(tc, pc);
    const int32_t ii = (int32_t)(cb + i);  // idle lanes read the centre's own packed position
    // stage b: positions gathered; stage c: (j, shift) loaded
    int32_t wb = 0, jc = ii, wc = 0;
    double4 rb;
    {
      int32_t jb = ii;
      const int p = pb + lane;
      if (p < pass_end(tb)) { jb = nb.j[base + p]; wb = nb.shift[base + p]; }
      if (tc < t1 && pc + lane < pass_end(tc)) { jc = nb.j[base + pc + lane]; wc = nb.shift[base + pc + lane]; }
      rb = rw4[jb];
    }
    Acc<MODE, NM> acc;
    acc.zero();
    while (tb < t1) {
      const int ta = tb, pa = pb;
      const int32_t w = wb;
      const double rjx = rb.x, rjy = rb.y, rjz = rb.z, occj = rb.w;  // w: occupancy of j
      // advance the pipeline
      tb = tc; pb = pc; wb = wc;
      rb = rw4[jc];
      jc = ii; wc = 0;
      if (tc < t1) {
        advance(tc, pc);
        if (tc < t1 && pc + lane < pass_end(tc)) { jc = nb.j[base + pc + lane]; wc = nb.shift[base + pc + lane]; }
      }
      // current step: slot sig_order[ta], pairs pa + lane
      const int sgm = __builtin_amdgcn_readlane(so_lane, ta);
      const int p = pa + lane;
      if (DENS && p < pass_end(ta) && sgm == P.dens_slot) {
        // local density (order -1): the degree-0 moment of sum_k B exp(-beta q)
        double shx = 0.0, shy = 0.0, shz = 0.0;
        if (pbc) image_shift(cell, shift_n(w, 0), shift_n(w, 1), shift_n(w, 2), shx, shy, shz);
        const double dx = (rjx - rix) + shx;
        const double dy = (rjy - riy) + shy;
        const double dz = (rjz - riz) + shz;
        const double q = (dx * dx + dy * dy) + dz * dz;
        const TR qv = (TR)q;
        const int e = shift_species(w);
        const int K = TAB ? 0 : lds_k[e];
        const size_t roff = ((size_t)(sgm * E + e) * KB) * kCoefStride;
        TR c0 = (TR)0;
        if constexpr (TAB && !F64) {
          float ct[1];
          radial_from_table<0>(P, sgm, e, qv, ct);
          c0 = ct[0];
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          if (k < K) {
            const size_t o = roff + k * kCoefStride;
            bool use = true;
            if constexpr (SCREEN) {  // the primitive's own radius; skipped by the wavefront when no lane needs it
              use = (float)q <= (float)(LDS ? tabl[o + 7] : tabg[o + 7]);
              if (__ballot(use) == 0) continue;
            }
            const TR ek = exp_scaled(LDS ? tabl[o] : tabg[o], qv);
            c0 = fma_(LDS ? tabl[o + 1] : tabg[o + 1], use ? ek : (TR)0, c0);
          }
        }
        c0 = c0 * (TR)occj;
        if constexpr (MODE == ACC_TWOSUM) acc.add(0, c0);
        else acc.v[0] += (double)c0;
      } else if (p < pass_end(ta)) {
        double shx = 0.0, shy = 0.0, shz = 0.0;
        if (pbc) image_shift(cell, shift_n(w, 0), shift_n(w, 1), shift_n(w, 2), shx, shy, shz);
        const double dx = (rjx - rix) + shx;
        const double dy = (rjy - riy) + shy;
        const double dz = (rjz - riz) + shz;
        const double q = (dx * dx + dy * dy) + dz * dz;
        const TR qv = (TR)q;
        const int e = shift_species(w);
        const int K = lds_k[e];
        const size_t roff = ((size_t)(sgm * E + e) * KB) * kCoefStride;
        TR cl[LMAX + 1];
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) cl[l] = (TR)0;
        if constexpr (TAB && !F64) {
          radial_from_table<LMAX>(P, sgm, e, qv, cl);
        } else if constexpr (!SCREEN && !F64) {
          // FP32 table rows past an element's own primitive count are zero
          // (they add exact zeros), so every lane runs the plan's largest
          // count with wavefront-uniform control flow, and the LDS read of
          // row k+1 is issued before row k is used (the empty asm statement
          // keeps the compiler from sinking it)
          const TR *row = (LDS ? tabl : tabg) + roff;
          const int kmx = P.kmax;
          float4 ra = *(const float4 *)row;
          float2 rb2 = *(const float2 *)(row + 4);
          auto row_step = [&](int k) {
            float4 na; float2 nb2;
            if (k + 1 < KB) { na = *(const float4 *)(row + (k + 1) * kCoefStride); nb2 = *(const float2 *)(row + (k + 1) * kCoefStride + 4); }
            asm volatile("" ::: "memory");
            const TR ek = exp_scaled(ra.x, qv);
            const TR av[5] = {ra.y, ra.z, ra.w, rb2.x, rb2.y};
#pragma unroll
            for (int l = 0; l <= LMAX; ++l) cl[l] = fma_(av[l], ek, cl[l]);
            if (k + 1 < KB) { ra = na; rb2 = nb2; }
          };
          if constexpr (KB <= 8) {  // full unroll with an early exit (trip count bound <= 8)
#pragma unroll
            for (int k = 0; k < KB; ++k) {
              if (k >= kmx) break;
              row_step(k);
            }
          } else {  // 16-row tables: a wavefront-uniform guard keeps the trip count constant
#pragma unroll
            for (int k = 0; k < KB; ++k)
              if (k < kmx) row_step(k);
          }
        } else {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          if (k < K) {
            const size_t o = roff + k * kCoefStride;
            bool use = true;
            if constexpr (SCREEN) {  // the primitive's own radius; skipped by the wavefront when no lane needs it
              use = (float)q <= (float)(LDS ? tabl[o + 7] : tabg[o + 7]);
              if (__ballot(use) == 0) continue;
            }
            TR ek = exp_scaled(LDS ? tabl[o] : tabg[o], qv);
            if constexpr (SCREEN) ek = use ? ek : (TR)0;
#pragma unroll
            for (int l = 0; l <= LMAX; ++l) cl[l] = fma_(LDS ? tabl[o + 1 + l] : tabg[o + 1 + l], ek, cl[l]);
          }
        }
        }
        // monomials degree by degree from their parents, each accumulated as
        // soon as it is formed (only the previous degree's stay live)
        double cd[LMAX + 1];
        if constexpr (MODE != ACC_TWOSUM) {
#pragma unroll
          for (int l = 0; l <= LMAX; ++l) cd[l] = (double)cl[l];
        }
        TM mono[NM];
        const TM xv = (TM)dx, yv = (TM)dy, zv = (TM)dz;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          if (m == 0) {
            mono[0] = (TM)occj;  // the occupancy scales every monomial of the pair
          } else {
            const TM v = kMT.var[m] == 0 ? xv : (kMT.var[m] == 1 ? yv : zv);
            mono[m] = v * mono[kMT.parent[m]];
          }
          if constexpr (MODE == ACC_TWOSUM) acc.add(m, cl[kMT.deg[m]] * mono[m]);
          else acc.v[m] = fma(cd[kMT.deg[m]], mono[m], acc.v[m]);
        }
      }
      if (tb != ta) {  // the pass of slot sgm is complete: FP64 cross-lane reduction, store, restart
        double vals[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) vals[m] = acc.value(m);
        wave_reduce_store<NM>(vals, dst_item + (size_t)sgm * NM, lds_red[wv]);
        acc.zero();
      }
    }
  }
}

// One wavefront per centre: sum chunk partials in order, map moments to
// components with the exact integer matrices, then the weighted norm
// F_{l,s} = sqrt(sum_abc l!/(a!b!c!) mu_abc^2).  Order -1 takes the degree-0
// moment of the density slot as its component rho and |rho| as its feature.
// Where every component and feature comes from (order, slot, position) is
// decoded once per workgroup into LDS tables, so the per-centre loops are
// table reads and dot products; the partials of a centre with one work item
// (the common case) are read directly.
template <int LMAX, bool F64OUT>
__global__ __launch_bounds__(256) void k_finish(PlanDev P, int64_t N, const double *partial,
                                                const int64_t *chunk_off, const int32_t *order, void *features,
                                                double *components) {
  extern __shared__ double lds_f[];
  // moment -> component maps of all orders and the multinomial weights,
  // staged in LDS once per workgroup (read with lane-varying indices)
  __shared__ double lds_T[kTmat];
  __shared__ double lds_w[nmono(kMaxL)];
  constexpr int NM = nmono(LMAX);  // compile-time: the index splits below are not divisions
  const int S = P.S, NC = P.ncomp_total, NF = P.nf;
  // decode tables after the four wavefronts' moment and component buffers:
  // component t: T row offset | moment offset << 10 | length << 22 (bit 31:
  // the density component, moment offset only); feature t: component offset |
  // weight offset << 12 | length << 20 (bit 31: the density feature)
  int32_t *cdec = (int32_t *)(lds_f + (size_t)4 * (S * NM + NC));
  int32_t *fdec = cdec + NC;
  for (int t = threadIdx.x; t < kTmat; t += blockDim.x) lds_T[t] = P.T[t];
  for (int t = threadIdx.x; t < nmono(kMaxL); t += blockDim.x) lds_w[t] = P.weight[t];
  for (int t = threadIdx.x; t < NC; t += blockDim.x) {
    int o = 0;
    while (o + 1 < P.n_orders && P.comp_off[o + 1] <= t) ++o;
    const int l = P.orders[o];
    if (l < 0) {
      cdec[t] = (int32_t)(0x80000000u | (uint32_t)((P.dens_slot * NM) << 10));
    } else {
      const int nc = ncomp(l), r = t - P.comp_off[o];
      const int sl = r / nc, cc = r - sl * nc;
      cdec[t] = (P.toff[l] + cc * nc) | ((sl * NM + doff(l)) << 10) | (nc << 22);
    }
  }
  for (int t = threadIdx.x; t < NF; t += blockDim.x) {
    int o = 0;
    while (o + 1 < P.n_orders && P.feat_off[o + 1] <= t) ++o;
    const int l = P.orders[o];
    if (l < 0) {
      fdec[t] = (int32_t)(0x80000000u | (uint32_t)P.comp_off[o]);
    } else {
      const int nc = ncomp(l);
      fdec[t] = (P.comp_off[o] + (t - P.feat_off[o]) * nc) | (doff(l) << 12) | (nc << 20);
    }
  }
  __syncthreads();
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + w;  // list slot
  double *mom = lds_f + (size_t)w * (S * NM + NC);
  double *mu = mom + S * NM;
  const bool live = i < N;
  const int64_t row = live ? order[i] : 0;  // the slot's centre: its row of the outputs
  if (live) {
    const int64_t q0 = chunk_off[i], q1 = chunk_off[i + 1];
    for (int t = lane; t < S * NM; t += kWave) {
      const int s = t / NM, m = t - s * NM;
      double a = 0.0;
      if (s == P.dens_slot ? m == 0 : ((P.order_mask >> kMT.deg[m]) & 1)) {
        if (q1 - q0 == 1) {
          a = partial[((size_t)q0 * S + s) * NM + m];
        } else {
          for (int64_t q = q0; q < q1; ++q) a += partial[((size_t)q * S + s) * NM + m];
        }
      }
      mom[t] = a;
    }
  }
  wave_lds_sync();
  if (live) {
    for (int t = lane; t < NC; t += kWave) {
      const int32_t d = cdec[t];
      double v = 0.0;
      if (d < 0) {
        v = mom[(d >> 10) & 0xfff];
      } else {
        const int nc = (d >> 22) & 0xf;
        const double *Tl = lds_T + (d & 0x3ff);
        const double *ms = mom + ((d >> 10) & 0xfff);
        for (int mm = 0; mm < nc; ++mm) v += Tl[mm] * ms[mm];
      }
      mu[t] = v;
      if (components) components[(size_t)row * NC + t] = v;
    }
  }
  wave_lds_sync();
  if (live) {
    for (int t = lane; t < NF; t += kWave) {
      const int32_t d = fdec[t];
      double F;
      if (d < 0) {
        F = fabs(mu[d & 0xfff]);
      } else {
        const int nc = (d >> 20) & 0xf;
        const double *mv = mu + (d & 0xfff);
        const double *wl = lds_w + ((d >> 12) & 0xff);
        double a = 0.0;
        for (int cc = 0; cc < nc; ++cc) a += wl[cc] * mv[cc] * mv[cc];
        F = sqrt(a);
      }
      if (F64OUT) ((double *)features)[(size_t)row * NF + t] = F;
      else ((float *)features)[(size_t)row * NF + t] = (float)F;
    }
  }
}

using OverlapFn = void (*)(PlanDev, BatchDev, NbrDev, const double4 *, const int32_t *, double *, const int64_t *,
                           int, int, unsigned long long *, const void *);

// DENS: the plan has the density slot of order -1; SCREEN: per-primitive
// screening (separate instantiations keep both branches out of the loop of
// plans without them)
template <int L, int MODE, bool LDS, bool DENS, bool SCREEN> OverlapFn pick_k(int kb) {
  if (kb <= 4) return k_overlap<L, 4, MODE, LDS, DENS, SCREEN>;
  if (kb <= 8) return k_overlap<L, 8, MODE, LDS, DENS, SCREEN>;
  return k_overlap<L, 16, MODE, LDS, DENS, SCREEN>;
}

template <int MODE, bool LDS, bool DENS, bool SCREEN> OverlapFn pick_l(int lmax, int kb) {
  switch (lmax) {
    case 0: return pick_k<0, MODE, LDS, DENS, SCREEN>(kb);
    case 1: return pick_k<1, MODE, LDS, DENS, SCREEN>(kb);
    case 2: return pick_k<2, MODE, LDS, DENS, SCREEN>(kb);
    case 3: return pick_k<3, MODE, LDS, DENS, SCREEN>(kb);
    default: return pick_k<4, MODE, LDS, DENS, SCREEN>(kb);
  }
}

template <bool LDS, bool DENS, bool SCREEN> OverlapFn pick_d(gmp_precision prec, int lmax, int kb) {
  if (prec == GMP_FP64) return pick_l<ACC_F64, LDS, DENS, SCREEN>(lmax, kb);
  if (prec == GMP_FP32_WIDE) return pick_l<ACC_WIDE, LDS, DENS, SCREEN>(lmax, kb);
  return pick_l<ACC_TWOSUM, LDS, DENS, SCREEN>(lmax, kb);
}

// tabulated radial factors (FP32 modes): no coefficient table, no primitive loop
template <int MODE, bool DENS> OverlapFn pick_tab_l(int lmax) {
  switch (lmax) {
    case 0: return k_overlap<0, 4, MODE, false, DENS, false, true>;
    case 1: return k_overlap<1, 4, MODE, false, DENS, false, true>;
    case 2: return k_overlap<2, 4, MODE, false, DENS, false, true>;
    case 3: return k_overlap<3, 4, MODE, false, DENS, false, true>;
    default: return k_overlap<4, 4, MODE, false, DENS, false, true>;
  }
}
OverlapFn pick_tab(gmp_precision prec, int lmax, bool dens) {
  if (prec == GMP_FP32_WIDE) return dens ? pick_tab_l<ACC_WIDE, true>(lmax) : pick_tab_l<ACC_WIDE, false>(lmax);
  return dens ? pick_tab_l<ACC_TWOSUM, true>(lmax) : pick_tab_l<ACC_TWOSUM, false>(lmax);
}

template <bool LDS> OverlapFn pick_m(gmp_precision prec, int lmax, int kb, bool dens, bool screen) {
  if (screen) return dens ? pick_d<LDS, true, true>(prec, lmax, kb) : pick_d<LDS, false, true>(prec, lmax, kb);
  return dens ? pick_d<LDS, true, false>(prec, lmax, kb) : pick_d<LDS, false, false>(prec, lmax, kb);
}

}  // namespace

// Scratch memory of gmp_features_noalloc: a fixed array in device memory
// (each GPU the library runs on holds its own copy until the process ends).
// Host code never passes the array's name to a kernel: it takes the device
// address from hipGetSymbolAddress once per device and passes that.
constexpr size_t kNoallocScratchBytes = (size_t)GMP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

// Device address of this GPU's scratch array (looked up on the first call on
// each device, with that device current), or null with *err set.
void *noalloc_scratch(size_t *bytes, hipError_t *err) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static void *addr[kMaxDev] = {};
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDev) { *err = hipErrorInvalidDevice; return nullptr; }
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    addr[dev] = ptr;
  }
  *bytes = kNoallocScratchBytes;
  return addr[dev];
}

int chunk_size(const gmp_plan *p) { return p->tuning.chunk_pairs > 0 ? p->tuning.chunk_pairs : 0; }

// groups of cutoff slots per chunk (each a work item of its own)
int slot_groups(const gmp_plan *p) {
  const int g = p->tuning.sigma_groups > 0 ? p->tuning.sigma_groups : 1;
  return g < p->dev.S ? g : (p->dev.S > 0 ? p->dev.S : 1);
}

// upper bound on the number of work items of a batch with at most `pairs` pairs
int64_t max_chunks(const gmp_plan *p, int64_t n_atoms, int64_t pairs) {
  const int kc = chunk_size(p);
  return (n_atoms + (kc > 0 ? pairs / kc + 1 : 0)) * slot_groups(p);
}

static int cus_cached() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, c = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
    cus = c > 0 ? c : 256;
  }
  return cus;
}

int persistent_blocks(const void *fn, size_t smem, int blocks_per_cu) {
  static std::mutex mu;
  static std::map<std::pair<const void *, size_t>, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(fn, smem);
  auto itc = cache.find(key);
  if (itc != cache.end()) {
    const int per_c = itc->second / (cus_cached() > 0 ? cus_cached() : 1);
    return blocks_per_cu > 0 && blocks_per_cu < per_c ? cus_cached() * blocks_per_cu : itc->second;
  }
  int dev = 0, cus = 256, per = 2;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, smem) != hipSuccess || per < 1) per = 1;
  cache[key] = cus * per;
  return blocks_per_cu > 0 && blocks_per_cu < per ? cus * blocks_per_cu : cus * per;
}

void launch_overlap(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, double *partial, int64_t *nch,
                    int64_t *chunk_off, int64_t *scan_aux, unsigned long long *counter, double4 *rw4,
                    int32_t *astruct, int64_t pairs_bound, hipStream_t s) {
  const int64_t N = n_centres(bt), NT = n_total(bt);  // NT >= N
  const int kc = chunk_size(p), ng = slot_groups(p);
  GMP_LAUNCH("overlap_prep", k_overlap_prep, dim3((unsigned)((NT + 255) / 256)), dim3(256), 0, s, bt, nb, kc, ng,
             nch, rw4, astruct, counter);
  scan_i64(nch, chunk_off, N, scan_aux, s);
  const bool f64 = p->prec == GMP_FP64;
  const size_t tab_bytes = (size_t)p->dev.S * p->dev.E * p->dev.kb * kCoefStride * (f64 ? 8 : 4);
  const bool tabulated = p->dev.tab_n > 0 && !f64;
  const bool use_lds = tab_bytes <= 48 * 1024 && !tabulated;
  const size_t smem = use_lds ? tab_bytes : 0;
  const void *tab = f64 ? (const void *)p->dev.coef64 : (const void *)p->dev.coef32;
  const bool dens = p->dev.dens_slot >= 0;
  const bool screen = p->dev.screen != 0;
  OverlapFn fn = tabulated ? pick_tab(p->prec, p->dev.lmax, dens)
                 : use_lds ? pick_m<true>(p->prec, p->dev.lmax, p->dev.kb, dens, screen)
                           : pick_m<false>(p->prec, p->dev.lmax, p->dev.kb, dens, screen);
  const int64_t items_bound = max_chunks(p, N, pairs_bound);
  int64_t blocks = persistent_blocks((const void *)fn, smem, p->tuning.blocks_per_cu);
  const int64_t need = (items_bound + 3) / 4;
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  GMP_LAUNCH("overlap", fn, dim3((unsigned)blocks), dim3(256), smem, s, p->dev, bt, nb, (const double4 *)rw4,
             (const int32_t *)astruct, partial, chunk_off, kc, ng, counter, tab);
}

void launch_finish(const gmp_plan *p, int64_t N, const double *partial, const int64_t *chunk_off,
                   const int32_t *order, void *features, double *components, hipStream_t s) {
  if (N == 0) return;
  const int NM = nmono(p->dev.lmax);
  size_t smem = sizeof(double) * 4 * (size_t)(p->dev.S * NM + p->dev.ncomp_total) +
                sizeof(int32_t) * (size_t)(p->dev.ncomp_total + p->dev.nf);  // + the decode tables
  int64_t blocks = (N + 3) / 4;
  using FinishFn = void (*)(PlanDev, int64_t, const double *, const int64_t *, const int32_t *, void *, double *);
  static const FinishFn fns[2][kMaxL + 1] = {
      {k_finish<0, false>, k_finish<1, false>, k_finish<2, false>, k_finish<3, false>, k_finish<4, false>},
      {k_finish<0, true>, k_finish<1, true>, k_finish<2, true>, k_finish<3, true>, k_finish<4, true>}};
  const int lm = p->dev.lmax < 0 ? 0 : (p->dev.lmax > kMaxL ? kMaxL : p->dev.lmax);
  GMP_LAUNCH("norm", fns[p->prec == GMP_FP64 ? 1 : 0][lm], dim3((unsigned)blocks), dim3(256), smem, s, p->dev, N,
             partial, chunk_off, order, features, components);
}

}  // namespace gmp
