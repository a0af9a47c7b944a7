// Overlap kernel (multipole moments) and norm kernel.
//
// Closed form of one pair's contribution (derived from the Gaussian product
// theorem and the mean-value property of harmonic polynomials; the paper
// defines the probe as an MCSH angular probe times a Gaussian radial probe
// and the density as per-element Gaussian primitives):
//   mu_{i,l,s,abc} += c_{l,s,e_j}(q) P_abc(d),
//   c_{l,s,e}(q) = sum_k A_{l,s,e,k} exp(-gamma_{s,e,k} q).
// P_abc is a homogeneous polynomial of degree l, so the kernel accumulates
// the Cartesian moments  M_{i,s,m} = sum_j c_{deg m,s,e_j}(q_j) x^a y^b z^c
// of every monomial m of each requested degree, and the norm kernel maps
// moments to components with the plan's exact integer matrices (FP64).
//
// Work decomposition: one wavefront per (centre, sigma group, chunk of the
// centre's list); lanes take consecutive pairs.  Each centre's list is
// grouped by neighbour species, so within a segment the density primitives
// are wavefront-uniform and are read through the scalar cache; within a
// segment the pairs a sigma uses form a prefix, so a sigma's lanes stop at
// its own cutoff without testing q.
//
// Precision policies:
//   F64=false  displacement rounded to FP32; monomials, exp2, radial sums and
//              products in FP32; accumulation as FP32 (hi, lo) two-sum pairs;
//              cross-lane reduction in FP64.
//   F64=true   everything FP64 (exp in FP64), plain accumulation.
#include "gmp_internal.h"

namespace gmp {
namespace {

constexpr MonoTable kMT = make_mono_table();

template <bool F64> struct Real;
template <> struct Real<false> { using T = float; };
template <> struct Real<true> { using T = double; };

__device__ inline float exp_scaled(float a, float q) { return __builtin_amdgcn_exp2f(a * q); }
__device__ inline double exp_scaled(double a, double q) { return exp(a * q); }

__device__ inline float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fma_(double a, double b, double c) { return fma(a, b, c); }

template <bool F64> __device__ inline const typename Real<F64>::T *coef_ptr(const PlanDev &P, int s, int e);
template <> __device__ inline const float *coef_ptr<false>(const PlanDev &P, int s, int e) {
  return P.coef32 + ((size_t)(s * P.E + e) * P.kmax) * kCoefStride;
}
template <> __device__ inline const double *coef_ptr<true>(const PlanDev &P, int s, int e) {
  return P.coef64 + ((size_t)(s * P.E + e) * P.kmax) * kCoefStride;
}

// Accumulator of one sigma: two-sum pairs in FP32, plain sum in FP64.
template <bool F64, int NM> struct Acc;
template <int NM> struct Acc<false, NM> {
  float hi[NM], lo[NM];
  __device__ void zero() {
#pragma unroll
    for (int m = 0; m < NM; ++m) { hi[m] = 0.f; lo[m] = 0.f; }
  }
  __device__ void add(int m, float p) {
    float s = hi[m] + p;
    float bp = s - hi[m];
    float ap = s - bp;
    lo[m] += (hi[m] - ap) + (p - bp);
    hi[m] = s;
  }
  __device__ double value(int m) const { return (double)hi[m] + (double)lo[m]; }
};
template <int NM> struct Acc<true, NM> {
  double v[NM];
  __device__ void zero() {
#pragma unroll
    for (int m = 0; m < NM; ++m) v[m] = 0.0;
  }
  __device__ void add(int m, double p) { v[m] += p; }
  __device__ double value(int m) const { return v[m]; }
};

// Chunks of one centre's list: fixed-size pieces of kc pairs (kc = 0: whole
// list), so the decomposition of a centre depends on its own list only and
// a batched launch sums in the same order as a launch over one structure.
__global__ void k_chunk_count(NbrDev nb, int64_t N, int kc, int64_t *nch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t cnt = nb.offsets[i + 1] - nb.offsets[i];
  nch[i] = kc > 0 ? (cnt > kc ? (cnt + kc - 1) / kc : 1) : 1;
}

__device__ inline int64_t centre_of_chunk(const int64_t *chunk_off, int64_t N, int64_t q) {
  int64_t lo = 0, hi = N;  // chunk_off[lo] <= q < chunk_off[lo+1]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= q) lo = mid; else hi = mid;
  }
  return lo;
}

template <int LMAX, int G, bool F64>
__global__ __launch_bounds__(256) void k_overlap(PlanDev P, BatchDev bt, NbrDev nb, double *partial,
                                                 const int64_t *chunk_off, int n_groups, int kc,
                                                 int64_t n_items) {
  using T = typename Real<F64>::T;
  constexpr int NM = nmono(LMAX);
  const int lane = lane_id();
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (item >= n_items) return;
  const int64_t N = bt.n_atoms;
  const int64_t qc = item / n_groups;
  const int g = (int)(item - qc * n_groups);
  if (qc >= chunk_off[N]) return;
  const int64_t i = centre_of_chunk(chunk_off, N, qc);
  const int c = (int)(qc - chunk_off[i]);
  const int S = P.S, E = P.E;

  const int st = struct_of_atom(bt.atom_offsets, bt.n_structs, i);
  const double *cell = bt.cell + 9 * (int64_t)st;
  const int pbc = bt.pbc[st] & 7;
  const double rix = nb.rw[i], riy = nb.rw[N + i], riz = nb.rw[2 * N + i];
  const int64_t base = nb.offsets[i];
  const int cnt = (int)(nb.offsets[i + 1] - base);
  const int clo = kc > 0 ? c * kc : 0;
  const int chi = kc > 0 ? (clo + kc < cnt ? clo + kc : cnt) : cnt;

  int sg[G];
#pragma unroll
  for (int t = 0; t < G; ++t) {
    int gi = g * G + t;
    sg[t] = gi < S ? P.sig_order[gi] : -1;
  }
  Acc<F64, NM> acc[G];
#pragma unroll
  for (int t = 0; t < G; ++t) acc[t].zero();

  for (int e = 0; e < E; ++e) {
    const int es = nb.elem_start[i * (E + 1) + e];
    const int lo = es > clo ? es : clo;
    int endg[G];
    int emax = lo;
#pragma unroll
    for (int t = 0; t < G; ++t) {
      int en = lo;
      if (sg[t] >= 0) {
        en = nb.sigma_end[(i * E + e) * S + sg[t]];
        en = en < chi ? en : chi;
      }
      endg[t] = en;
      emax = en > emax ? en : emax;
    }
    if (emax <= lo) continue;
    const int K = P.kcount[e];
    for (int p0 = lo; p0 < emax; p0 += kWave) {
      const int p = p0 + lane;
      const bool act = p < emax;
      int32_t j = (int32_t)i, w = 0;
      if (act) { j = nb.j[base + p]; w = nb.shift[base + p]; }
      double shx = 0.0, shy = 0.0, shz = 0.0;
      if (pbc) image_shift(cell, shift_n(w, 0), shift_n(w, 1), shift_n(w, 2), shx, shy, shz);
      const double dx = (nb.rw[j] - rix) + shx;
      const double dy = (nb.rw[N + j] - riy) + shy;
      const double dz = (nb.rw[2 * N + j] - riz) + shz;
      const double q = (dx * dx + dy * dy) + dz * dz;
      const T xv = (T)dx, yv = (T)dy, zv = (T)dz, qv = (T)q;
      T mono[NM];
      mono[0] = (T)1;
#pragma unroll
      for (int m = 1; m < NM; ++m) {
        const T v = kMT.var[m] == 0 ? xv : (kMT.var[m] == 1 ? yv : zv);
        mono[m] = v * mono[kMT.parent[m]];
      }
#pragma unroll
      for (int t = 0; t < G; ++t) {
        if (p < endg[t]) {
          const T *cf = coef_ptr<F64>(P, sg[t], e);
          T cl[LMAX + 1];
#pragma unroll
          for (int l = 0; l <= LMAX; ++l) cl[l] = (T)0;
          for (int k = 0; k < K; ++k) {
            const T ek = exp_scaled(cf[k * kCoefStride], qv);
#pragma unroll
            for (int l = 0; l <= LMAX; ++l) cl[l] = fma_(cf[k * kCoefStride + 1 + l], ek, cl[l]);
          }
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            if ((P.order_mask >> kMT.deg[m]) & 1) acc[t].add(m, cl[kMT.deg[m]] * mono[m]);
          }
        }
      }
    }
  }
  // cross-lane reduction in FP64; partial layout [chunk][sigma][monomial]
#pragma unroll
  for (int t = 0; t < G; ++t) {
    if (sg[t] < 0) continue;
    double *dst = partial + ((size_t)qc * S + sg[t]) * NM;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      if (!((P.order_mask >> kMT.deg[m]) & 1)) continue;
      const double v = wave_sum(acc[t].value(m));
      if (lane == (m & (kWave - 1))) dst[m] = v;
    }
  }
}

// One wavefront per centre: sum chunk partials in order, map moments to
// components with the exact integer matrices, then the weighted norm
// F_{l,s} = sqrt(sum_abc l!/(a!b!c!) mu_abc^2).
template <bool F64OUT>
__global__ __launch_bounds__(256) void k_finish(PlanDev P, int64_t N, const double *partial,
                                                const int64_t *chunk_off, void *features, double *components) {
  extern __shared__ double lds_f[];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + w;
  const int S = P.S, NM = nmono(P.lmax);
  double *mom = lds_f + (size_t)w * (S * NM + P.ncomp_total);
  double *mu = mom + S * NM;
  const bool live = i < N;
  if (live) {
    for (int t = lane; t < S * NM; t += kWave) {
      const int s = t / NM, m = t - s * NM;
      double a = 0.0;
      if ((P.order_mask >> kMT.deg[m]) & 1) {
        const int64_t q1 = chunk_off[i + 1];
        for (int64_t q = chunk_off[i]; q < q1; ++q) a += partial[((size_t)q * S + s) * NM + m];
      }
      mom[t] = a;
    }
  }
  wave_lds_sync();
  if (live) {
    for (int t = lane; t < P.ncomp_total; t += kWave) {
      int o = 0;
      while (o + 1 < P.n_orders && P.comp_off[o + 1] <= t) ++o;
      const int l = P.orders[o], nc = ncomp(l);
      const int r = t - P.comp_off[o];
      const int s = r / nc, cc = r - s * nc;
      const double *Tl = P.T + P.toff[l] + cc * nc;
      const double *ms = mom + s * NM + doff(l);
      double v = 0.0;
      for (int mm = 0; mm < nc; ++mm) v += Tl[mm] * ms[mm];
      mu[t] = v;
      if (components) components[(size_t)i * P.ncomp_total + t] = v;
    }
  }
  wave_lds_sync();
  if (live) {
    for (int t = lane; t < P.nf; t += kWave) {
      const int o = t / S, s = t - o * S;
      const int l = P.orders[o], nc = ncomp(l);
      const double *mv = mu + P.comp_off[o] + s * nc;
      double a = 0.0;
      for (int cc = 0; cc < nc; ++cc) a += P.weight[doff(l) + cc] * mv[cc] * mv[cc];
      const double F = sqrt(a);
      if (F64OUT) ((double *)features)[(size_t)i * P.nf + t] = F;
      else ((float *)features)[(size_t)i * P.nf + t] = (float)F;
    }
  }
}

using OverlapFn = void (*)(PlanDev, BatchDev, NbrDev, double *, const int64_t *, int, int, int64_t);

template <int L, bool F64> OverlapFn pick_g(int G) {
  if (G >= 4) return k_overlap<L, 4, F64>;
  if (G == 2) return k_overlap<L, 2, F64>;
  return k_overlap<L, 1, F64>;
}

template <bool F64> OverlapFn pick(int lmax, int G) {
  switch (lmax) {
    case 0: return pick_g<0, F64>(G);
    case 1: return pick_g<1, F64>(G);
    case 2: return pick_g<2, F64>(G);
    case 3: return pick_g<3, F64>(G);
    default: return pick_g<4, F64>(G);
  }
}

}  // namespace

int normalized_group(const gmp_plan *p) {
  int G = p->tuning.sigma_group;
  if (G >= 4) G = 4; else if (G >= 2) G = 2; else G = 1;
  return G;
}

int chunk_size(const gmp_plan *p) { return p->tuning.chunk_pairs > 0 ? p->tuning.chunk_pairs : 0; }

// upper bound on the number of chunks of a batch with at most `pairs` pairs
int64_t max_chunks(const gmp_plan *p, int64_t n_atoms, int64_t pairs) {
  const int kc = chunk_size(p);
  return n_atoms + (kc > 0 ? pairs / kc + 1 : 0);
}

void launch_overlap(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, double *partial, int64_t *nch,
                    int64_t *chunk_off, int64_t *scan_aux, int64_t pairs_bound, hipStream_t s) {
  const int64_t N = bt.n_atoms;
  const int G = normalized_group(p);
  const int n_groups = (p->dev.S + G - 1) / G;
  const int kc = chunk_size(p);
  GMP_LAUNCH("overlap_chunks", k_chunk_count, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, nb, N, kc, nch);
  scan_i64(nch, chunk_off, N, scan_aux, s);
  const int64_t n_items = max_chunks(p, N, pairs_bound) * n_groups;
  const int64_t blocks = (n_items + 3) / 4;
  OverlapFn fn = p->prec == GMP_FP64 ? pick<true>(p->dev.lmax, G) : pick<false>(p->dev.lmax, G);
  GMP_LAUNCH("overlap", fn, dim3((unsigned)blocks), dim3(256), 0, s, p->dev, bt, nb, partial, chunk_off, n_groups,
             kc, n_items);
}

void launch_finish(const gmp_plan *p, int64_t N, const double *partial, const int64_t *chunk_off, void *features,
                   double *components, hipStream_t s) {
  if (N == 0) return;
  const int NM = nmono(p->dev.lmax);
  size_t smem = sizeof(double) * 4 * (size_t)(p->dev.S * NM + p->dev.ncomp_total);
  int64_t blocks = (N + 3) / 4;
  if (p->prec == GMP_FP64)
    GMP_LAUNCH("norm", k_finish<true>, dim3((unsigned)blocks), dim3(256), smem, s, p->dev, N, partial, chunk_off,
               features, components);
  else
    GMP_LAUNCH("norm", k_finish<false>, dim3((unsigned)blocks), dim3(256), smem, s, p->dev, N, partial, chunk_off,
               features, components);
}

}  // namespace gmp
