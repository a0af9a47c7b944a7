// Full per-pair feature Jacobian (the paper's feature derivatives with
// respect to atom positions): for centre i and pair p = (j, n) of its list,
//   J[f][k][p] = dF_{i,f} / d d_{p,k},   d_p = R_j + n.cell - R_i,
// from which dF/dR_j (+J), dF/dR_i (-J, summed over the list) and dF/dcell
// (sum (n - m_j + m_i) J) assemble.  It is the adjoint's pair kernel without
// the contraction over features: with the unit upstream gradient the
// per-centre coefficients of each (order l, slot s) describe
// Q_{l,s}(d) = sum_abc (w_abc mu_abc / F_{l,s}) P_abc(d), and feature (l, s)
// gets 2 c'_{l,s}(q) Q d + c_{l,s}(q) grad Q (times the neighbour's
// occupancy); pairs outside a slot's cutoff get 0 for its features.
//
// Layout: feature-major planes over the pair list, jac[(f * 3 + k) * ld + p],
// so consecutive lanes (consecutive pairs) store contiguously.
#include <type_traits>

#include "gmp_internal.h"

namespace gmp {
namespace {

constexpr MonoTable kMT = make_mono_table();

__device__ inline float exp_scaled(float a, float q) { return __builtin_amdgcn_exp2f(a * q); }
__device__ inline double exp_scaled(double a, double q) { return exp(a * q); }
__device__ inline float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fma_(double a, double b, double c) { return fma(a, b, c); }

// Persistent: wavefronts pull (centre, chunk) items; lanes take consecutive
// pairs; the centre's coefficients are staged in LDS per item.
template <int LMAX, int KB, bool F64, bool LDS>
__global__ __launch_bounds__(256) void k_jac_pairs(PlanDev P, BatchDev bt, NbrDev nb, const double4 *rw4,
                                                   const int32_t *astruct, const void *bcoef_, void *jac_,
                                                   int64_t ld, int C, int64_t n_items, unsigned long long *counter,
                                                   const void *tab_global) {
  using T = typename std::conditional<F64, double, float>::type;
  constexpr int NM = nmono(LMAX);
  constexpr int NB = coef_block(LMAX);
  extern __shared__ __align__(16) double lds_dyn[];
  __shared__ int lds_k[kMaxElements];
  const int S = P.S, E = P.E;
  const T *__restrict__ tabg = (const T *)tab_global;
  T *tabl = (T *)lds_dyn;
  const int tab_n = LDS ? S * E * KB * kCoefStride : 0;
  if (LDS)
    for (int idx = threadIdx.x; idx < tab_n; idx += blockDim.x) tabl[idx] = tabg[idx];
  for (int e = threadIdx.x; e < E; e += blockDim.x) lds_k[e] = P.kcount[e];
  __syncthreads();
  const int lane = lane_id();
  T *jac = (T *)jac_;
  const int mask = P.order_mask, dens = P.dens_slot;
  T *bcoef = tabl + tab_n + (size_t)(threadIdx.x / kWave) * S * NB;
  for (;;) {
    const int64_t item = next_item(counter);
    if (item >= n_items) break;
    const int64_t k = item / C;  // list slot
    const int c = (int)(item - k * C);
    if (nb.offsets[k + 1] > nb.capacity) continue;  // list not written (overflowed no-sync build)
    const int64_t i = nb.order[k];  // its centre
    {
      const T *src = (const T *)bcoef_ + (size_t)i * S * NB;
      for (int t = lane; t < S * NB; t += kWave) bcoef[t] = src[t];
      wave_lds_sync();
    }
    const int64_t g = centre_base(bt) + i;
    const int st = astruct[g];
    const Cell9 cell = load_cell(bt.cell + 9 * (int64_t)st);
    const int pbc = bt.pbc[st] & 7;
    const double4 ri4 = rw4[g];
    const int64_t base = nb.offsets[k];
    const int cnt = (int)(nb.offsets[k + 1] - base);
    const int clo = (int)((int64_t)cnt * c / C), chi = (int)((int64_t)cnt * (c + 1) / C);
    const int end_lane = lane < S ? nb.sigma_end[k * S + lane] : 0;
    for (int p0 = clo; p0 < chi; p0 += kWave) {
      const int p = p0 + lane;
      const bool act = p < chi && base + p < ld;
      int32_t j = (int32_t)g, w = 0;
      if (act) { j = nb.j[base + p]; w = nb.shift[base + p]; }
      const double4 rj = rw4[j];
      double shx = 0.0, shy = 0.0, shz = 0.0;
      if (pbc) image_shift(cell, shift_n(w, 0), shift_n(w, 1), shift_n(w, 2), shx, shy, shz);
      const double dx = (rj.x - ri4.x) + shx;
      const double dy = (rj.y - ri4.y) + shy;
      const double dz = (rj.z - ri4.z) + shz;
      const double q = (dx * dx + dy * dy) + dz * dz;
      const T xv = (T)dx, yv = (T)dy, zv = (T)dz, qv = (T)q, occ = (T)rj.w;
      const int e = shift_species(w);
      const int K = lds_k[e];
      T mono[NM];
      mono[0] = (T)1;
#pragma unroll
      for (int m = 1; m < NM; ++m) {
        const T v = kMT.var[m] == 0 ? xv : (kMT.var[m] == 1 ? yv : zv);
        mono[m] = v * mono[kMT.parent[m]];
      }
      T *dst = jac + base + p;
      for (int s = 0; s < S; ++s) {
        const bool inside = act && p < __builtin_amdgcn_readlane(end_lane, s);
        const size_t roff = ((size_t)(s * E + e) * KB) * kCoefStride;
        const T *bc = (const T *)__builtin_assume_aligned(bcoef + (size_t)s * NB, 16);
        if (s == dens) {  // local density: dF/dd = 2 rho'(q) sign(rho) d
          T cp0 = (T)0;
          if (inside) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
              if (k < K) {
                const size_t o = roff + k * kCoefStride;
                if (P.screen && !((float)q <= (float)(LDS ? tabl[o + 7] : tabg[o + 7]))) continue;
                const T ek = exp_scaled(LDS ? tabl[o] : tabg[o], qv);
                cp0 = fma_(LDS ? tabl[o + 1] : tabg[o + 1], (LDS ? tabl[o + 6] : tabg[o + 6]) * ek, cp0);
              }
            }
          }
          const T A2 = (T)2 * cp0 * bc[0] * occ;
          const int64_t f = P.feat_off[P.dens_order];
          if (act) {
            dst[(f * 3 + 0) * ld] = A2 * xv;
            dst[(f * 3 + 1) * ld] = A2 * yv;
            dst[(f * 3 + 2) * ld] = A2 * zv;
          }
          continue;
        }
        T cl[LMAX + 1], cp[LMAX + 1];
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) { cl[l] = (T)0; cp[l] = (T)0; }
        bool radial_done = false;
        if constexpr (!F64) {
          if (inside && !P.screen) {
            // as in the adjoint kernel: zero rows past an element's own count,
            // the plan's largest count for every lane, row k+1 read ahead
            const float *row = (LDS ? tabl : tabg) + roff;
            const int kmx = P.kmax;
            float4 ra = *(const float4 *)row, rb4 = *(const float4 *)(row + 4);
            auto row_step = [&](int k) {
              float4 na, nb4;
              if (k + 1 < KB) { na = *(const float4 *)(row + (k + 1) * kCoefStride); nb4 = *(const float4 *)(row + (k + 1) * kCoefStride + 4); }
              asm volatile("" ::: "memory");
              const T ek = exp_scaled(ra.x, qv);
              const T gk = rb4.z * ek;
              const T av[5] = {ra.y, ra.z, ra.w, rb4.x, rb4.y};
#pragma unroll
              for (int l = 0; l <= LMAX; ++l) {
                cl[l] = fma_(av[l], ek, cl[l]);
                cp[l] = fma_(av[l], gk, cp[l]);
              }
              if (k + 1 < KB) { ra = na; rb4 = nb4; }
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
            radial_done = true;
          }
        }
        if (inside && !radial_done) {
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            if (k < K) {
              const size_t o = roff + k * kCoefStride;
              if (P.screen && !((float)q <= (float)(LDS ? tabl[o + 7] : tabg[o + 7]))) continue;
              const T ek = exp_scaled(LDS ? tabl[o] : tabg[o], qv);
              const T gk = (LDS ? tabl[o + 6] : tabg[o + 6]) * ek;
#pragma unroll
              for (int l = 0; l <= LMAX; ++l) {
                const T al = LDS ? tabl[o + 1 + l] : tabg[o + 1 + l];
                cl[l] = fma_(al, ek, cl[l]);
                cp[l] = fma_(al, gk, cp[l]);
              }
            }
          }
        }
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
          if (!((mask >> l) & 1)) continue;
          // the polynomial and its gradient from the same coefficients, as in
          // the adjoint pair kernel
          T Q = (T)0, gx = (T)0, gy = (T)0, gz = (T)0;
#pragma unroll
          for (int mm = 0; mm < ncomp(l); ++mm) {
            const int m = doff(l) + mm;
            const T Mv = bc[m];
            Q = fma_(Mv, mono[m], Q);
            const int a = kMT.ea[m], b = kMT.eb[m], c = kMT.ec[m];
            if (a >= 1) gx = fma_(a == 1 ? Mv : (T)a * Mv, mono[doff(l - 1) + midx(l - 1, a - 1, b)], gx);
            if (b >= 1) gy = fma_(b == 1 ? Mv : (T)b * Mv, mono[doff(l - 1) + midx(l - 1, a, b - 1)], gy);
            if (c >= 1) gz = fma_(c == 1 ? Mv : (T)c * Mv, mono[doff(l - 1) + midx(l - 1, a, b)], gz);
          }
          const T A2 = (T)2 * cp[l] * Q;
          const int64_t f = P.feat_off[P.order_idx[l]] + s;
          if (act) {
            dst[(f * 3 + 0) * ld] = fma_(A2, xv, cl[l] * gx) * occ;
            dst[(f * 3 + 1) * ld] = fma_(A2, yv, cl[l] * gy) * occ;
            dst[(f * 3 + 2) * ld] = fma_(A2, zv, cl[l] * gz) * occ;
          }
        }
      }
    }
    wave_lds_sync();  // every lane is done with this centre's coefficients
  }
}

using JacFn = void (*)(PlanDev, BatchDev, NbrDev, const double4 *, const int32_t *, const void *, void *, int64_t,
                       int, int64_t, unsigned long long *, const void *);
template <int L, bool F64, bool LDS> JacFn pick_kb(int kb) {
  if (kb <= 4) return k_jac_pairs<L, 4, F64, LDS>;
  if (kb <= 8) return k_jac_pairs<L, 8, F64, LDS>;
  return k_jac_pairs<L, 16, F64, LDS>;
}
template <bool F64, bool LDS> JacFn pick_jac(int lmax, int kb) {
  switch (lmax) {
    case 0: return pick_kb<0, F64, LDS>(kb);
    case 1: return pick_kb<1, F64, LDS>(kb);
    case 2: return pick_kb<2, F64, LDS>(kb);
    case 3: return pick_kb<3, F64, LDS>(kb);
    default: return pick_kb<4, F64, LDS>(kb);
  }
}

}  // namespace

void launch_bwd_coef(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const double *components,
                     const void *grad_features, const WsLayout &L, hipStream_t s);
int persistent_blocks(const void *fn, size_t smem, int blocks_per_cu);

void launch_jacobian(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const double *components, void *jac,
                     int64_t ld, const WsLayout &L, int C, hipStream_t s) {
  const int64_t N = n_centres(bt);
  if (N == 0) return;
  launch_bwd_coef(p, bt, nb, components, nullptr, L, s);
  const bool f64 = p->prec == GMP_FP64;
  const int64_t n_items = N * (int64_t)C;
  const size_t tab_bytes = (size_t)p->dev.S * p->dev.E * p->dev.kb * kCoefStride * (f64 ? 8 : 4);
  const bool use_lds = tab_bytes <= 48 * 1024;
  const size_t tsm = (use_lds ? tab_bytes : 0) + 4 * (size_t)p->dev.S * coef_block(p->dev.lmax) * (f64 ? 8 : 4);
  const void *tab = f64 ? (const void *)p->dev.coef64 : (const void *)p->dev.coef32;
  JacFn fn = f64 ? (use_lds ? pick_jac<true, true>(p->dev.lmax, p->dev.kb) : pick_jac<true, false>(p->dev.lmax, p->dev.kb))
                 : (use_lds ? pick_jac<false, true>(p->dev.lmax, p->dev.kb)
                            : pick_jac<false, false>(p->dev.lmax, p->dev.kb));
  int64_t pb = persistent_blocks((const void *)fn, tsm, p->tuning.blocks_per_cu);
  if (pb > (n_items + 3) / 4) pb = (n_items + 3) / 4;
  if (pb < 1) pb = 1;
  GMP_LAUNCH("jacobian", fn, dim3((unsigned)pb), dim3(256), tsm, s, p->dev, bt, nb, (const double4 *)L.rw4,
             (const int32_t *)L.astruct, L.bcoef, jac, ld, C, n_items, L.counter, tab);
}

}  // namespace gmp
