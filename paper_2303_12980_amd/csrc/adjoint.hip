// Adjoint of the features: dL/dR and dL/dcell for L = sum G F (the paper's
// feature derivatives with respect to atom positions, contracted with an
// upstream gradient).
//
//   W_{i,l,s,abc} = G_{i,l,s} w_abc mu_abc / F_{i,l,s}   (0 when F = 0)
//   For centre i and sigma s the polynomial Q_{i,s,l}(d) = sum_abc W P_abc(d)
//   is stored in monomial form (coefficients M); the pair kernel evaluates
//   it and its gradient (the exponents are constants) from M, so per pair
//   v_{ijn} = grad_d sum_{s,l} c_{l,s}(q) Q_{i,s,l}(d)
//          = sum_{s,l} [ 2 c'_{l,s}(q) Q_{i,s,l}(d) d + c_{l,s}(q) grad Q_{i,s,l}(d) ].
//   dL/dR_j += v, dL/dR_i -= v, dL/da_m += (n_m - m_{j,m} + m_{i,m}) v,
//   v carrying the neighbour's occupancy factor (disordered structures).
//   The local density of order -1 (F = |rho|) has W = G rho / |rho| on the
//   degree-0 coefficient of its own cutoff slot, whose radial factor is
//   sum_k B exp(-beta q).
//
// Determinism without atomics: every centre writes the v of its own pairs
// into a per-pair buffer; each atom then gathers, in list order, -v of its
// own pairs plus v of the reverse pairs (j, i, -n) found through the
// reverse-pair index; the cell gradient is a fixed-order per-structure
// reduction of per-atom partials.
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


// One wavefront per index: centres get their coefficients, every index
// (atoms, and reference points) its structure and packed position.  The
// centre's components are staged in LDS, and where every feature and every
// (slot, monomial) coefficient comes from is decoded once per workgroup
// into LDS tables.
template <int LMAX, bool F64>
__global__ __launch_bounds__(256) void k_bwd_coef(PlanDev P, BatchDev bt, NbrDev nb, const double *components,
                                                  const void *grad_features, void *bcoef, double4 *rw4,
                                                  int32_t *astruct, unsigned long long *counter) {
  const int64_t N = n_centres(bt);
  using T = typename Real<F64>::T;
  extern __shared__ double lds_b[];
  // moment -> component maps of all orders and the multinomial weights,
  // staged in LDS once per workgroup (read with lane-varying indices)
  __shared__ double lds_T[kTmat];
  __shared__ double lds_w[nmono(kMaxL)];
  // block sizes are compile-time constants (the index splits below are then
  // multiplications, not integer divisions)
  constexpr int NM = nmono(LMAX), NB = coef_block(LMAX);
  const int S = P.S, NC = P.ncomp_total, NF = P.nf;
  // decode tables after the four wavefronts' buffers.  Feature t: component
  // offset | weight offset << 12 | length << 20 (bit 31: the density
  // feature).  Coefficient (s, m): component offset | T column << 12 |
  // length << 22, or bit 31 alone (zero: order not requested, or a density
  // slot moment past degree 0), or bit 31 | bit 30 | component offset (the
  // density coefficient); mfeat: its feature | weight offset << 12.
  int32_t *fdec = (int32_t *)(lds_b + (size_t)4 * (NF + S * NM + NC));
  int32_t *mdec = fdec + NF;
  int32_t *mfeat = mdec + S * NM;
  for (int t = threadIdx.x; t < kTmat; t += blockDim.x) lds_T[t] = P.T[t];
  for (int t = threadIdx.x; t < nmono(kMaxL); t += blockDim.x) lds_w[t] = P.weight[t];
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
  for (int t = threadIdx.x; t < S * NM; t += blockDim.x) {
    const int sl = t / NM, m = t - sl * NM;
    const int l = kMT.deg[m];
    int32_t d = (int32_t)0x80000000u, f = 0;
    if (sl == P.dens_slot) {
      if (m == 0) {
        const int o = P.dens_order;
        d = (int32_t)(0xC0000000u | (uint32_t)P.comp_off[o]);
        f = P.feat_off[o];
      }
    } else if (P.order_idx[l] >= 0) {
      const int o = P.order_idx[l], nc = ncomp(l), mm = m - doff(l);
      d = (P.comp_off[o] + sl * nc) | ((P.toff[l] + mm) << 12) | (nc << 22);
      f = (P.feat_off[o] + sl) | (doff(l) << 12);
    }
    mdec[t] = d;
    mfeat[t] = f;
  }
  __syncthreads();
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + w;
  double *scale = lds_b + (size_t)w * (NF + S * NM + NC);  // [nf]
  double *M = scale + NF;                                  // [S][NM]
  double *mus = M + S * NM;                                // [ncomp_total] the centre's components
  const bool live = i < N;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0ull;  // work items of the pair kernel
  // AoS wrapped position (one 32-byte gather per neighbour in the pair kernel)
  if (i < n_total(bt) && lane == 0) {
    const int st = struct_of_index(bt, i);
    astruct[i] = st;
    rw4[i] = wrapped_position(bt, nb, i, st);
  }
  if (live) {
    const double *mu = components + (size_t)i * NC;
    for (int t = lane; t < NC; t += kWave) mus[t] = mu[t];
  }
  wave_lds_sync();
  if (live) {
    for (int t = lane; t < NF; t += kWave) {
      const int32_t d = fdec[t];
      double F;
      if (d < 0) {
        F = fabs(mus[d & 0xfff]);
      } else {
        const int nc = (d >> 20) & 0xf;
        const double *mv = mus + (d & 0xfff);
        const double *wl = lds_w + ((d >> 12) & 0xff);
        double a = 0.0;
        for (int cc = 0; cc < nc; ++cc) a += wl[cc] * mv[cc] * mv[cc];
        F = sqrt(a);
      }
      // unit upstream gradient (grad_features null): the coefficients of dF/dd per feature
      const double G = grad_features ? (double)((const T *)grad_features)[(size_t)i * NF + t] : 1.0;
      scale[t] = F > 0.0 ? G / F : 0.0;
    }
  }
  wave_lds_sync();
  if (live) {
    // M_{s,m} = sum_abc W_abc T_l[abc][m],  W_abc = scale w_abc mu_abc
    for (int t = lane; t < S * NM; t += kWave) {
      const int32_t d = mdec[t];
      const int32_t f = mfeat[t];
      double v = 0.0;
      if (d < 0) {
        if (d & 0x40000000) v = mus[d & 0xfff] * scale[f & 0xfff];  // density coefficient
      } else {
        const int nc = (d >> 22) & 0xf;
        const double *mv = mus + (d & 0xfff);
        const double *Tc = lds_T + ((d >> 12) & 0x3ff);
        const double *wl = lds_w + ((f >> 12) & 0xff);
        for (int cc = 0; cc < nc; ++cc) v += wl[cc] * mv[cc] * Tc[cc * nc];
        v *= scale[f & 0xfff];
      }
      M[t] = v;
    }
  }
  wave_lds_sync();
  if (live) {
    T *out = (T *)bcoef + (size_t)i * S * NB;
    for (int t = lane; t < S * NB; t += kWave) {
      const int s = t / NB, r = t - s * NB;
      const double v = r < NM ? M[s * NM + r] : 0.0;
      out[t] = (T)v;
    }
  }
}

// Per-pair adjoint vectors, persistent: wavefronts pull (centre, chunk)
// items.  Lanes take consecutive pairs of the centre's list; a pair is used
// by every sigma whose prefix contains it.  Radial coefficients come from
// the LDS copy of the plan table (row of the lane's neighbour species); the
// centre's polynomial coefficients M are staged in LDS per item and read
// wavefront-uniformly (the gradient reuses them: one LDS value per monomial).  The loads of pair data (j, shift) run two
// steps ahead and the gathers of the neighbours' wrapped positions one step
// ahead.  Dynamic LDS: [coefficient table if staged][4 wavefronts][S * NB].
template <int LMAX, int KB, bool F64, bool LDS, bool SCREEN>
__global__ __launch_bounds__(256) void k_bwd_pairs(PlanDev P, BatchDev bt, NbrDev nb, const double4 *rw4,
                                                   const int32_t *astruct, const void *bcoef_, void *vbuf_, int C,
                                                   int64_t n_items,
                                                   unsigned long long *counter, const void *tab_global) {
  using T = typename Real<F64>::T;
  constexpr int NM = nmono(LMAX);
  constexpr int NB = coef_block(LMAX);
  extern __shared__ __align__(16) double lds_dyn[];
  __shared__ int lds_k[kMaxElements];
  const int S = P.S, E = P.E;
  const T *__restrict__ tabg = (const T *)tab_global;
  T *tabl = (T *)lds_dyn;
  // LDS copy with a 16-byte gap after every (slot, element) block: lanes of
  // different species then read their rows from different banks
  constexpr int BLK = KB * kCoefStride, BLKL = BLK + 16 / (int)sizeof(T);
  const int tab_n = LDS ? S * E * BLKL : 0;
  if (LDS)
    for (int idx = threadIdx.x; idx < S * E * BLK; idx += blockDim.x) tabl[(idx / BLK) * BLKL + idx % BLK] = tabg[idx];
  for (int e = threadIdx.x; e < E; e += blockDim.x) lds_k[e] = P.kcount[e];
  __syncthreads();
  const int lane = lane_id();
  T *vbuf = (T *)vbuf_;
  const int mask = P.order_mask, dens = P.dens_slot;
  T *bcoef = tabl + tab_n + (size_t)(threadIdx.x / kWave) * S * NB;
  for (;;) {
    const int64_t item = next_item(counter);
    if (item >= n_items) break;
    const int64_t k = item / C;   // list slot
    const int c = (int)(item - k * C);
    if (nb.offsets[k + 1] > nb.capacity) continue;  // list not written (overflowed no-sync build)
    const int64_t i = nb.order[k];  // its centre
    {
      const T *src = (const T *)bcoef_ + (size_t)i * S * NB;
      for (int t = lane; t < S * NB; t += kWave) bcoef[t] = src[t];
      wave_lds_sync();
    }
    const int64_t g = centre_base(bt) + i;  // index of the centre (atom, or reference point)
    const int st = astruct[g];
    const Cell9 cell = load_cell(bt.cell + 9 * (int64_t)st);
    const int pbc = bt.pbc[st] & 7;
    const double4 ri4 = rw4[g];
    const double rix = ri4.x, riy = ri4.y, riz = ri4.z;
    const int64_t base = nb.offsets[k];
    const int cnt = (int)(nb.offsets[k + 1] - base);
    const int clo = (int)((int64_t)cnt * c / C), chi = (int)((int64_t)cnt * (c + 1) / C);
    // sigma prefix ends, one per lane (lane s <-> sigma s)
    const int end_lane = lane < S ? nb.sigma_end[k * S + lane] : 0;
    // pipeline: (jb, wb, rb) current step, (jc, wc) the step after
    const int32_t ii = (int32_t)g;  // idle lanes read the centre's own packed position
    int32_t jb = ii, wb = 0, jc = ii, wc = 0;
    if (clo + lane < chi) { jb = nb.j[base + clo + lane]; wb = nb.shift[base + clo + lane]; }
    if (clo + kWave + lane < chi) { jc = nb.j[base + clo + kWave + lane]; wc = nb.shift[base + clo + kWave + lane]; }
    double4 rb = rw4[jb];
    for (int p0 = clo; p0 < chi; p0 += kWave) {
      const int p = p0 + lane;
      const bool act = p < chi;
      const int32_t w = wb;
      const double rjx = rb.x, rjy = rb.y, rjz = rb.z, occj = rb.w;  // w: occupancy of j
      rb = rw4[jc];
      wb = wc;
      jc = ii;
      wc = 0;
      if (p + 2 * kWave < chi) { jc = nb.j[base + p + 2 * kWave]; wc = nb.shift[base + p + 2 * kWave]; }
      double shx = 0.0, shy = 0.0, shz = 0.0;
      if (pbc) image_shift(cell, shift_n(w, 0), shift_n(w, 1), shift_n(w, 2), shx, shy, shz);
      const double dx = (rjx - rix) + shx;
      const double dy = (rjy - riy) + shy;
      const double dz = (rjz - riz) + shz;
      const double q = (dx * dx + dy * dy) + dz * dz;
      const T xv = (T)dx, yv = (T)dy, zv = (T)dz, qv = (T)q;
      const int e = shift_species(w);
      const int K = lds_k[e];
      T mono[NM];
      mono[0] = (T)1;
#pragma unroll
      for (int m = 1; m < NM; ++m) {
        const T v = kMT.var[m] == 0 ? xv : (kMT.var[m] == 1 ? yv : zv);
        mono[m] = v * mono[kMT.parent[m]];
      }
      double vx = 0.0, vy = 0.0, vz = 0.0;
      for (int s = 0; s < S; ++s) {
        const int ends = __builtin_amdgcn_readlane(end_lane, s);
        if (!(act && p < ends)) continue;
        const size_t roff = (size_t)(s * E + e) * (LDS ? BLKL : BLK);
        const T *bc = (const T *)__builtin_assume_aligned(bcoef + (size_t)s * NB, 16);
        if (s == dens) {  // local density: v = 2 rho'(q) W d, rho'(q) = sum_k B (-beta) e_k
          T cp0 = (T)0;
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            if (k < K) {
              const size_t o = roff + k * kCoefStride;
              bool use = true;
              if constexpr (SCREEN) {  // per-primitive screening: the primitive's own radius
                use = (float)q <= (float)(LDS ? tabl[o + 7] : tabg[o + 7]);
                if (__ballot(use) == 0) continue;
              }
              T ek = exp_scaled(LDS ? tabl[o] : tabg[o], qv);
              if constexpr (SCREEN) ek = use ? ek : (T)0;
              cp0 = fma_(LDS ? tabl[o + 1] : tabg[o + 1], (LDS ? tabl[o + 6] : tabg[o + 6]) * ek, cp0);
            }
          }
          const T A = cp0 * bc[0];
          const T A2 = A + A;
          vx += (double)(A2 * xv);
          vy += (double)(A2 * yv);
          vz += (double)(A2 * zv);
          continue;
        }
        // c_l = sum_k A e_k and c'_l = sum_k A (-gamma_k e_k)
        T cl[LMAX + 1], cp[LMAX + 1];
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) { cl[l] = (T)0; cp[l] = (T)0; }
        if constexpr (!SCREEN && !F64) {
          // as in the overlap kernel: zero rows past an element's own count,
          // the plan's largest count for every lane, row k+1 read ahead
          const T *row = (LDS ? tabl : tabg) + roff;
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
        } else
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          if (k < K) {
            const size_t o = roff + k * kCoefStride;
            bool use = true;
            if constexpr (SCREEN) {  // per-primitive screening: the primitive's own radius
              use = (float)q <= (float)(LDS ? tabl[o + 7] : tabg[o + 7]);
              if (__ballot(use) == 0) continue;
            }
            T ek = exp_scaled(LDS ? tabl[o] : tabg[o], qv);
            if constexpr (SCREEN) ek = use ? ek : (T)0;
            const T gk = (LDS ? tabl[o + 6] : tabg[o + 6]) * ek;
#pragma unroll
            for (int l = 0; l <= LMAX; ++l) {
              const T al = LDS ? tabl[o + 1 + l] : tabg[o + 1 + l];
              cl[l] = fma_(al, ek, cl[l]);
              cp[l] = fma_(al, gk, cp[l]);
            }
          }
        }
        T A = (T)0, Bx = (T)0, By = (T)0, Bz = (T)0;
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
          if (!((mask >> l) & 1)) continue;
          // P(d) = sum_m M_m d^m and its gradient from the same coefficients:
          // d/dx of x^a y^b z^c is a x^(a-1) y^b z^c (exponents are constants).
          // FP32: gradient terms summed per exponent value e, then combined as
          // sum e g_e (fewer instructions); FP64: each term scaled by its e.
          T Q = (T)0, gx[LMAX + 1], gy[LMAX + 1], gz[LMAX + 1];
#pragma unroll
          for (int e = 0; e <= LMAX; ++e) { gx[e] = (T)0; gy[e] = (T)0; gz[e] = (T)0; }
#pragma unroll
          for (int mm = 0; mm < ncomp(l); ++mm) {
            const int m = doff(l) + mm;
            const T Mv = bc[m];
            Q = fma_(Mv, mono[m], Q);
            const int a = kMT.ea[m], b = kMT.eb[m], c = kMT.ec[m];
            const int ia = F64 ? 1 : a, ib = F64 ? 1 : b, ic = F64 ? 1 : c;  // accumulator index
            if (a >= 1) gx[ia] = fma_(F64 && a > 1 ? (T)a * Mv : Mv, mono[doff(l - 1) + midx(l - 1, a - 1, b)], gx[ia]);
            if (b >= 1) gy[ib] = fma_(F64 && b > 1 ? (T)b * Mv : Mv, mono[doff(l - 1) + midx(l - 1, a, b - 1)], gy[ib]);
            if (c >= 1) gz[ic] = fma_(F64 && c > 1 ? (T)c * Mv : Mv, mono[doff(l - 1) + midx(l - 1, a, b)], gz[ic]);
          }
          A = fma_(cp[l], Q, A);
          if (l >= 1) {
            T sx = gx[1], sy = gy[1], sz = gz[1];
            if constexpr (!F64) {
#pragma unroll
              for (int e = 2; e <= l; ++e) {
                sx = fma_((T)e, gx[e], sx);
                sy = fma_((T)e, gy[e], sy);
                sz = fma_((T)e, gz[e], sz);
              }
            }
            Bx = fma_(cl[l], sx, Bx);
            By = fma_(cl[l], sy, By);
            Bz = fma_(cl[l], sz, Bz);
          }
        }
        const T A2 = A + A;
        vx += (double)fma_(A2, xv, Bx);
        vy += (double)fma_(A2, yv, By);
        vz += (double)fma_(A2, zv, Bz);
      }
      if (act) {
        T *dst = vbuf + (size_t)(base + p) * 4;
        dst[0] = (T)(vx * occj);
        dst[1] = (T)(vy * occj);
        dst[2] = (T)(vz * occj);
        dst[3] = (T)0;
      }
    }
    wave_lds_sync();  // every lane is done with this centre's coefficients
  }
}

// One wavefront per atom: grad_pos in list order and the atom's cell partial.
template <bool F64>
__global__ __launch_bounds__(256) void k_bwd_gather(BatchDev bt, NbrDev nb, const void *vbuf_, double *grad_pos,
                                                    double *cellpart) {
  using T = typename Real<F64>::T;
  const T *vbuf = (const T *)vbuf_;
  const int lane = lane_id();
  // each XCD takes one contiguous range of atoms: their mirror reads fall in
  // the same stretch of every partner bucket (sorted by atom), so in shared lines
  const int64_t a = xcd_contiguous(blockIdx.x, gridDim.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int64_t N = bt.n_atoms;
  if (a >= N) return;
  const int64_t k = nb.slot[a];  // the atom's list slot
  const int64_t base = nb.offsets[k];
  // a list that ends past the capacity was not written (overflowed no-sync
  // build); mirrors lie in the written lists, below the capacity
  const int64_t end = nb.offsets[k + 1] > nb.capacity ? base : nb.offsets[k + 1];
  const int64_t total = nb.capacity;
  const int ma0 = nb.wrap[3 * a], ma1 = nb.wrap[3 * a + 1], ma2 = nb.wrap[3 * a + 2];
  double g[3] = {0.0, 0.0, 0.0};
  double cp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t p = base + lane; p < end; p += kWave) {
    const int32_t j = nb.j[p];
    const int32_t w = nb.shift[p];
    const int32_t rv = nb.reverse[p];  // the mirror's pair index
    // a missing mirror is flagged by the neighbour build; never for a consistent list
    if (rv < 0 || (int64_t)rv >= total) continue;
    const T *va = vbuf + (size_t)p * 4;
    const T *vr = vbuf + (size_t)rv * 4;
    const double v0 = (double)va[0], v1 = (double)va[1], v2 = (double)va[2];
    g[0] += (double)vr[0] - v0;
    g[1] += (double)vr[1] - v1;
    g[2] += (double)vr[2] - v2;
    const double nt[3] = {(double)(shift_n(w, 0) - nb.wrap[3 * j] + ma0),
                          (double)(shift_n(w, 1) - nb.wrap[3 * j + 1] + ma1),
                          (double)(shift_n(w, 2) - nb.wrap[3 * j + 2] + ma2)};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      cp[3 * m] += nt[m] * v0;
      cp[3 * m + 1] += nt[m] * v1;
      cp[3 * m + 2] += nt[m] * v2;
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) g[k] = wave_sum(g[k]);
#pragma unroll
  for (int k = 0; k < 9; ++k) cp[k] = wave_sum(cp[k]);
  if (lane == 0) {
    grad_pos[a] = g[0];
    grad_pos[N + a] = g[1];
    grad_pos[2 * N + a] = g[2];
  }
  if (lane < 9) {
    double v = cp[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) v = lane == k ? cp[k] : v;
    cellpart[(size_t)a * 9 + lane] = v;
  }
}

// Reference points, atoms' side: one wavefront per atom; its pairs (those
// naming it as neighbour) in ascending pair order: dL/dR_a = sum v.
template <bool F64>
__global__ __launch_bounds__(256) void k_bwd_gather_atoms(BatchDev bt, const void *vbuf_, const uint32_t *order,
                                                          const int64_t *start, int64_t n_sorted, double *grad_pos) {
  using T = typename Real<F64>::T;
  const T *vbuf = (const T *)vbuf_;
  const int lane = lane_id();
  // one contiguous range of atoms per XCD, as in the atoms-only gather
  const int64_t a = xcd_contiguous(blockIdx.x, gridDim.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int64_t N = bt.n_atoms, NT = n_total(bt);
  if (a >= N) return;
  double g[3] = {0.0, 0.0, 0.0};
  int64_t t0 = start[a], t1 = start[a + 1];
  if (t0 < 0 || t1 > n_sorted || t0 > t1) t0 = t1 = 0;  // never for a consistent sort
  for (int64_t t = t0 + lane; t < t1; t += kWave) {
    const uint32_t p = order[t];
    if ((int64_t)p >= n_sorted) continue;
    const T *v = vbuf + (size_t)p * 4;
    g[0] += (double)v[0];
    g[1] += (double)v[1];
    g[2] += (double)v[2];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) g[k] = wave_sum(g[k]);
  if (lane == 0) {
    grad_pos[a] = g[0];
    grad_pos[NT + a] = g[1];
    grad_pos[2 * NT + a] = g[2];
  }
}

// Reference points, points' side: one wavefront per point, its own pairs in
// list order: dL/dP = -sum v, and the point's cell partial
// sum (n - m_j + m_P) (x) v.
template <bool F64>
__global__ __launch_bounds__(256) void k_bwd_point_centres(BatchDev bt, NbrDev nb, const void *vbuf_,
                                                           double *grad_pos, double *cellpart) {
  using T = typename Real<F64>::T;
  const T *vbuf = (const T *)vbuf_;
  const int lane = lane_id();
  const int64_t c = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (c >= n_centres(bt)) return;
  const int64_t NT = n_total(bt), gi = bt.n_atoms + c;
  const int64_t base = nb.offsets[c];
  const int64_t end = nb.offsets[c + 1] > nb.capacity ? base : nb.offsets[c + 1];
  const int mp0 = nb.wrap[3 * gi], mp1 = nb.wrap[3 * gi + 1], mp2 = nb.wrap[3 * gi + 2];
  double g[3] = {0.0, 0.0, 0.0};
  double cp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t p = base + lane; p < end; p += kWave) {
    const int32_t j = nb.j[p];
    const int32_t w = nb.shift[p];
    const T *va = vbuf + (size_t)p * 4;
    const double v0 = (double)va[0], v1 = (double)va[1], v2 = (double)va[2];
    g[0] -= v0;
    g[1] -= v1;
    g[2] -= v2;
    const double nt[3] = {(double)(shift_n(w, 0) - nb.wrap[3 * j] + mp0),
                          (double)(shift_n(w, 1) - nb.wrap[3 * j + 1] + mp1),
                          (double)(shift_n(w, 2) - nb.wrap[3 * j + 2] + mp2)};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      cp[3 * m] += nt[m] * v0;
      cp[3 * m + 1] += nt[m] * v1;
      cp[3 * m + 2] += nt[m] * v2;
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) g[k] = wave_sum(g[k]);
#pragma unroll
  for (int k = 0; k < 9; ++k) cp[k] = wave_sum(cp[k]);
  if (lane == 0) {
    grad_pos[gi] = g[0];
    grad_pos[NT + gi] = g[1];
    grad_pos[2 * NT + gi] = g[2];
  }
  if (lane < 9) {
    double v = cp[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) v = lane == k ? cp[k] : v;
    cellpart[(size_t)c * 9 + lane] = v;
  }
}

// One workgroup (four wavefronts) per structure: fixed-order sum of the
// per-centre cell partials (centres of structure s: [offs[s], offs[s+1])),
// strided over the 256 threads, then over the four wavefronts.
__global__ __launch_bounds__(256) void k_cell_reduce(BatchDev bt, const int64_t *offs, const double *cellpart,
                                                     double *grad_cell) {
  __shared__ double part[4][9];
  const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  const int64_t s = blockIdx.x;
  if (s >= bt.n_structs) return;  // uniform over the workgroup
  const int64_t a0 = offs[s], a1 = offs[s + 1];
  double cp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t a = a0 + tid; a < a1; a += blockDim.x)
#pragma unroll
    for (int k = 0; k < 9; ++k) cp[k] += cellpart[(size_t)a * 9 + k];
#pragma unroll
  for (int k = 0; k < 9; ++k) cp[k] = wave_sum(cp[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 9; ++k) part[w][k] = cp[k];
  __syncthreads();
  if (tid < 9) grad_cell[s * 9 + tid] = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
}

using PairsFn = void (*)(PlanDev, BatchDev, NbrDev, const double4 *, const int32_t *, const void *, void *, int,
                         int64_t, unsigned long long *, const void *);
// SCREEN: per-primitive screening (its own instantiation keeps the branch
// out of the loop of plans without it)
template <int L, bool F64, bool LDS, bool SCREEN> PairsFn pick_kb(int kb) {
  if (kb <= 4) return k_bwd_pairs<L, 4, F64, LDS, SCREEN>;
  if (kb <= 8) return k_bwd_pairs<L, 8, F64, LDS, SCREEN>;
  return k_bwd_pairs<L, 16, F64, LDS, SCREEN>;
}
template <bool F64, bool LDS, bool SCREEN> PairsFn pick_l(int lmax, int kb) {
  switch (lmax) {
    case 0: return pick_kb<0, F64, LDS, SCREEN>(kb);
    case 1: return pick_kb<1, F64, LDS, SCREEN>(kb);
    case 2: return pick_kb<2, F64, LDS, SCREEN>(kb);
    case 3: return pick_kb<3, F64, LDS, SCREEN>(kb);
    default: return pick_kb<4, F64, LDS, SCREEN>(kb);
  }
}
template <bool F64, bool LDS> PairsFn pick_pairs(int lmax, int kb, bool screen) {
  return screen ? pick_l<F64, LDS, true>(lmax, kb) : pick_l<F64, LDS, false>(lmax, kb);
}

}  // namespace

size_t bwd_coef_elems(const gmp_plan *p, int64_t n_atoms) {
  return (size_t)n_atoms * p->dev.S * coef_block(p->dev.lmax);
}

int persistent_blocks(const void *fn, size_t smem, int blocks_per_cu);

void transpose_by_neighbour(const NbrDev &nb, int64_t n_centres, int64_t n_atoms, int64_t n, uint32_t *key_a,
                            uint32_t *key_b, uint32_t *val_a, uint32_t *val_b, int32_t *hist, int64_t *off,
                            int64_t *scan_aux, int64_t *start, uint32_t **vals_out, hipStream_t s);

// Per-centre adjoint coefficients (grad_features null: unit upstream
// gradient, i.e. the coefficients of dF/dd of every feature), and the packed
// positions and structures of all indices.
void launch_bwd_coef(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const double *components,
                     const void *grad_features, const WsLayout &L, hipStream_t s) {
  const int64_t blocks_all = (n_total(bt) + 3) / 4;
  if (blocks_all == 0) return;
  const size_t sm = (size_t)p->dev.S * nmono(p->dev.lmax);
  size_t smem = sizeof(double) * 4 * ((size_t)p->dev.nf + sm + p->dev.ncomp_total) +
                sizeof(int32_t) * ((size_t)p->dev.nf + 2 * sm);  // + the decode tables
  using CoefFn = void (*)(PlanDev, BatchDev, NbrDev, const double *, const void *, void *, double4 *, int32_t *,
                          unsigned long long *);
  static const CoefFn fns[2][kMaxL + 1] = {
      {k_bwd_coef<0, false>, k_bwd_coef<1, false>, k_bwd_coef<2, false>, k_bwd_coef<3, false>, k_bwd_coef<4, false>},
      {k_bwd_coef<0, true>, k_bwd_coef<1, true>, k_bwd_coef<2, true>, k_bwd_coef<3, true>, k_bwd_coef<4, true>}};
  const int lm = p->dev.lmax < 0 ? 0 : (p->dev.lmax > kMaxL ? kMaxL : p->dev.lmax);
  GMP_LAUNCH("adj_coef", fns[p->prec == GMP_FP64 ? 1 : 0][lm], dim3((unsigned)blocks_all), dim3(256), smem, s,
             p->dev, bt, nb, components, grad_features, L.bcoef, L.rw4, L.astruct, L.counter);
}

void launch_backward(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const double *components,
                     const void *grad_features, double *grad_pos, double *grad_cell, const WsLayout &L, int C,
                     int64_t pairs_bound, hipStream_t s) {
  const int64_t N = n_centres(bt), NT = n_total(bt);
  if (N == 0) return;
  void *bcoef = L.bcoef, *vbuf = L.vbuf;
  double *cellpart = L.cellpart;
  unsigned long long *counter = L.counter;
  double4 *rw4 = L.rw4;
  int32_t *astruct = L.astruct;
  const bool f64 = p->prec == GMP_FP64;
  const int64_t blocks = (N + 3) / 4;
  (void)NT;
  launch_bwd_coef(p, bt, nb, components, grad_features, L, s);
  const int64_t n_items = N * (int64_t)C;
  const size_t tab_bytes = (size_t)p->dev.S * p->dev.E * p->dev.kb * kCoefStride * (f64 ? 8 : 4);
  const bool use_lds = tab_bytes <= 48 * 1024;
  const size_t tsm = (use_lds ? tab_bytes + (size_t)p->dev.S * p->dev.E * 16 : 0) +  // table with its gaps
                     4 * (size_t)p->dev.S * coef_block(p->dev.lmax) * (f64 ? 8 : 4);
  const void *tab = f64 ? (const void *)p->dev.coef64 : (const void *)p->dev.coef32;
  const bool scr = p->dev.screen != 0;
  PairsFn fn = f64 ? (use_lds ? pick_pairs<true, true>(p->dev.lmax, p->dev.kb, scr)
                              : pick_pairs<true, false>(p->dev.lmax, p->dev.kb, scr))
                   : (use_lds ? pick_pairs<false, true>(p->dev.lmax, p->dev.kb, scr)
                              : pick_pairs<false, false>(p->dev.lmax, p->dev.kb, scr));
  int64_t pb = persistent_blocks((const void *)fn, tsm, p->tuning.blocks_per_cu);
  if (pb > (n_items + 3) / 4) pb = (n_items + 3) / 4;
  if (pb < 1) pb = 1;
  GMP_LAUNCH("adj_pairs", fn, dim3((unsigned)pb), dim3(256), tsm, s, p->dev, bt, nb, (const double4 *)rw4,
             (const int32_t *)astruct, bcoef, vbuf, C, n_items, counter, tab);
  if (!point_mode(bt)) {
    if (f64)
      GMP_LAUNCH("adj_gather", k_bwd_gather<true>, dim3((unsigned)blocks), dim3(256), 0, s, bt, nb, vbuf, grad_pos,
                 cellpart);
    else
      GMP_LAUNCH("adj_gather", k_bwd_gather<false>, dim3((unsigned)blocks), dim3(256), 0, s, bt, nb, vbuf, grad_pos,
                 cellpart);
  } else {
    // reference points: atoms gather the pairs that name them, in pair order
    uint32_t *order = nullptr;
    transpose_by_neighbour(nb, N, bt.n_atoms, pairs_bound, L.tr_key_in, L.tr_key_out, L.tr_val_in, L.tr_val_out,
                           L.tr_hist, L.tr_off, L.scan_aux, L.tr_start, &order, s);
    const int64_t ab = (bt.n_atoms + 3) / 4;
    if (ab > 0) {
      if (f64)
        GMP_LAUNCH("adj_gather", k_bwd_gather_atoms<true>, dim3((unsigned)ab), dim3(256), 0, s, bt, vbuf, order,
                   L.tr_start, pairs_bound, grad_pos);
      else
        GMP_LAUNCH("adj_gather", k_bwd_gather_atoms<false>, dim3((unsigned)ab), dim3(256), 0, s, bt, vbuf, order,
                   L.tr_start, pairs_bound, grad_pos);
    }
    if (f64)
      GMP_LAUNCH("adj_points", k_bwd_point_centres<true>, dim3((unsigned)blocks), dim3(256), 0, s, bt, nb, vbuf,
                 grad_pos, cellpart);
    else
      GMP_LAUNCH("adj_points", k_bwd_point_centres<false>, dim3((unsigned)blocks), dim3(256), 0, s, bt, nb, vbuf,
                 grad_pos, cellpart);
  }
  if (grad_cell && bt.n_structs > 0) {
    GMP_LAUNCH("adj_cell", k_cell_reduce, dim3((unsigned)bt.n_structs), dim3(256), 0, s, bt,
               point_mode(bt) ? bt.point_offsets : bt.atom_offsets, cellpart, grad_cell);
  }
}

}  // namespace gmp
