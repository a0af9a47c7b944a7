// Neighbour build: lattice wrap, cell-list binning, per-centre count, fill
// and canonical sort, reverse-pair index.
//
// The cutoff is inferred from the overlap threshold (the paper's "Examples"
// section): a pair (j, n) belongs to centre i when its squared distance q is
// at most the largest rc(sigma)^2.  Image shifts n range over every lattice
// translation on periodic axes, so atoms (and the centre itself) appear as
// often as they fit inside the cutoff sphere.
//
// Floating point: reciprocal rows, fractional coordinates, wrap, image
// shifts, displacements and q are FP64 in a fixed operation order with no
// contraction (the file is built with -ffp-contract=off), so every kernel that
// recomputes q gets the same bits and (j,i,-n) has exactly the q of (i,j,n).
//
// Cell list: fractional space of each structure is cut into nb_k bins per
// periodic axis (edge ~ rc_max / bin_divisor); a centre visits the "virtual"
// bins V_k in [floor((f_k - reach_k) nb_k), floor((f_k + reach_k) nb_k)],
// each of which is real bin V mod nb with image shift floor(V / nb).  Atoms
// are stored bin-sorted in SoA arrays so a bin is read with coalesced loads.
#include "gmp_internal.h"

namespace gmp {
namespace {

__device__ inline void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double *a, const double *b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

__device__ inline int floordiv(int a, int b) { int q = a / b; return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q; }
__device__ inline int pmod(int a, int b) { int r = a % b; return r < 0 ? r + b : r; }

__global__ void k_struct_setup(BatchDev bt, StructInfo *info, double rcmax, int bin_div, uint32_t *status) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= bt.n_structs) return;
  StructInfo I;
  const int pbc = bt.pbc[s] & 7;
  const int64_t n_s = bt.atom_offsets[s + 1] - bt.atom_offsets[s];
  I.pbc = pbc;
  I.bin_base = bt.atom_offsets[s] + s;
  for (int k = 0; k < 9; ++k) I.b[k] = 0.0;
  for (int k = 0; k < 3; ++k) { I.nb[k] = 1; I.reach[k] = 0.0; }
  I.lam_lo = 0.0;
  if (pbc) {
    const double *a = bt.cell + 9 * (int64_t)s;
    double c23[3], c31[3], c12[3];
    cross3(a + 3, a + 6, c23);
    cross3(a + 6, a, c31);
    cross3(a, a + 3, c12);
    double V = dot3(a, c23);
    bool ok = isfinite(V) && V != 0.0;
    for (int k = 0; k < 9; ++k) ok = ok && isfinite(a[k]);
    if (!ok) {
      atomicOr(status, ST_CELL);
    } else {
      for (int k = 0; k < 3; ++k) { I.b[k] = c23[k] / V; I.b[3 + k] = c31[k] / V; I.b[6 + k] = c12[k] / V; }
      const double ell = rcmax / (double)bin_div;
      for (int k = 0; k < 3; ++k) {
        if (!(pbc & (1 << k))) continue;
        double inv_h = sqrt(dot3(I.b + 3 * k, I.b + 3 * k));
        double h = 1.0 / inv_h;
        double nbk = ell > 0.0 ? floor(h / ell) : 1.0;
        if (!(nbk >= 1.0)) nbk = 1.0;
        if (nbk > 1024.0) nbk = 1024.0;
        I.nb[k] = (int)nbk;
        I.reach[k] = rcmax * inv_h * (1.0 + 1e-12) + 1e-12;
        // image shifts must fit a signed byte
        if (I.reach[k] + 2.0 > 126.0) atomicOr(status, ST_SHIFT_RANGE);
      }
      // smallest eigenvalue of the metric G = A A^T (rows of A are the lattice vectors), for a lower
      // bound |n.A|^2 >= lambda_min |n|^2 that lets the cell list skip bin images outside the cutoff
      {
        double Gm[3][3];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) Gm[r][c] = dot3(a + 3 * r, a + 3 * c);
        const double p1 = Gm[0][1] * Gm[0][1] + Gm[0][2] * Gm[0][2] + Gm[1][2] * Gm[1][2];
        const double qq = (Gm[0][0] + Gm[1][1] + Gm[2][2]) / 3.0;
        const double d0 = Gm[0][0] - qq, d1 = Gm[1][1] - qq, d2 = Gm[2][2] - qq;
        const double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1;
        double lmin;
        if (p2 <= 0.0) {
          lmin = qq;
        } else {
          const double pp = sqrt(p2 / 6.0);
          const double b00 = d0 / pp, b11 = d1 / pp, b22 = d2 / pp;
          const double b01 = Gm[0][1] / pp, b02 = Gm[0][2] / pp, b12 = Gm[1][2] / pp;
          double r = 0.5 * (b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02));
          r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
          const double phi = acos(r) / 3.0;
          lmin = qq + 2.0 * pp * cos(phi + 2.0943951023931957);
        }
        I.lam_lo = (isfinite(lmin) && lmin > 0.0) ? 0.99 * lmin : 0.0;
      }
      // never more bins than atoms (bin slots per structure are n_s + 1)
      int64_t cap = n_s > 1 ? n_s : 1;
      while ((int64_t)I.nb[0] * I.nb[1] * I.nb[2] > cap) {
        int kk = 0;
        if (I.nb[1] > I.nb[kk]) kk = 1;
        if (I.nb[2] > I.nb[kk]) kk = 2;
        I.nb[kk] = I.nb[kk] > 1 ? (I.nb[kk] + 1) / 2 : 1;
      }
    }
  }
  for (int k = 0; k < 3; ++k) I.inv_nb[k] = 1.0 / (double)I.nb[k];
  info[s] = I;
}

// One thread per index g: atoms (wrapped, binned) and reference points
// (wrapped only; they are centres, never neighbours).  rw, wrap and fw are
// over the n_total indices.
__global__ void k_wrap(BatchDev bt, const StructInfo *info, NbrDev nb, double *fw, int32_t *bin_of,
                       int32_t *bin_count, int32_t *astruct, int n_elements, uint32_t *status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = n_total(bt);
  if (i >= N) return;
  const bool atom = i < bt.n_atoms;
  if (atom) {
    const int sp = bt.species[i];
    if (sp < 0 || sp >= n_elements) atomicOr(status, ST_SPECIES);
  }
  const int s = struct_of_index(bt, i);
  astruct[i] = s;
  const StructInfo &I = info[s];
  const int64_t k = atom ? i : i - bt.n_atoms;
  const double *X = atom ? bt.x : bt.px, *Y = atom ? bt.y : bt.py, *Z = atom ? bt.z : bt.pz;
  const double R[3] = {X[k], Y[k], Z[k]};
  if (!(isfinite(R[0]) && isfinite(R[1]) && isfinite(R[2]))) atomicOr(status, ST_NONFINITE);
  if (atom && bt.occ && !isfinite(bt.occ[i])) atomicOr(status, ST_NONFINITE);
  int m[3] = {0, 0, 0};
  int b[3] = {0, 0, 0};
  double f3[3] = {0.0, 0.0, 0.0};
  double rwv[3] = {R[0], R[1], R[2]};
  if (I.pbc) {
    const double *a = bt.cell + 9 * (int64_t)s;
    for (int k = 0; k < 3; ++k) {
      if (!(I.pbc & (1 << k))) continue;
      double f = dot3(R, I.b + 3 * k);
      if (!(fabs(f) < 1.0e9)) { atomicOr(status, ST_NONFINITE); f = 0.0; }
      double fl = floor(f);
      m[k] = (int)fl;
      double w = f - fl;  // exact, in [0, 1)
      f3[k] = w;
      int bk = (int)(w * (double)I.nb[k]);
      if (bk > I.nb[k] - 1) bk = I.nb[k] - 1;
      if (bk < 0) bk = 0;
      b[k] = bk;
    }
    for (int c = 0; c < 3; ++c) {
      double t = (double)m[0] * a[c] + (double)m[1] * a[3 + c];
      t = t + (double)m[2] * a[6 + c];
      rwv[c] = R[c] - t;
    }
  }
  nb.rw[i] = rwv[0];
  nb.rw[N + i] = rwv[1];
  nb.rw[2 * N + i] = rwv[2];
  nb.wrap[3 * i] = m[0];
  nb.wrap[3 * i + 1] = m[1];
  nb.wrap[3 * i + 2] = m[2];
  fw[i] = f3[0];
  fw[N + i] = f3[1];
  fw[2 * N + i] = f3[2];
  if (!atom) {  // reference points keep their own list order
    nb.order[k] = (int32_t)k;
    nb.slot[k] = (int32_t)k;
    return;
  }
  int64_t bin = I.bin_base + ((int64_t)b[0] * I.nb[1] + b[1]) * I.nb[2] + b[2];
  bin_of[i] = (int32_t)bin;
  atomicAdd(&bin_count[bin], 1);
}

// Atoms into their bins, in arrival order (the slot within a bin comes
// from an atomic counter); k_bin_order then orders every bin by atom index.
__global__ void k_scatter(BatchDev bt, const int32_t *bin_of, const int64_t *bin_start, int32_t *bin_fill,
                          int32_t *sid_tmp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bt.n_atoms) return;
  int32_t b = bin_of[i];
  int64_t p = bin_start[b] + atomicAdd(&bin_fill[b], 1);
  sid_tmp[p] = (int32_t)i;
}

// Deterministic cell-list order: the atom at arrival slot p of bin b goes to
// position bin_start[b] + (number of atoms of b with a smaller index); the
// bin-sorted SoA copies (wrapped positions, atom index, species) are written
// there, and with atoms as centres the list-slot order follows it.  One
// thread per arrival slot; the threads of one bin read the same members.
__global__ void k_bin_order(BatchDev bt, NbrDev nb, const int32_t *bin_of, const int64_t *bin_start,
                            const int32_t *sid_tmp, double *sx, double *sy, double *sz, int32_t *sid, int32_t *ssp,
                            int n_elements) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= bt.n_atoms) return;
  const int64_t N = n_total(bt);  // stride of rw
  const int32_t i = sid_tmp[p];
  const int32_t b = bin_of[i];
  const int64_t lo = bin_start[b], hi = bin_start[b + 1];
  int64_t r = 0;
  for (int64_t q = lo; q < hi; ++q) r += sid_tmp[q] < i ? 1 : 0;
  const int64_t k = lo + r;
  sx[k] = nb.rw[i];
  sy[k] = nb.rw[N + i];
  sz[k] = nb.rw[2 * N + i];
  sid[k] = i;
  const int sp = bt.species[i];
  ssp[k] = sp < 0 ? 0 : (sp >= n_elements ? n_elements - 1 : sp);  // out-of-range species are flagged in k_wrap
  if (!point_mode(bt)) {
    nb.order[k] = i;
    nb.slot[i] = (int32_t)k;
  }
}

// Range of virtual bins along axis k for a centre at fractional f.
__device__ inline void vrange(const StructInfo &I, int k, double f, int &lo, int &hi) {
  if (!(I.pbc & (1 << k))) { lo = hi = 0; return; }
  double nbk = (double)I.nb[k];
  lo = (int)floor((f - I.reach[k]) * nbk - 1e-6);
  hi = (int)floor((f + I.reach[k]) * nbk + 1e-6);
}

struct Cand {
  const StructInfo *I;
  const double *cell;
  double f[3];
  int lo[3], hi[3], nv[3];
  double inv_nv[3];
  int total;
};

__device__ inline void cand_setup(Cand &C, const StructInfo *info, const BatchDev &bt, int s,
                                  const double *fw, int64_t i) {
  const int64_t N = n_total(bt);  // stride of fw
  C.I = info + s;
  C.cell = bt.cell + 9 * (int64_t)s;
  C.f[0] = fw[i]; C.f[1] = fw[N + i]; C.f[2] = fw[2 * N + i];
  C.total = 1;
  for (int k = 0; k < 3; ++k) {
    vrange(*C.I, k, C.f[k], C.lo[k], C.hi[k]);
    C.nv[k] = C.hi[k] - C.lo[k] + 1;
    C.inv_nv[k] = 1.0 / (double)C.nv[k];
    C.total *= C.nv[k];
  }
}

// Virtual bin v (linear index) -> real bin slot and image shift; returns -1
// when the whole bin image lies outside the cutoff sphere (fractional gaps
// g_k to the centre satisfy lam_lo * |g|^2 > rc_max^2).
__device__ inline int64_t cand_bin(const Cand &C, int v, int n[3], double rcmax2) {
  // small non-negative / signed integer quotients through FP64 reciprocals:
  // (x + 1/2) / d keeps its fractional part at least 1/(2d) from an integer,
  // far above the rounding of the product
  int r[3];
  int t = v;
  int q = (int)floor(((double)t + 0.5) * C.inv_nv[2]);
  r[2] = t - q * C.nv[2]; t = q;
  q = (int)floor(((double)t + 0.5) * C.inv_nv[1]);
  r[1] = t - q * C.nv[1]; t = q;
  r[0] = t;
  int b[3];
  double g2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    const int V = C.lo[k] + r[k];
    const int nbk = C.I->nb[k];
    n[k] = (int)floor(((double)V + 0.5) * C.I->inv_nb[k]);
    b[k] = V - n[k] * nbk;
    if (C.I->pbc & (1 << k)) {
      // bin-image bounds in fractional coordinates; a product with the
      // reciprocal is within 2 ulp of the quotient, far inside the 1e-9
      // slack that keeps the culling conservative
      const double x0 = (double)V * C.I->inv_nb[k], x1 = (double)(V + 1) * C.I->inv_nb[k];
      double g = x0 - C.f[k];
      const double g1 = C.f[k] - x1;
      g = g > g1 ? g : g1;
      g -= 1e-9;
      if (g > 0.0) g2 += g * g;
    }
  }
  if (C.I->lam_lo * g2 > rcmax2) return -1;
  return C.I->bin_base + ((int64_t)b[0] * C.I->nb[1] + b[1]) * C.I->nb[2] + b[2];
}

// Per-wavefront LDS scratch of the candidate enumeration.
struct CandLds {
  int delta[kWave];  // bin start minus the bin's first flattened position
  int npk[kWave];
  double sh[3][kWave];
};

// Calls f(t, n, shx, shy, shz) for every candidate atom t (index into the
// bin-sorted arrays) of every bin image that is not culled.  Bin images are
// taken 64 at a time (one per lane); their atoms are then flattened so that
// consecutive lanes read consecutive atoms.  With several wavefronts on one
// centre (wave w of nw), each wavefront takes every nw-th block of 64
// flattened candidates of every chunk.  The bin of flattened position c is
// the last lane whose exclusive prefix pre is <= c: the prefixes grow with the
// lane, so for a block starting at c0 it is the count of lanes with pre <= c0
// less one, moved on past every non-empty bin that starts inside the block
// (one or two for bins of tens of atoms).
template <typename F>
__device__ inline void for_each_candidate(const Cand &C, const int64_t *bin_start, double rcmax2, int w, int nw,
                                          CandLds &L, F &&f) {
  const int lane = lane_id();
  for (int v0 = 0; v0 < C.total; v0 += kWave) {
    const int v = v0 + lane;
    int cnt = 0, start = 0, npk = 0;
    double shx = 0.0, shy = 0.0, shz = 0.0;
    if (v < C.total) {
      int n[3];
      const int64_t bin = cand_bin(C, v, n, rcmax2);
      if (bin >= 0) {
        start = (int)bin_start[bin];
        cnt = (int)(bin_start[bin + 1] - start);
        npk = (n[0] & 0xff) | ((n[1] & 0xff) << 8) | ((n[2] & 0xff) << 16);
        if (C.I->pbc) image_shift(C.cell, n[0], n[1], n[2], shx, shy, shz);
      }
    }
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    const int tot = __shfl(incl, kWave - 1, kWave);
    const int pre = incl - cnt;  // lanes past the last bin image: pre = tot
    L.delta[lane] = start - pre;
    L.npk[lane] = npk;
    L.sh[0][lane] = shx;
    L.sh[1][lane] = shy;
    L.sh[2][lane] = shz;
    wave_lds_sync();
    for (int c0 = w * kWave; c0 < tot; c0 += nw * kWave) {
      const int c = c0 + lane;
      int own = __popcll(__ballot(pre <= c0)) - 1;
      for (uint64_t starts = __ballot(cnt > 0 && pre > c0 && pre - c0 < kWave); starts; starts &= starts - 1) {
        const int l = __builtin_ctzll(starts);
        if (c >= __builtin_amdgcn_readlane(pre, l)) own = l;
      }
      if (c < tot) {
        const int t = c + L.delta[own];
        const int pk = L.npk[own];
        const int n[3] = {(int)(int8_t)(pk & 0xff), (int)(int8_t)((pk >> 8) & 0xff), (int)(int8_t)((pk >> 16) & 0xff)};
        f(t, n, L.sh[0][own], L.sh[1][own], L.sh[2][own]);
      }
    }
    wave_lds_sync();
  }
}

// Shell of a squared distance q: the number of cutoffs rc2[s] < q.  The
// cutoffs sit in registers, padded to SM (8, 12 or 16) with +infinity, so
// the count is a fixed run of compares against uniform operands.
template <int SM>
struct Shells {
  double r[SM];
  __device__ explicit Shells(const PlanDev &P) {
#pragma unroll
    for (int s = 0; s < SM; ++s) r[s] = s < P.S ? P.rc2[s] : __builtin_huge_val();
  }
  __device__ int of(double q) const {
    int sh = 0;
#pragma unroll
    for (int s = 0; s < SM; ++s) sh += r[s] < q ? 1 : 0;
    return sh;
  }
};

// One workgroup per centre (centres in cell-list order): count neighbours
// per (shell, species) bucket; the wavefronts share the centre's candidates.
template <int SM>
__global__ __launch_bounds__(256) void k_count(PlanDev P, BatchDev bt, NbrDev nb, const StructInfo *info,
                                               const double *fw, const int64_t *bin_start,
                                               const double *sx, const double *sy, const double *sz,
                                               const int32_t *sid, const int32_t *ssp, const int32_t *astruct,
                                               int32_t *cnt, int64_t *ptotal, uint32_t *status) {
  extern __shared__ int32_t lds_cnt[];
  __shared__ CandLds lds_cand[4];
  __shared__ int64_t lds_tot[4];
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave, lane = lane_id();
  const int nbk = P.E * P.S;
  int32_t *c = lds_cnt;
  const int64_t N = n_total(bt);  // stride of rw
  // list slot k (atoms: cell-list order, each XCD one contiguous range), centre i, index g
  const int64_t k = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t i = point_mode(bt) ? k : sid[k];
  const int64_t g = centre_base(bt) + i;
  for (int t = threadIdx.x; t < nbk; t += blockDim.x) c[t] = 0;
  __syncthreads();
  const int s = astruct[g];
  Cand C;
  cand_setup(C, info, bt, s, fw, g);
  const Shells<SM> shells(P);
  const double rix = nb.rw[g], riy = nb.rw[N + g], riz = nb.rw[2 * N + g];
  for_each_candidate(C, bin_start, P.rcmax2, w, nw, lds_cand[w],
                     [&](int t, const int *n, double shx, double shy, double shz) {
                       const double dx = (sx[t] - rix) + shx;
                       const double dy = (sy[t] - riy) + shy;
                       const double dz = (sz[t] - riz) + shz;
                       const double q = (dx * dx + dy * dy) + dz * dz;
                       if (q <= P.rcmax2) atomicAdd(&c[shells.of(q) * P.E + ssp[t]], 1);
                     });
  __syncthreads();
  int64_t tot = 0;
  for (int t = threadIdx.x; t < nbk; t += blockDim.x) {
    cnt[k * nbk + t] = c[t];
    tot += c[t];
  }
  for (int o = 32; o >= 1; o >>= 1) tot += __shfl_xor(tot, o, kWave);
  if (lane == 0) lds_tot[w] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t all = 0;
    for (int u = 0; u < nw; ++u) all += lds_tot[u];
    ptotal[k] = all;
  }
}

// Longest list (status word 4) and longest (shell, species) bucket (word 5)
// of the counted lists, for the synchronous build's sort sizes: a grid-stride
// maximum with one atomic per workgroup and word.
__global__ __launch_bounds__(256) void k_list_stats(const int64_t *ptotal, int64_t n_centres, const int32_t *cnt,
                                                    int64_t n_cnt, uint32_t *status) {
  __shared__ int64_t lds_m[2][4];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t lmax = 0, bmax = 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_centres; t += stride)
    lmax = ptotal[t] > lmax ? ptotal[t] : lmax;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_cnt; t += stride)
    bmax = cnt[t] > bmax ? cnt[t] : bmax;
  for (int o = 32; o >= 1; o >>= 1) {
    const int64_t a = __shfl_xor(lmax, o, kWave), b = __shfl_xor(bmax, o, kWave);
    lmax = a > lmax ? a : lmax;
    bmax = b > bmax ? b : bmax;
  }
  if (lane == 0) { lds_m[0][w] = lmax; lds_m[1][w] = bmax; }
  __syncthreads();
  if (threadIdx.x < 2) {
    int64_t m = 0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) m = lds_m[threadIdx.x][k] > m ? lds_m[threadIdx.x][k] : m;
    if (m > 0) atomicMax(status + 4 + threadIdx.x, (uint32_t)(m > 0x7fffffff ? 0x7fffffff : m));
  }
}

__device__ inline void cmpswap(uint64_t *a, int i, int l) {
  uint64_t x = a[i], y = a[l];
  if (x > y) { a[i] = y; a[l] = x; }
}

// Four elements e0 < e1 < e2 < e3 through two comparator stages in
// registers: mirror = true compares (e0, e3), (e1, e2) and then (e0, e1),
// (e2, e3); otherwise (e0, e2), (e1, e3) and then (e0, e1), (e2, e3).
// Positions >= n read as +infinity and are not written.
__device__ inline void group4(uint64_t *a, int n, int e0, int e1, int e2, int e3, bool mirror) {
  uint64_t x0 = e0 < n ? a[e0] : ~0ull, x1 = e1 < n ? a[e1] : ~0ull;
  uint64_t x2 = e2 < n ? a[e2] : ~0ull, x3 = e3 < n ? a[e3] : ~0ull;
  uint64_t u;
  if (mirror) {
    if (x0 > x3) { u = x0; x0 = x3; x3 = u; }
    if (x1 > x2) { u = x1; x1 = x2; x2 = u; }
  } else {
    if (x0 > x2) { u = x0; x0 = x2; x2 = u; }
    if (x1 > x3) { u = x1; x1 = x3; x3 = u; }
  }
  if (x0 > x1) { u = x0; x0 = x1; x1 = u; }
  if (x2 > x3) { u = x2; x2 = x3; x3 = u; }
  if (e0 < n) a[e0] = x0;
  if (e1 < n) a[e1] = x1;
  if (e2 < n) a[e2] = x2;
  if (e3 < n) a[e3] = x3;
}

// Sort a[0..n) of distinct keys ascending by one wavefront.  Up to 128
// keys: each lane holds one or two keys, counts the keys below each in one
// pass of broadcast LDS reads and stores them at those ranks (one pass
// instead of the 16 synchronised passes of a 128-key network; measured
// faster up to 128 keys, slower at 256).  Longer: bitonic network whose
// first merge stage compares mirror pairs, so every comparator is ascending
// and indices >= n act as +infinity without being touched.
__device__ void wave_sort(uint64_t *a, int n) {
  const int lane = lane_id();
  if (n <= 1) return;
  if (n <= kWave) {
    const uint64_t k = lane < n ? a[lane] : 0ull;
    int rank = 0;
    for (int m = 0; m < n; ++m) rank += a[m] < k ? 1 : 0;
    wave_lds_sync();
    if (lane < n) a[rank] = k;
    wave_lds_sync();
    return;
  }
  if (n <= 2 * kWave) {
    // keys are below ~0 (the top bits hold a shell < 16), so ~0 pads
    const uint64_t k0 = a[lane], k1 = lane + kWave < n ? a[lane + kWave] : ~0ull;
    int r0 = 0, r1 = 0;
    for (int m = 0; m < n; ++m) {
      const uint64_t x = a[m];
      r0 += x < k0 ? 1 : 0;
      r1 += x < k1 ? 1 : 0;
    }
    wave_lds_sync();
    a[r0] = k0;
    if (lane + kWave < n) a[r1] = k1;
    wave_lds_sync();
    return;
  }
  int lp2 = 1;
  while ((1 << lp2) < n) ++lp2;
  const int half = 1 << (lp2 - 1);
  // Comparators in groups of four that are closed under two consecutive
  // stages: each pass reads a lane's group once, compares in registers and
  // writes it once (indices >= n stay +infinity, never written); block
  // sizes are powers of two, so block and offset are shifts and masks.
  const int quarter = half >> 1;
  for (int lk = 1; lk <= lp2; ++lk) {
    const int k = 1 << lk;
    int lj;
    if (lk == 1) {  // blocks of two: the mirror stage alone
      for (int t = lane; t < half; t += kWave) {
        const int i = t << 1;
        if (i + 1 < n) cmpswap(a, i, i + 1);
      }
      wave_lds_sync();
      lj = -1;
    } else {  // mirror stage and the stage of distance k/4
      const int lq = lk - 2, Q = 1 << lq;
      for (int t = lane; t < quarter; t += kWave) {
        const int base = (t >> lq) << lk, off = t & (Q - 1);
        group4(a, n, base + off, base + off + Q, base + k - 1 - off - Q, base + k - 1 - off, true);
      }
      wave_lds_sync();
      lj = lk - 3;
    }
    for (; lj >= 1; lj -= 2) {  // the stages of distance j and j/2
      const int J = 1 << lj, H = J >> 1;
      for (int t = lane; t < quarter; t += kWave) {
        const int b = ((t >> (lj - 1)) << (lj + 1)) + (t & (H - 1));
        group4(a, n, b, b + H, b + J, b + J + H, false);
      }
      wave_lds_sync();
    }
    if (lj == 0) {  // a last stage of distance 1
      for (int t = lane; t < half; t += kWave) {
        const int i = t << 1;
        if (i + 1 < n) cmpswap(a, i, i + 1);
      }
      wave_lds_sync();
    }
  }
}

// Sort key of a pair inside one bucket: (j, n) with the bucket's shell in the
// top bits (constant within a bucket, so the order is that of (j, n)); the
// reverse-index search reads the shell from it.
__device__ inline uint64_t make_key(int64_t j, int n1, int n2, int n3, int shell = 0) {
  return ((uint64_t)shell << 60) | ((uint64_t)j << 24) | ((uint64_t)(n1 + 128) << 16) |
         ((uint64_t)(n2 + 128) << 8) | (uint64_t)(n3 + 128);
}

// Fill of one centre's list by one workgroup: its buckets (shell h,
// species e), in bucket order h * E + e, in LDS; every bucket sorted by
// (j, n); j / shift, the bucket starts and the sigma-prefix ends written.
// The in-LDS sort holds lds_keys entries.  RANGED = false (the short-list
// kernel) takes lists that fit in one candidate pass and hands longer ones
// to the long-list queue; RANGED = true fills range by range of consecutive
// buckets that fit, enumerating the candidates once per range; a single
// bucket longer than the sort leaves placeholders and is reported.
template <bool RANGED, int SM>
__device__ inline void fill_centre(const PlanDev &P, const BatchDev &bt, const NbrDev &nb, const StructInfo *info,
                                   const double *fw, const int64_t *bin_start, const double *sx, const double *sy,
                                   const double *sz, const int32_t *sid, const int32_t *ssp, const int32_t *astruct,
                                   const int32_t *cnt, int lds_keys, uint64_t *pair_key, int32_t *pair_centre,
                                   uint64_t *pair_sum, int64_t *abs_bstart, uint32_t *status, int32_t *long_q,
                                   int64_t k, int64_t i, uint64_t *keys, CandLds *lds_cand, int32_t &lds_bmax) {
  const int nbk = P.E * P.S;
  int32_t *bstart = (int32_t *)(keys + lds_keys);  // [nbk+1]
  int32_t *cursor = bstart + nbk + 1;              // [nbk]
  const int64_t g = centre_base(bt) + i;
  const int64_t N = n_total(bt);  // stride of rw
  const int tid = threadIdx.x, w = tid / kWave, nw = blockDim.x / kWave, lane = lane_id();
  const int64_t base = nb.offsets[k];
  const int64_t total = nb.offsets[k + 1] - base;
  const bool overflow = nb.offsets[k + 1] > nb.capacity;
  if (w == 0) {  // bucket starts: exclusive scan of the centre's bucket counts
    int32_t carry = 0, vmax = 0;
    for (int b0 = 0; b0 < nbk; b0 += kWave) {
      const int b = b0 + lane;
      const int32_t v = b < nbk ? cnt[k * nbk + b] : 0;
      vmax = v > vmax ? v : vmax;
      int32_t incl = v;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
      }
      if (b < nbk) bstart[b] = carry + incl - v;
      carry += __shfl(incl, kWave - 1, kWave);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const int32_t y = __shfl_xor(vmax, o, kWave);
      vmax = y > vmax ? y : vmax;
    }
    if (lane == 0) {
      bstart[nbk] = carry;
      lds_bmax = vmax;
      if (overflow) atomicOr(status, ST_OVERFLOW);
      if (RANGED && vmax > lds_keys) atomicOr(status, ST_SORT_SIZE);
      if ((int64_t)carry != total) atomicOr(status, ST_INTERNAL);
      // a list the short-list kernel cannot sort in one pass goes to the queue
      if (!RANGED && !overflow && total > lds_keys) long_q[atomicAdd(status + 6, 1u)] = (int32_t)k;
    }
  }
  __syncthreads();
  if (!RANGED && !overflow && total > lds_keys) return;  // the long-list kernel writes this centre
  for (int b = tid; b <= nbk; b += blockDim.x) {
    nb.bucket_start[k * (nbk + 1) + b] = bstart[b];
    if (pair_key) abs_bstart[i * (nbk + 1) + b] = base + bstart[b];  // row of the atom: one probe less
  }
  for (int s = tid; s < P.S; s += blockDim.x) nb.sigma_end[k * P.S + s] = bstart[(P.rank_lt[s] + 1) * P.E];
  if (overflow) return;  // consumers skip centres whose list ends past the capacity
  if (RANGED && lds_bmax > lds_keys) {
    // a bucket does not fit the in-LDS sort: leave in-range placeholder
    // entries (the centre itself, or atom 0 for a reference point; no shift)
    // so no consumer reads outside its arrays; the status word reports it
    const int64_t jp = point_mode(bt) ? 0 : i;
    int ei = bt.species[jp];
    ei = ei < 0 ? 0 : (ei >= P.E ? P.E - 1 : ei);
    for (int64_t t = tid; t < total; t += blockDim.x) {
      nb.j[base + t] = (int32_t)jp;
      nb.shift[base + t] = (int32_t)((uint32_t)ei << 24);
      if (pair_key) {
        const uint64_t k = make_key(i, 0, 0, 0);
        pair_key[base + t] = k;
        if (((base + t) & 15) == 0) pair_sum[(base + t) >> 4] = k;
        pair_centre[base + t] = (int32_t)i;
        nb.reverse[base + t] = -1;
      }
    }
    return;
  }
  const int s = astruct[g];
  Cand C;
  cand_setup(C, info, bt, s, fw, g);
  const Shells<SM> shells(P);
  const double rix = nb.rw[g], riy = nb.rw[N + g], riz = nb.rw[2 * N + g];
  // buckets [b_lo, b_hi) whose entries fit the sort together (all of them
  // in the short-list kernel)
  for (int b_lo = 0; b_lo < nbk;) {
    int b_hi = nbk;
    if (RANGED) {
      b_hi = b_lo + 1;
      while (b_hi < nbk && bstart[b_hi + 1] - bstart[b_lo] <= lds_keys) ++b_hi;
      b_hi = __builtin_amdgcn_readfirstlane(b_hi);  // the same for every thread
    }
    const int key0 = RANGED ? __builtin_amdgcn_readfirstlane(bstart[b_lo]) : 0;
    for (int b = b_lo + tid; b < b_hi; b += blockDim.x) cursor[b] = bstart[b] - key0;
    __syncthreads();
    for_each_candidate(C, bin_start, P.rcmax2, w, nw, lds_cand[w],
                       [&](int t, const int *n, double shx, double shy, double shz) {
                         const double dx = (sx[t] - rix) + shx;
                         const double dy = (sy[t] - riy) + shy;
                         const double dz = (sz[t] - riz) + shz;
                         const double q = (dx * dx + dy * dy) + dz * dz;
                         if (q <= P.rcmax2) {
                           const int sh = shells.of(q);
                           const int bk = sh * P.E + ssp[t];
                           if (!RANGED || (bk >= b_lo && bk < b_hi)) {
                             const int pos = atomicAdd(&cursor[bk], 1);
                             if (pos < bstart[bk + 1] - key0) keys[pos] = make_key(sid[t], n[0], n[1], n[2], sh);
                             else atomicOr(status, ST_INTERNAL);
                           }
                         }
                       });
    __syncthreads();
    for (int b = b_lo + w; b < b_hi; b += nw) {
      const int b0 = bstart[b], bn = bstart[b + 1] - b0;
      if (bn == 0) continue;
      uint64_t *kb = keys + (b0 - key0);
      wave_sort(kb, bn);
      const int e = b % P.E;
      for (int t = lane; t < bn; t += kWave) {
        uint64_t k = kb[t];
        int32_t jj = (int32_t)((k >> 24) & 0x7fffffffull);
        uint32_t n1 = (uint32_t)(((k >> 16) & 0xff) - 128) & 0xffu;
        uint32_t n2 = (uint32_t)(((k >> 8) & 0xff) - 128) & 0xffu;
        uint32_t n3 = (uint32_t)((k & 0xff) - 128) & 0xffu;
        nb.j[base + b0 + t] = jj;
        nb.shift[base + b0 + t] = (int32_t)(n1 | (n2 << 8) | (n3 << 16) | ((uint32_t)e << 24));
        if (pair_key) {  // inputs of the reverse-index kernel; the index starts unresolved
          const int64_t gp = base + b0 + t;
          pair_key[gp] = k;
          if ((gp & 15) == 0) pair_sum[gp >> 4] = k;
          pair_centre[gp] = (int32_t)i;
          nb.reverse[gp] = -1;
        }
      }
    }
    if (!RANGED) break;
    __syncthreads();  // the next range reuses the keys and cursors
    b_lo = b_hi;
  }
}

// Short-list fill: one workgroup per centre, centres in cell-list order
// (reference points in index order).
template <int SM>
__global__ __launch_bounds__(256) void k_fill(PlanDev P, BatchDev bt, NbrDev nb, const StructInfo *info,
                                              const double *fw, const int64_t *bin_start,
                                              const double *sx, const double *sy, const double *sz,
                                              const int32_t *sid, const int32_t *ssp, const int32_t *astruct,
                                              const int32_t *cnt, int lds_keys, uint64_t *pair_key,
                                              int32_t *pair_centre, uint64_t *pair_sum, int64_t *abs_bstart,
                                              uint32_t *status, int32_t *long_q) {
  extern __shared__ uint64_t lds_u64[];
  __shared__ CandLds lds_cand[4];
  __shared__ int32_t lds_bmax;
  const int64_t k = xcd_contiguous(blockIdx.x, gridDim.x);  // list slot
  const int64_t i = point_mode(bt) ? k : sid[k];
  fill_centre<false, SM>(P, bt, nb, info, fw, bin_start, sx, sy, sz, sid, ssp, astruct, cnt, lds_keys, pair_key,
                     pair_centre, pair_sum, abs_bstart, status, long_q, k, i, lds_u64, lds_cand, lds_bmax);
}

// Long-list fill: persistent workgroups take the queued centres one at a
// time (status word 6 holds the queue length, word 7 the next entry); every
// workgroup exits once the queue is drained, also when it is empty.
template <int SM>
__global__ __launch_bounds__(256) void k_fill_long(PlanDev P, BatchDev bt, NbrDev nb, const StructInfo *info,
                                                   const double *fw, const int64_t *bin_start,
                                                   const double *sx, const double *sy, const double *sz,
                                                   const int32_t *sid, const int32_t *ssp, const int32_t *astruct,
                                                   const int32_t *cnt, int lds_keys, uint64_t *pair_key,
                                                   int32_t *pair_centre, uint64_t *pair_sum, int64_t *abs_bstart,
                                                   uint32_t *status, int32_t *long_q) {
  extern __shared__ uint64_t lds_u64[];
  __shared__ CandLds lds_cand[4];
  __shared__ int32_t lds_bmax;
  __shared__ uint32_t lds_next;
  const uint32_t nq = __atomic_load_n(status + 6, __ATOMIC_RELAXED);
  for (;;) {
    if (threadIdx.x == 0) lds_next = atomicAdd(status + 7, 1u);
    __syncthreads();
    const uint32_t q = lds_next;
    if (q >= nq) break;
    const int64_t k = long_q[q];
    fill_centre<true, SM>(P, bt, nb, info, fw, bin_start, sx, sy, sz, sid, ssp, astruct, cnt, lds_keys, pair_key,
                      pair_centre, pair_sum, abs_bstart, status, long_q, k, point_mode(bt) ? k : sid[k], lds_u64,
                      lds_cand, lds_bmax);
    __syncthreads();  // lds_next, the keys and the bucket starts are reused
  }
}

// Reverse index: pair (i, j, n) and its mirror (j, i, -n).  One thread per
// pair; only the owner of each mirror couple -- i < j, or i == j with n >= 0
// lexicographically -- searches its mirror among the packed keys of j's
// bucket (shell, species of i; the mirror has the same q, so the shell
// stored in the pair's key) and writes both entries.  The search is bound by
// the cache lines it fetches from lists that do not fit in L2, so it runs on
// two levels: the fill also stores every 16th key (a 16-key window is one
// 128-byte line) and the bucket starts as global indices.
__global__ __launch_bounds__(256) void k_reverse(PlanDev P, BatchDev bt, NbrDev nb, const uint64_t *pair_key,
                                                 const int32_t *pair_centre, const uint64_t *pair_sum,
                                                 const int64_t *abs_bstart, int64_t n_pairs, uint32_t *status) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = bt.n_atoms;
  const int64_t total = nb.offsets[N];
  if (p >= n_pairs || p >= total || total > nb.capacity) return;
  const int nbk = P.E * P.S;
  const uint64_t kp = pair_key[p];
  const int64_t i = pair_centre[p];
  const int32_t j = (int32_t)((kp >> 24) & 0x7fffffffull);
  const int h = (int)(kp >> 60);
  if (i < 0 || i >= N || (int64_t)j >= N || h >= P.S) {  // never for lists the fill wrote
    atomicOr(status, ST_INTERNAL);
    return;
  }
  const int n1 = (int)((kp >> 16) & 0xff) - 128, n2 = (int)((kp >> 8) & 0xff) - 128, n3 = (int)(kp & 0xff) - 128;
  const int lex = n1 != 0 ? n1 : (n2 != 0 ? n2 : n3);
  if (!((int64_t)j > i || ((int64_t)j == i && lex >= 0))) return;
  int ei = bt.species[i];
  ei = ei < 0 ? 0 : (ei >= P.E ? P.E - 1 : ei);
  const int b = h * P.E + ei;  // the mirror has the same q, hence the same shell
  const int64_t *ab = abs_bstart + (int64_t)j * (nbk + 1);  // j's bucket starts (rows by atom)
  const int64_t A = ab[b], Z = ab[b + 1];  // the bucket as global pair indices
  const uint64_t key = make_key(i, -n1, -n2, -n3, h);
  // two levels: the every-16th keys that fall inside the bucket (one or two
  // cache lines) select a 16-key window (one line), searched in turn
  int64_t lo = A, hi = Z;
  if (Z - A > 16) {
    const int64_t sA = (A + 15) >> 4, sB = (Z - 1) >> 4;
    int64_t a = sA, c = sB + 1;  // first sampled key above the key sought
    while (a < c) {
      const int64_t m = (a + c) >> 1;
      if (pair_sum[m] <= key) a = m + 1; else c = m;
    }
    lo = a == sA ? A : (a - 1) * 16;
    hi = a * 16 < Z ? a * 16 : Z;
  }
  int64_t found = -1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const uint64_t km = pair_key[mid];
    if (km == key) { found = mid; break; }
    if (km < key) lo = mid + 1; else hi = mid;
  }
  if (found < 0) {
    atomicOr(status, ST_INTERNAL);
    return;
  }
  nb.reverse[p] = (int32_t)found;
  nb.reverse[found] = (int32_t)p;
}

}  // namespace

// ------------------------------------------------------------------ host launchers
void launch_struct_setup(const gmp_plan *p, const BatchDev &bt, const WsLayout &L, hipStream_t s) {
  int nb = (bt.n_structs + 63) / 64;
  double rcmax = sqrt(p->dev.rcmax2);
  GMP_LAUNCH("nbr_struct_setup", k_struct_setup, dim3(nb), dim3(64), 0, s, bt, L.sinfo, rcmax,
             p->tuning.bin_divisor, L.status);
}

void launch_wrap(const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int n_elements, hipStream_t s) {
  int64_t blocks = (n_total(bt) + 255) / 256;
  if (blocks == 0) return;
  GMP_LAUNCH("nbr_wrap", k_wrap, dim3((unsigned)blocks), dim3(256), 0, s, bt, L.sinfo, nb, L.fw, L.bin_of,
             L.bin_count, L.astruct, n_elements, L.status);
}

void launch_scatter(const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int n_elements, hipStream_t s) {
  int64_t blocks = (bt.n_atoms + 255) / 256;
  if (blocks == 0) return;
  GMP_LAUNCH("nbr_scatter", k_scatter, dim3((unsigned)blocks), dim3(256), 0, s, bt, L.bin_of, L.bin_start,
             L.bin_fill, L.sid_tmp);
  GMP_LAUNCH("nbr_bin_order", k_bin_order, dim3((unsigned)blocks), dim3(256), 0, s, bt, nb, L.bin_of, L.bin_start,
             L.sid_tmp, L.sx, L.sy, L.sz, L.sid, L.ssp, n_elements);
}

void launch_count(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const WsLayout &L, hipStream_t s) {
  int64_t blocks = n_centres(bt);
  if (blocks == 0) return;
  size_t smem = sizeof(int32_t) * p->dev.E * p->dev.S;
  auto kern = p->dev.S <= 8 ? k_count<8> : (p->dev.S <= 12 ? k_count<12> : k_count<kMaxSigmas>);
  GMP_LAUNCH("nbr_count", kern, dim3((unsigned)blocks), dim3(256), smem, s, p->dev, bt, nb, L.sinfo, L.fw,
             L.bin_start, L.sx, L.sy, L.sz, L.sid, L.ssp, L.astruct, L.cnt, L.ptotal, L.status);
}

void launch_list_stats(const gmp_plan *p, const BatchDev &bt, const WsLayout &L, hipStream_t s) {
  const int64_t nc = n_centres(bt), ncnt = nc * p->dev.E * p->dev.S;
  int64_t blocks = (ncnt + 256 * 16 - 1) / (256 * 16);
  blocks = blocks < 1 ? 1 : (blocks > 256 ? 256 : blocks);
  if (nc > 0)
    GMP_LAUNCH("nbr_list_stats", k_list_stats, dim3((unsigned)blocks), dim3(256), 0, s, L.ptotal, nc, L.cnt, ncnt,
               L.status);
}

void launch_fill(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int lds_keys,
                 int long_keys, hipStream_t s) {
  int nbk = p->dev.E * p->dev.S;
  if (n_centres(bt) == 0) return;
  uint64_t *pk = (nb.reverse && !point_mode(bt)) ? L.pair_key : (uint64_t *)nullptr;
  size_t smem = sizeof(uint64_t) * lds_keys + sizeof(int32_t) * (2 * nbk + 2);
  auto kern = p->dev.S <= 8 ? k_fill<8> : (p->dev.S <= 12 ? k_fill<12> : k_fill<kMaxSigmas>);
  GMP_LAUNCH("nbr_fill_sort", kern, dim3((unsigned)n_centres(bt)), dim3(256), smem, s, p->dev, bt, nb, L.sinfo,
             L.fw, L.bin_start, L.sx, L.sy, L.sz, L.sid, L.ssp, L.astruct, L.cnt, lds_keys, pk, L.pair_centre,
             L.pair_sum, L.abs_bstart, L.status, L.long_q);
  if (long_keys > 0) {  // one workgroup per CU (its LDS takes most of the CU's), capped by the centre count
    smem = sizeof(uint64_t) * long_keys + sizeof(int32_t) * (2 * nbk + 2);
    const int64_t blocks = n_centres(bt) < 256 ? n_centres(bt) : 256;
    auto kern_long = p->dev.S <= 8 ? k_fill_long<8> : (p->dev.S <= 12 ? k_fill_long<12> : k_fill_long<kMaxSigmas>);
    GMP_LAUNCH("nbr_fill_long", kern_long, dim3((unsigned)blocks), dim3(256), smem, s, p->dev, bt, nb, L.sinfo,
               L.fw, L.bin_start, L.sx, L.sy, L.sz, L.sid, L.ssp, L.astruct, L.cnt, long_keys, pk, L.pair_centre,
               L.pair_sum, L.abs_bstart, L.status, L.long_q);
  }
}

void launch_reverse(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int64_t n_pairs,
                    hipStream_t s) {
  // every entry of every written list was set to -1 (unresolved) by the fill
  const int64_t blocks = (n_pairs + 255) / 256;
  if (blocks > 0)
    GMP_LAUNCH("nbr_reverse", k_reverse, dim3((unsigned)blocks), dim3(256), 0, s, p->dev, bt, nb, L.pair_key,
               L.pair_centre, L.pair_sum, L.abs_bstart, n_pairs, L.status);
}

}  // namespace gmp
