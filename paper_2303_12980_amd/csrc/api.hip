// C ABI entry points: plan construction, workspace layout, argument
// validation, kernel sequencing, per-kernel event timing.
#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gmp_internal.h"

namespace gmp {

// launchers defined in the kernel translation units
void launch_struct_setup(const gmp_plan *p, const BatchDev &bt, const WsLayout &L, hipStream_t s);
void launch_wrap(const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int n_elements, hipStream_t s);
void launch_scatter(const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int n_elements, hipStream_t s);
void launch_count(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const WsLayout &L, hipStream_t s);
void launch_list_stats(const gmp_plan *p, const BatchDev &bt, const WsLayout &L, hipStream_t s);
void launch_fill(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int lds_keys,
                 int long_keys, hipStream_t s);
void launch_reverse(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int64_t n_pairs,
                    hipStream_t s);
int64_t max_chunks(const gmp_plan *p, int64_t n_atoms, int64_t pairs);
void launch_overlap(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, double *partial, int64_t *nch,
                    int64_t *chunk_off, int64_t *scan_aux, unsigned long long *counter, double4 *rw4,
                    int32_t *astruct, int64_t pairs_bound, hipStream_t s);
void launch_finish(const gmp_plan *p, int64_t N, const double *partial, const int64_t *chunk_off,
                   const int32_t *order, void *features,
                   double *components, hipStream_t s);
void *noalloc_scratch(size_t *bytes, hipError_t *err);
size_t bwd_coef_elems(const gmp_plan *p, int64_t n_atoms);
void launch_backward(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const double *components,
                     const void *grad_features, double *grad_pos, double *grad_cell, const WsLayout &L, int C,
                     int64_t pairs_bound, hipStream_t s);
void fill_zero3(void *p0, size_t b0, void *p1, size_t b1, void *p2, size_t b2, hipStream_t s);
void launch_jacobian(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const double *components, void *jac,
                     int64_t ld, const WsLayout &L, int C, hipStream_t s);

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

gmp_status set_error(gmp_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

gmp_status hip_error(hipError_t e, const char *where) {
  return set_error(GMP_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------------ profiling
namespace {
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;
ProfRec g_pending;

hipEvent_t pool_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
}  // namespace

void prof_before(const char *name, hipStream_t s) {
  if (!g_prof_on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_pending.name = name;
  g_pending.a = pool_event();
  g_pending.b = pool_event();
  (void)hipEventRecord(g_pending.a, s);
}

void prof_after(hipStream_t s) {
  if (!g_prof_on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  (void)hipEventRecord(g_pending.b, s);
  g_prof.push_back(g_pending);
}

// ------------------------------------------------------------------ workspace
int64_t partial_slots(const gmp_plan *p, int64_t n_atoms, int64_t capacity) {
  return max_chunks(p, n_atoms, capacity) * p->dev.S * nmono(p->dev.lmax);
}

// N atoms, M reference points (0 without): per-index arrays cover N + M,
// per-centre arrays max(N, M) (enough for either kind of centre).
WsLayout carve(const gmp_plan *p, int n_structs, int64_t N, int64_t M, int64_t capacity, void *ws,
               size_t ws_bytes) {
  Carver c(ws, ws_bytes);
  WsLayout L;
  const int64_t NB = N + n_structs, NT = N + M, NC = N > M ? N : M;
  const int64_t tiles = M > 0 ? transpose_tiles(capacity) : 0;
  int64_t scan_n = NB > NC ? NB : NC;
  if (256 * tiles > scan_n) scan_n = 256 * tiles;
  const size_t tsz = p->prec == GMP_FP64 ? sizeof(double) : sizeof(float);
  L.status = c.take<uint32_t>(64);
  L.sinfo = c.take<StructInfo>((size_t)n_structs);
  L.bin_of = c.take<int32_t>(N);
  L.astruct = c.take<int32_t>(NT);
  L.bin_count = c.take<int32_t>(NB);
  L.bin_fill = c.take<int32_t>(NB);
  L.bin_start = c.take<int64_t>(NB + 1);
  L.fw = c.take<double>(3 * NT);
  L.sx = c.take<double>(N);
  L.sy = c.take<double>(N);
  L.sz = c.take<double>(N);
  L.sid = c.take<int32_t>(N);
  L.ssp = c.take<int32_t>(N);
  L.cnt = c.take<int32_t>((size_t)NC * p->dev.E * p->dev.S);
  L.ptotal = c.take<int64_t>(NC);
  L.long_q = c.take<int32_t>(NC);
  L.sid_tmp = c.take<int32_t>(N);
  L.scan_aux = c.take<int64_t>(scan_aux_size(scan_n));
  L.partial = c.take<double>(partial_slots(p, NC, capacity));
  L.nch = c.take<int64_t>(NC);
  L.chunk_off = c.take<int64_t>(NC + 1);
  L.counter = c.take<unsigned long long>(32);
  L.rw4 = c.take<double4>(NT);
  L.bcoef = c.take<char>(bwd_coef_elems(p, NC) * tsz);
  L.vbuf = c.take<char>((size_t)capacity * 4 * tsz);
  L.pair_key = c.take<uint64_t>(M > 0 ? 0 : (size_t)capacity);
  L.pair_centre = c.take<int32_t>(M > 0 ? 0 : (size_t)capacity);
  L.pair_sum = c.take<uint64_t>(M > 0 ? 0 : (size_t)(capacity / 16 + 1));
  L.abs_bstart = c.take<int64_t>(M > 0 ? 0 : (size_t)N * (p->dev.E * p->dev.S + 1));
  L.cellpart = c.take<double>((size_t)NC * 9);
  const size_t trn = M > 0 ? (size_t)capacity : 0;
  L.tr_key_in = c.take<uint32_t>(trn);
  L.tr_key_out = c.take<uint32_t>(trn);
  L.tr_val_in = c.take<uint32_t>(trn);
  L.tr_val_out = c.take<uint32_t>(trn);
  L.tr_hist = c.take<int32_t>((size_t)(256 * tiles));
  L.tr_off = c.take<int64_t>(M > 0 ? (size_t)(256 * tiles + 1) : 0);
  L.tr_start = c.take<int64_t>(M > 0 ? (size_t)(N + 1) : 0);
  L.bytes = c.off + 256;
  return L;
}

}  // namespace gmp

using namespace gmp;

// ------------------------------------------------------------------ moment -> component maps
// P_abc(u) = (-1)^l |u|^(2l+1) d^a_x d^b_y d^c_z (1/|u|), expanded into
// monomials of degree l.  Terms coef * x^a y^b z^c r^-k are differentiated
// symbolically, then r^(2l+1-k) (an even power) is expanded as a multinomial.
namespace {
struct Term { int a, b, c, k; };
bool operator<(const Term &x, const Term &y) {
  if (x.a != y.a) return x.a < y.a;
  if (x.b != y.b) return x.b < y.b;
  if (x.c != y.c) return x.c < y.c;
  return x.k < y.k;
}
using Poly = std::map<Term, double>;

Poly diff(const Poly &P, int axis) {
  Poly out;
  for (const auto &kv : P) {
    Term t = kv.first;
    double c = kv.second;
    int e = axis == 0 ? t.a : axis == 1 ? t.b : t.c;
    if (e > 0) {  // derivative of the monomial part
      Term u = t;
      (axis == 0 ? u.a : axis == 1 ? u.b : u.c) -= 1;
      out[u] += c * e;
    }
    // d/dx r^-k = -k x r^-(k+2)
    Term v = t;
    (axis == 0 ? v.a : axis == 1 ? v.b : v.c) += 1;
    v.k += 2;
    out[v] += -c * t.k;
  }
  return out;
}

double fact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

// row-major ncomp(l) x ncomp(l): T[abc][monomial] for degree l
std::vector<double> harmonic_matrix(int l) {
  const int nc = ncomp(l);
  std::vector<double> T((size_t)nc * nc, 0.0);
  for (int a = l; a >= 0; --a)
    for (int b = l - a; b >= 0; --b) {
      const int c = l - a - b;
      Poly P;
      P[Term{0, 0, 0, 1}] = 1.0;
      for (int t = 0; t < a; ++t) P = diff(P, 0);
      for (int t = 0; t < b; ++t) P = diff(P, 1);
      for (int t = 0; t < c; ++t) P = diff(P, 2);
      const double sign = (l % 2) ? -1.0 : 1.0;
      const int row = midx(l, a, b);
      for (const auto &kv : P) {
        const Term &t = kv.first;
        if (kv.second == 0.0) continue;
        const int pw = 2 * l + 1 - t.k;  // remaining power of r, even and >= 0
        const int mexp = pw / 2;
        for (int i = 0; i <= mexp; ++i)
          for (int j = 0; i + j <= mexp; ++j) {
            const int k = mexp - i - j;
            const double mult = fact(mexp) / (fact(i) * fact(j) * fact(k));
            const int A = t.a + 2 * i, B = t.b + 2 * j;
            T[(size_t)row * nc + midx(l, A, B)] += sign * kv.second * mult;
          }
      }
    }
  return T;
}
}  // namespace

// ------------------------------------------------------------------ ABI
extern "C" {

const char *gmp_last_error(void) { return g_err.c_str(); }

static gmp_status validate_desc(const gmp_probe_desc *d, int *mask_out, int *kmax_out, int *dens_out) {
  if (!d) return set_error(GMP_E_INVALID, "null argument");
  if (d->n_orders < 1 || d->n_orders > kMaxOrders || !d->orders)
    return set_error(GMP_E_INVALID, "n_orders must be 1..6");
  if (d->n_sigmas < 1 || d->n_sigmas > kMaxSigmas || !d->sigmas)
    return set_error(GMP_E_INVALID, "n_sigmas must be 1..16");
  if (d->n_elements < 1 || d->n_elements > kMaxElements || !d->prim_offsets)
    return set_error(GMP_E_INVALID, "n_elements must be 1..64");
  if (!(d->overlap_threshold > 0.0) || !isfinite(d->overlap_threshold))
    return set_error(GMP_E_INVALID, "overlap_threshold must be positive and finite");
  if (d->screening != 0 && d->screening != 1) return set_error(GMP_E_INVALID, "screening must be 0 or 1");
  if (d->radial_intervals != 0 && (d->radial_intervals < 16 || d->radial_intervals > 65536))
    return set_error(GMP_E_INVALID, "radial_intervals must be 0 or 16..65536");
  if (d->radial_intervals != 0 && d->screening != 0)
    return set_error(GMP_E_UNSUPPORTED, "tabulated radial factors with per-primitive screening");
  int mask = 0, dens = 0;
  for (int o = 0; o < d->n_orders; ++o) {
    int l = d->orders[o];
    if (l < -1 || l > kMaxL) return set_error(GMP_E_INVALID, "orders must be in -1..4");
    if (l == -1) {
      if (dens) return set_error(GMP_E_INVALID, "orders must be distinct");
      dens = 1;
      continue;
    }
    if (mask & (1 << l)) return set_error(GMP_E_INVALID, "orders must be distinct");
    mask |= 1 << l;
  }
  if (d->n_sigmas + dens > kMaxSigmas)
    return set_error(GMP_E_INVALID, "n_sigmas must be 1..15 with order -1 (at most 16 cutoff slots)");
  for (int s = 0; s < d->n_sigmas; ++s)
    if (!(d->sigmas[s] > 0.0) || !isfinite(d->sigmas[s])) return set_error(GMP_E_INVALID, "sigmas must be > 0");
  if (d->prim_offsets[0] != 0) return set_error(GMP_E_INVALID, "prim_offsets[0] must be 0");
  int kmax = 1;
  for (int e = 0; e < d->n_elements; ++e) {
    int k = d->prim_offsets[e + 1] - d->prim_offsets[e];
    if (k < 0) return set_error(GMP_E_INVALID, "prim_offsets must be ascending");
    if (k > 16) return set_error(GMP_E_UNSUPPORTED, "at most 16 primitives per element");
    if (k > kmax) kmax = k;
  }
  const int np = d->prim_offsets[d->n_elements];
  if (np > 0 && (!d->B || !d->beta)) return set_error(GMP_E_INVALID, "null B or beta");
  for (int k = 0; k < np; ++k) {
    if (!(d->beta[k] > 0.0) || !isfinite(d->beta[k])) return set_error(GMP_E_INVALID, "beta must be > 0");
    if (!isfinite(d->B[k])) return set_error(GMP_E_INVALID, "B must be finite");
  }
  if (mask_out) *mask_out = mask;
  if (kmax_out) *kmax_out = kmax;
  if (dens_out) *dens_out = dens;
  return GMP_OK;
}

// rc(sigma)^2 = max over (e, k) with |A0| > tau of ln(|A0| / tau) / gamma, with
// A0 = |B| (alpha/lambda)^(3/2): beyond it every primitive's l = 0 overlap is
// below the threshold.
static double cutoff2(const gmp_probe_desc *d, int s) {
  const double sg = d->sigmas[s];
  const double alpha = 1.0 / (2.0 * sg * sg);
  double best = 0.0;
  for (int e = 0; e < d->n_elements; ++e)
    for (int k = d->prim_offsets[e]; k < d->prim_offsets[e + 1]; ++k) {
      const double lam = alpha + d->beta[k];
      const double gam = alpha * d->beta[k] / lam;
      const double A0 = fabs(d->B[k]) * pow(alpha / lam, 1.5);
      if (!(A0 > d->overlap_threshold)) continue;
      const double r2 = log(A0 / d->overlap_threshold) / gam;
      if (r2 > best) best = r2;
    }
  return best;
}

// Cutoff of the local density (order -1): rc_{-1}^2 = max over (e, k) with
// |B| > tau of ln(|B| / tau) / beta, where every primitive's density
// |B| exp(-beta q) has fallen below the threshold (the sigma -> 0 limit of
// cutoff2: A0 -> |B|, gamma -> beta).
static double density_cutoff2(const gmp_probe_desc *d) {
  double best = 0.0;
  for (int k = 0; k < d->prim_offsets[d->n_elements]; ++k) {
    const double b = fabs(d->B[k]);
    if (!(b > d->overlap_threshold)) continue;
    const double r2 = log(b / d->overlap_threshold) / d->beta[k];
    if (r2 > best) best = r2;
  }
  return best;
}

gmp_status gmp_probe_cutoffs(const gmp_probe_desc *d, double *rc2) {
  int dens = 0;
  gmp_status st = validate_desc(d, nullptr, nullptr, &dens);
  if (st) return st;
  if (!rc2) return set_error(GMP_E_INVALID, "null rc2");
  for (int s = 0; s < d->n_sigmas; ++s) rc2[s] = cutoff2(d, s);
  if (dens) rc2[d->n_sigmas] = density_cutoff2(d);
  return GMP_OK;
}

gmp_status gmp_plan_create(const gmp_probe_desc *d, gmp_precision precision, gmp_plan **out) {
  if (!d || !out) return set_error(GMP_E_INVALID, "null argument");
  *out = nullptr;
  if (precision != GMP_FP64 && precision != GMP_FP32_COMPENSATED && precision != GMP_FP32_WIDE)
    return set_error(GMP_E_INVALID, "unknown precision");
  int mask = 0, kmax = 1, dens = 0;
  gmp_status vst = validate_desc(d, &mask, &kmax, &dens);
  if (vst) return vst;
  if (d->radial_intervals != 0 && precision == GMP_FP64)
    return set_error(GMP_E_UNSUPPORTED, "tabulated radial factors are an FP32 variant");
  if ((size_t)(d->n_sigmas + dens) * d->n_elements * d->radial_intervals * 80 > (size_t(512) << 20))
    return set_error(GMP_E_UNSUPPORTED, "radial table larger than 512 MB");

  gmp_plan *p = new gmp_plan();
  memset(&p->dev, 0, sizeof(p->dev));
  p->prec = precision;
  p->S = d->n_sigmas + dens;
  p->E = d->n_elements;
  p->n_orders = d->n_orders;
  PlanDev &P = p->dev;
  P.S = p->S;
  P.n_sig = d->n_sigmas;
  P.dens_slot = dens ? d->n_sigmas : -1;
  P.dens_order = -1;
  P.screen = d->screening;
  P.E = p->E;
  P.n_orders = p->n_orders;
  P.order_mask = mask;
  P.kmax = kmax;
  const int kb = kmax <= 4 ? 4 : (kmax <= 8 ? 8 : 16);
  P.kb = kb;
  P.lmax = 0;
  int coff = 0, foff = 0;
  for (int l = 0; l <= kMaxL; ++l) P.order_idx[l] = -1;
  for (int o = 0; o < p->n_orders; ++o) {
    const int l = d->orders[o];
    p->orders[o] = l;
    P.orders[o] = l;
    P.comp_off[o] = coff;
    P.feat_off[o] = foff;
    if (l < 0) {  // the density: one component, one feature
      P.dens_order = o;
      coff += 1;
      foff += 1;
      continue;
    }
    P.order_idx[l] = o;
    coff += P.n_sig * ncomp(l);
    foff += P.n_sig;
    if (l > P.lmax) P.lmax = l;
  }
  P.ncomp_total = coff;
  P.nf = foff;

  std::vector<float> c32((size_t)p->S * p->E * kb * kCoefStride, 0.0f);
  std::vector<double> c64((size_t)p->S * p->E * kb * kCoefStride, 0.0);
  double rcmax2 = 0.0;
  if (dens) {  // density slot: exp(-beta q) with weights B for degree 0 only
    const int s = P.dens_slot;
    for (int e = 0; e < p->E; ++e)
      for (int k = d->prim_offsets[e]; k < d->prim_offsets[e + 1]; ++k) {
        const int kk = k - d->prim_offsets[e];
        const size_t idx = (((size_t)s * p->E + e) * kb + kk) * kCoefStride;
        c64[idx] = -d->beta[k];
        c32[idx] = (float)(-d->beta[k] * 1.4426950408889634);
        c64[idx + 1] = d->B[k];
        c32[idx + 1] = (float)d->B[k];
        c64[idx + 6] = -d->beta[k];
        c32[idx + 6] = (float)(-d->beta[k]);
        // screening radius^2: |B| exp(-beta q) >= tau (FP32 value, as the kernels compare)
        const double bb = fabs(d->B[k]);
        const float r2 = (float)(bb > d->overlap_threshold ? log(bb / d->overlap_threshold) / d->beta[k] : -1.0);
        c64[idx + 7] = r2;
        c32[idx + 7] = r2;
      }
    p->rc2[s] = P.rc2[s] = density_cutoff2(d);
    rcmax2 = P.rc2[s];
  }
  for (int s = 0; s < P.n_sig; ++s) {
    const double sg = d->sigmas[s];
    p->sigmas[s] = sg;
    const double alpha = 1.0 / (2.0 * sg * sg);
    const double best = cutoff2(d, s);
    for (int e = 0; e < p->E; ++e)
      for (int k = d->prim_offsets[e]; k < d->prim_offsets[e + 1]; ++k) {
        const double beta = d->beta[k];
        const double lam = alpha + beta;
        const double gam = alpha * beta / lam;
        const int kk = k - d->prim_offsets[e];
        const size_t idx = (((size_t)s * p->E + e) * kb + kk) * kCoefStride;
        c64[idx] = -gam;
        c32[idx] = (float)(-gam * 1.4426950408889634);  // exp(-g q) = exp2(-g log2(e) q)
        const double ratio = beta / lam;
        double Al = d->B[k] * pow(alpha / lam, 1.5);
        for (int l = 0; l <= kMaxL; ++l) {
          c64[idx + 1 + l] = Al;
          c32[idx + 1 + l] = (float)Al;
          Al *= ratio;
        }
        c64[idx + 6] = -gam;
        c32[idx + 6] = (float)(-gam);
        // screening radius^2: the primitive's own l = 0 overlap reaches tau (FP32 value)
        const double A0 = fabs(d->B[k]) * pow(alpha / lam, 1.5);
        const float r2 = (float)(A0 > d->overlap_threshold ? log(A0 / d->overlap_threshold) / gam : -1.0);
        c64[idx + 7] = r2;
        c32[idx + 7] = r2;
      }
    p->rc2[s] = best;
    P.rc2[s] = best;
    if (best > rcmax2) rcmax2 = best;
  }
  P.rcmax2 = rcmax2;
  // sigma order by rc^2 (stable), rank_lt, shell tables
  for (int s = 0; s < p->S; ++s) P.sig_order[s] = s;
  for (int a = 1; a < p->S; ++a)
    for (int b = a; b > 0 && P.rc2[P.sig_order[b]] < P.rc2[P.sig_order[b - 1]]; --b) {
      int t = P.sig_order[b]; P.sig_order[b] = P.sig_order[b - 1]; P.sig_order[b - 1] = t;
    }
  for (int s = 0; s < p->S; ++s) {
    int r = 0;
    for (int t = 0; t < p->S; ++t) r += P.rc2[t] < P.rc2[s] ? 1 : 0;
    P.rank_lt[s] = r;
  }
  // moment -> component maps and weights
  std::vector<double> T;
  for (int l = 0; l <= kMaxL; ++l) {
    P.toff[l] = (int)T.size();
    std::vector<double> Tl = harmonic_matrix(l);
    T.insert(T.end(), Tl.begin(), Tl.end());
    for (int a = l; a >= 0; --a)
      for (int b = l - a; b >= 0; --b) {
        const int c = l - a - b;
        P.weight[doff(l) + midx(l, a, b)] = fact(l) / (fact(a) * fact(b) * fact(c));
      }
  }
  std::vector<int> kc(p->E);
  for (int e = 0; e < p->E; ++e) kc[e] = d->prim_offsets[e + 1] - d->prim_offsets[e];
  // tabulated radial factors: per (slot, element) and interval [r_k, r_k+1]
  // of r = sqrt(q), the cubic Hermite interpolant of every c_l from its values
  // and r-derivatives at both ends, as coefficients of t = (r - r_k) / h
  const int NTb = d->radial_intervals;
  P.tab_n = NTb;
  std::vector<float> rt((size_t)p->S * p->E * NTb * 5 * 4, 0.0f);
  for (int s = 0; s < p->S && NTb > 0; ++s) {
    const double rc = sqrt(p->rc2[s] > 0.0 ? p->rc2[s] : 0.0);
    const double h = rc > 0.0 ? rc / NTb : 1.0;
    P.tab_inv_h[s] = (float)(1.0 / h);
    const bool dslot = s == P.dens_slot;
    const double alpha = dslot ? 0.0 : 1.0 / (2.0 * p->sigmas[s] * p->sigmas[s]);
    for (int e = 0; e < p->E; ++e) {
      // value and r-derivative of c_l at r
      auto eval = [&](double r, double *f, double *df) {
        for (int l = 0; l <= kMaxL; ++l) { f[l] = 0.0; df[l] = 0.0; }
        for (int k = d->prim_offsets[e]; k < d->prim_offsets[e + 1]; ++k) {
          const double beta = d->beta[k];
          double gam, A0, ratio;
          if (dslot) { gam = beta; A0 = d->B[k]; ratio = 0.0; }
          else {
            const double lam = alpha + beta;
            gam = alpha * beta / lam;
            A0 = d->B[k] * pow(alpha / lam, 1.5);
            ratio = beta / lam;
          }
          const double ex = exp(-gam * r * r);
          double A = A0;
          for (int l = 0; l <= (dslot ? 0 : kMaxL); ++l) {
            f[l] += A * ex;
            df[l] += -2.0 * gam * r * A * ex;
            A *= ratio;
          }
        }
      };
      double f0[kMaxL + 1], d0[kMaxL + 1], f1[kMaxL + 1], d1[kMaxL + 1];
      eval(0.0, f0, d0);
      for (int k = 0; k < NTb; ++k) {
        eval((k + 1) * h, f1, d1);
        for (int l = 0; l <= kMaxL; ++l) {
          const size_t o = ((((size_t)s * p->E + e) * NTb + k) * 5 + l) * 4;
          rt[o] = (float)f0[l];
          rt[o + 1] = (float)(h * d0[l]);
          rt[o + 2] = (float)(3.0 * (f1[l] - f0[l]) - h * (2.0 * d0[l] + d1[l]));
          rt[o + 3] = (float)(2.0 * (f0[l] - f1[l]) + h * (d0[l] + d1[l]));
          f0[l] = f1[l];
          d0[l] = d1[l];
        }
      }
    }
  }

  const size_t b32 = c32.size() * sizeof(float), b64 = c64.size() * sizeof(double);
  const size_t bT = T.size() * sizeof(double), bk = kc.size() * sizeof(int);
  const size_t brt = rt.size() * sizeof(float);
  const size_t o64 = (b32 + 255) & ~size_t(255);
  const size_t oT = (o64 + b64 + 255) & ~size_t(255);
  const size_t ok = (oT + bT + 255) & ~size_t(255);
  const size_t ort = (ok + bk + 255) & ~size_t(255);
  const size_t total = ort + brt;
  hipError_t e = hipMalloc(&p->dmem, total);
  if (e != hipSuccess) { delete p; return hip_error(e, "hipMalloc(plan tables)"); }
  char *base = (char *)p->dmem;
  e = hipMemcpy(base, c32.data(), b32, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(base + o64, c64.data(), b64, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(base + oT, T.data(), bT, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(base + ok, kc.data(), bk, hipMemcpyHostToDevice);
  if (e == hipSuccess && brt > 0) e = hipMemcpy(base + ort, rt.data(), brt, hipMemcpyHostToDevice);
  if (e != hipSuccess) { (void)hipFree(p->dmem); delete p; return hip_error(e, "hipMemcpy(plan tables)"); }
  P.coef32 = (const float *)base;
  P.coef64 = (const double *)(base + o64);
  P.T = (const double *)(base + oT);
  P.kcount = (const int *)(base + ok);
  P.rtab = brt > 0 ? (const float4 *)(base + ort) : nullptr;
  p->tuning.chunk_pairs = 2048;
  p->tuning.bin_divisor = 2;
  p->tuning.blocks_per_cu = 0;
  p->tuning.adj_items = 0;
  p->tuning.sigma_groups = 1;
  *out = p;
  return GMP_OK;
}

void gmp_plan_destroy(gmp_plan *p) {
  if (!p) return;
  if (p->dmem) (void)hipFree(p->dmem);
  delete p;
}

gmp_status gmp_plan_info(const gmp_plan *p, int32_t *n_features, int32_t *n_components, int32_t *n_slots,
                         double *rc2) {
  if (!p) return set_error(GMP_E_INVALID, "null plan");
  if (n_features) *n_features = p->dev.nf;
  if (n_components) *n_components = p->dev.ncomp_total;
  if (n_slots) *n_slots = p->S;
  if (rc2) for (int s = 0; s < p->S; ++s) rc2[s] = p->rc2[s];
  return GMP_OK;
}

gmp_status gmp_plan_get_tuning(const gmp_plan *p, gmp_tuning *t) {
  if (!p || !t) return set_error(GMP_E_INVALID, "null argument");
  *t = p->tuning;
  return GMP_OK;
}

gmp_status gmp_plan_set_tuning(gmp_plan *p, const gmp_tuning *t) {
  if (!p || !t) return set_error(GMP_E_INVALID, "null argument");
  if (t->chunk_pairs < 0) return set_error(GMP_E_INVALID, "chunk_pairs must be >= 0");
  if (t->bin_divisor < 1 || t->bin_divisor > 4) return set_error(GMP_E_INVALID, "bin_divisor must be 1..4");
  if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64) return set_error(GMP_E_INVALID, "blocks_per_cu must be 0..64");
  if (t->adj_items < 0 || t->adj_items > 64) return set_error(GMP_E_INVALID, "adj_items must be 0..64");
  if (t->sigma_groups < 0 || t->sigma_groups > 16) return set_error(GMP_E_INVALID, "sigma_groups must be 0..16");
  p->tuning = *t;
  return GMP_OK;
}

gmp_status gmp_workspace_size(const gmp_plan *p, int32_t n_structs, int64_t n_atoms, int64_t n_points,
                              int64_t capacity, size_t *bytes) {
  if (!p || !bytes) return set_error(GMP_E_INVALID, "null argument");
  if (n_structs < 0 || n_atoms < 0 || n_points < 0 || capacity < 0) return set_error(GMP_E_INVALID, "negative size");
  *bytes = carve(p, n_structs, n_atoms, n_points, capacity, nullptr, 0).bytes;
  return GMP_OK;
}

}  // extern "C"

namespace {

gmp_status check_batch(const gmp_plan *p, const gmp_batch *b) {
  if (!p) return set_error(GMP_E_INVALID, "null plan");
  if (!b) return set_error(GMP_E_INVALID, "null batch");
  if (b->n_structs < 0 || b->n_atoms < 0) return set_error(GMP_E_INVALID, "negative batch size");
  if (b->n_atoms > 0x7ffffff0LL) return set_error(GMP_E_UNSUPPORTED, "at most 2^31-16 atoms per batch");
  if (b->n_atoms > 0 && b->n_structs == 0) return set_error(GMP_E_INVALID, "atoms without structures");
  if (b->n_structs > 0 && (!b->atom_offsets || !b->cell || !b->pbc))
    return set_error(GMP_E_INVALID, "null structure arrays");
  if (b->n_atoms > 0 && (!b->x || !b->y || !b->z || !b->species))
    return set_error(GMP_E_INVALID, "null atom arrays");
  if (b->point_offsets) {
    if (b->n_points < 0) return set_error(GMP_E_INVALID, "negative point count");
    if (b->n_atoms + b->n_points > 0x7ffffff0LL)
      return set_error(GMP_E_UNSUPPORTED, "at most 2^31-16 atoms and points per batch");
    if (b->n_points > 0 && (!b->px || !b->py || !b->pz)) return set_error(GMP_E_INVALID, "null point arrays");
    if (b->n_points > 0 && b->n_structs == 0) return set_error(GMP_E_INVALID, "points without structures");
  }
  return GMP_OK;
}

int64_t batch_points(const gmp_batch *b) { return b->point_offsets ? b->n_points : 0; }
int64_t batch_centres(const gmp_batch *b) { return b->point_offsets ? b->n_points : b->n_atoms; }

gmp_status check_nbrs(const gmp_plan *p, const gmp_batch *b, const gmp_neighbors *n, bool need_lists) {
  if (!n) return set_error(GMP_E_INVALID, "null neighbour lists");
  if (n->capacity < 0) return set_error(GMP_E_INVALID, "negative capacity");
  if (n->max_list < 0) return set_error(GMP_E_INVALID, "negative max_list");
  if (!n->offsets) return set_error(GMP_E_INVALID, "null neighbour offsets");
  if (batch_centres(b) > 0 && (!n->bucket_start || !n->sigma_end || !n->wrap || !n->rw || !n->order || !n->slot))
    return set_error(GMP_E_INVALID, "null neighbour arrays");
  if (need_lists && n->capacity > 0 && (!n->j || !n->shift)) return set_error(GMP_E_INVALID, "null j/shift");
  if (n->reverse && n->capacity > INT32_MAX)
    return set_error(GMP_E_UNSUPPORTED, "the reverse-pair index holds 32-bit pair indices: capacity < 2^31");
  (void)p;
  return GMP_OK;
}

BatchDev to_dev(const gmp_batch *b) {
  BatchDev d;
  d.n_structs = b->n_structs;
  d.n_atoms = b->n_atoms;
  d.atom_offsets = b->atom_offsets;
  d.x = b->x; d.y = b->y; d.z = b->z;
  d.species = b->species;
  d.cell = b->cell;
  d.pbc = b->pbc;
  d.occ = b->occupancy;
  d.n_points = b->point_offsets ? b->n_points : 0;
  d.point_offsets = b->point_offsets;
  d.px = b->px; d.py = b->py; d.pz = b->pz;
  return d;
}

NbrDev to_dev(const gmp_neighbors *n) {
  NbrDev d;
  d.capacity = n->capacity;
  d.offsets = n->offsets;
  d.j = n->j;
  d.shift = n->shift;
  d.bucket_start = n->bucket_start;
  d.sigma_end = n->sigma_end;
  d.wrap = n->wrap;
  d.rw = n->rw;
  d.reverse = n->reverse;
  d.order = n->order;
  d.slot = n->slot;
  return d;
}

gmp_status status_to_error(uint32_t st) {
  if (!st) return GMP_OK;
  if (st & ST_NONFINITE) return set_error(GMP_E_NONFINITE, "non-finite or out-of-range coordinate");
  if (st & ST_CELL) return set_error(GMP_E_CELL, "singular or non-finite lattice for a periodic structure");
  if (st & ST_SPECIES) return set_error(GMP_E_INVALID, "species index outside 0..n_elements-1");
  if (st & ST_SHIFT_RANGE) return set_error(GMP_E_UNSUPPORTED, "cutoff spans more than 126 cells along an axis");
  if (st & ST_OVERFLOW) return set_error(GMP_E_CAPACITY, "neighbour capacity exceeded (no-sync mode)");
  if (st & ST_SORT_SIZE)
    return set_error(GMP_E_STALE,
                     "a (shell, species) bucket is longer than the largest in-LDS sort of this device; the "
                     "centre holds placeholder entries");
  if (st & ST_INTERNAL) return set_error(GMP_E_INVALID, "inconsistent neighbour lists (internal check)");
  return set_error(GMP_E_INVALID, "device status " + std::to_string(st));
}

// In-LDS sort size of a no-sync rebuild: the longest list of the last
// synchronous build with headroom (1/8, at least 64 entries), so lists that
// grow a little between rebuilds of a changing geometry still sort.
int64_t nosync_sort_size(int64_t max_list) {
  const int64_t extra = max_list / 8 > 64 ? max_list / 8 : 64;
  return max_list + extra;
}

// Work items per centre of the adjoint and Jacobian pair kernels: the
// tuning's adj_items, else about 8,192 items over the batch with none
// shorter than chunk_pairs (256 when unsplit) on average.
int64_t adjoint_items(const gmp_plan *p, int64_t pairs, int64_t N) {
  if (p->tuning.adj_items > 0) return p->tuning.adj_items;
  const int64_t chunk = p->tuning.chunk_pairs > 0 ? p->tuning.chunk_pairs : 256;
  int64_t by_pairs = (pairs / N) / chunk;
  if (by_pairs < 1) by_pairs = 1;
  const int64_t want = (8192 + N - 1) / N;
  const int64_t C = want < by_pairs ? want : by_pairs;
  return C < 1 ? 1 : C;
}

// LDS a workgroup may hold on this device (160 KB on gfx950)
static int64_t lds_per_block() {
  static int64_t bytes = 0;
  if (bytes == 0) {
    int dev = 0, v = 65536;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v < 65536)
      v = 65536;
    bytes = v;
  }
  return bytes;
}

// Keys of the fill kernels' in-LDS sorts.  The short-list kernel sorts
// lists of up to maxcnt entries (rounded up to 64; <= 0: its cap), capped at
// kShortSortMax so that several of its workgroups share a CU; longer lists go
// to the long-list kernel, which sorts with the most LDS a workgroup may hold
// (its static LDS, candidate staging and bucket counters, takes up to
// kFillStaticLds bytes).
constexpr int64_t kFillStaticLds = 12 * 1024;
constexpr int64_t kShortSortMax = 8192;
int long_keys_for(const gmp_plan *p) {
  const int nbk = p->dev.E * p->dev.S;
  return (int)((lds_per_block() - kFillStaticLds - 4 * (2 * nbk + 2)) / 8);
}
int lds_keys_for(const gmp_plan *p, int64_t maxcnt) {
  int64_t want = maxcnt <= 0 ? kShortSortMax : ((maxcnt + 63) / 64) * 64;
  if (want > kShortSortMax) want = kShortSortMax;
  const int64_t avail = long_keys_for(p);
  return (int)(want < avail ? want : avail);
}

// The neighbour build; the reverse-pair search is launched only when
// `with_reverse` (gmp_build_lists leaves it to gmp_build_reverse).
gmp_status build_impl(const gmp_plan *p, const gmp_batch *b, gmp_neighbors *n, int64_t *n_pairs, void *ws,
                      size_t ws_bytes, void *stream, bool with_reverse) {
  gmp_status st = check_batch(p, b);
  if (st) return st;
  st = check_nbrs(p, b, n, true);
  if (st) return st;
  if (!ws) return set_error(GMP_E_INVALID, "null workspace");
  hipStream_t s = (hipStream_t)stream;
  WsLayout L = carve(p, b->n_structs, b->n_atoms, batch_points(b), n->capacity, ws, ws_bytes);
  if (L.bytes > ws_bytes) return set_error(GMP_E_NOMEM, "workspace too small");
  const int64_t N = b->n_atoms, NC = batch_centres(b);
  BatchDev bt = to_dev(b);
  NbrDev nb = to_dev(n);
  if (NC == 0) {
    fill_zero(L.status, 64 * sizeof(uint32_t), s);
    fill_zero(n->offsets, sizeof(int64_t), s);
    n->n_pairs = 0;
    if (n_pairs) *n_pairs = 0;
    return GMP_OK;
  }
  const int64_t NB = N + b->n_structs;
  fill_zero3(L.status, 64 * sizeof(uint32_t), L.bin_count, NB * sizeof(int32_t), L.bin_fill, NB * sizeof(int32_t), s);
  launch_struct_setup(p, bt, L, s);
  launch_wrap(bt, nb, L, p->dev.E, s);
  scan_i32_to_i64(L.bin_count, L.bin_start, NB, L.scan_aux, s);
  launch_scatter(bt, nb, L, p->dev.E, s);
  launch_count(p, bt, nb, L, s);
  scan_i64(L.ptotal, n->offsets, NC, L.scan_aux, s);
  int lds_keys, long_keys = long_keys_for(p);
  if (n_pairs) {
    int64_t total = 0;
    uint32_t stw[8];
    launch_list_stats(p, bt, L, s);
    hipError_t e = hipMemcpyAsync(&total, n->offsets + NC, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(stw, L.status, sizeof(stw), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "neighbour count readback");
    st = status_to_error(stw[0]);
    if (st) return st;
    *n_pairs = total;
    n->n_pairs = total;
    if (total > n->capacity)
      return set_error(GMP_E_CAPACITY, "neighbour capacity " + std::to_string(n->capacity) + " < required " +
                                           std::to_string(total));
    n->max_list = stw[4];
    lds_keys = lds_keys_for(p, stw[4]);
    if ((int64_t)stw[5] > long_keys)
      return set_error(GMP_E_UNSUPPORTED, "a centre has " + std::to_string(stw[5]) +
                                              " neighbours of one species in one cutoff shell; the in-LDS sort "
                                              "holds " + std::to_string(long_keys));
    if ((int64_t)stw[4] <= lds_keys) long_keys = 0;  // no list for the long-list kernel
  } else {
    // the pair count is known on the device only: every later call bounds
    // its pair range by the capacity and the device-side list ends; the
    // long-list kernel takes whatever outgrew the short-list sort
    n->n_pairs = 0;
    lds_keys = lds_keys_for(p, n->max_list > 0 ? nosync_sort_size(n->max_list) : 0);
  }
  launch_fill(p, bt, nb, L, lds_keys, long_keys, s);
  // the reverse index pairs mirror entries of atom-centred lists; with
  // reference points the backward orders pairs by neighbour itself
  if (n->reverse && with_reverse && !b->point_offsets)
    launch_reverse(p, bt, nb, L, n_pairs ? *n_pairs : n->capacity, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "neighbour kernels");
  return GMP_OK;
}

}  // namespace

extern "C" {

gmp_status gmp_build_neighbors(const gmp_plan *p, const gmp_batch *b, gmp_neighbors *n, int64_t *n_pairs,
                               void *ws, size_t ws_bytes, void *stream) {
  return build_impl(p, b, n, n_pairs, ws, ws_bytes, stream, true);
}

gmp_status gmp_build_lists(const gmp_plan *p, const gmp_batch *b, gmp_neighbors *n, int64_t *n_pairs, void *ws,
                           size_t ws_bytes, void *stream) {
  return build_impl(p, b, n, n_pairs, ws, ws_bytes, stream, false);
}

gmp_status gmp_build_reverse(const gmp_plan *p, const gmp_batch *b, gmp_neighbors *n, void *ws, size_t ws_bytes,
                             void *stream) {
  gmp_status st = check_batch(p, b);
  if (st) return st;
  st = check_nbrs(p, b, n, true);
  if (st) return st;
  if (!n->reverse) return set_error(GMP_E_INVALID, "null reverse index");
  if (!ws) return set_error(GMP_E_INVALID, "null workspace");
  WsLayout L = carve(p, b->n_structs, b->n_atoms, batch_points(b), n->capacity, ws, ws_bytes);
  if (L.bytes > ws_bytes) return set_error(GMP_E_NOMEM, "workspace too small");
  if (b->n_atoms == 0 || b->point_offsets) return GMP_OK;  // no mirror pairs with reference points
  const int64_t bound = n->n_pairs > 0 && n->n_pairs <= n->capacity ? n->n_pairs : n->capacity;
  launch_reverse(p, to_dev(b), to_dev(n), L, bound, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "reverse-index kernel");
  return GMP_OK;
}

gmp_status gmp_check_status(void *ws, size_t ws_bytes, void *stream) {
  if (!ws || ws_bytes < 256) return set_error(GMP_E_INVALID, "null workspace");
  uint32_t stw[8];
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(stw, ws, sizeof(stw), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "status readback");
  fill_zero(ws, 64 * sizeof(uint32_t), s);
  return status_to_error(stw[0]);
}

gmp_status gmp_features(const gmp_plan *p, const gmp_batch *b, const gmp_neighbors *n, void *features,
                        double *components, void *ws, size_t ws_bytes, void *stream) {
  gmp_status st = check_batch(p, b);
  if (st) return st;
  st = check_nbrs(p, b, n, true);
  if (st) return st;
  const int64_t N = batch_centres(b);
  if (N == 0) return GMP_OK;
  if (!features) return set_error(GMP_E_INVALID, "null features");
  if (!ws) return set_error(GMP_E_INVALID, "null workspace");
  hipStream_t s = (hipStream_t)stream;
  WsLayout L = carve(p, b->n_structs, b->n_atoms, batch_points(b), n->capacity, ws, ws_bytes);
  if (L.bytes > ws_bytes) return set_error(GMP_E_NOMEM, "workspace too small");
  BatchDev bt = to_dev(b);
  NbrDev nb = to_dev(n);
  const int64_t pairs = n->n_pairs > 0 && n->n_pairs <= n->capacity ? n->n_pairs : n->capacity;
  launch_overlap(p, bt, nb, L.partial, L.nch, L.chunk_off, L.scan_aux, L.counter, L.rw4, L.astruct, pairs, s);
  launch_finish(p, N, L.partial, L.chunk_off, n->order, features, components, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "feature kernels");
  return GMP_OK;
}

gmp_status gmp_features_noalloc(const gmp_plan *p, const gmp_batch *b, const gmp_neighbors *n, void *features,
                                double *components, void *stream) {
  gmp_status st = check_batch(p, b);
  if (st) return st;
  st = check_nbrs(p, b, n, true);
  if (st) return st;
  const int64_t N = batch_centres(b);
  if (N == 0) return GMP_OK;
  if (!features) return set_error(GMP_E_INVALID, "null features");
  hipError_t e = hipSuccess;
  size_t cap = 0;
  void *base = noalloc_scratch(&cap, &e);
  if (!base) return hip_error(e, "scratch array address");
  // the forward's scratch: partial moments per work item, chunk counts and
  // offsets, scan carries, the work-item counter, packed positions and
  // structure indices
  const int64_t NC = N, NT = b->n_atoms + batch_points(b);
  const int64_t pairs = n->n_pairs > 0 && n->n_pairs <= n->capacity ? n->n_pairs : n->capacity;
  Carver c(base, cap);
  double *partial = c.take<double>((size_t)max_chunks(p, NC, pairs) * p->dev.S * nmono(p->dev.lmax));
  int64_t *nch = c.take<int64_t>(NC);
  int64_t *chunk_off = c.take<int64_t>(NC + 1);
  int64_t *scan_aux = c.take<int64_t>(scan_aux_size(NC));
  unsigned long long *counter = c.take<unsigned long long>(32);
  double4 *rw4 = c.take<double4>(NT);
  int32_t *astruct = c.take<int32_t>(NT);
  if (c.off > cap)
    return set_error(GMP_E_NOMEM, "gmp_features_noalloc needs " + std::to_string(c.off) +
                                      " bytes of scratch; its fixed array holds " + std::to_string(cap));
  hipStream_t s = (hipStream_t)stream;
  launch_overlap(p, to_dev(b), to_dev(n), partial, nch, chunk_off, scan_aux, counter, rw4, astruct, pairs, s);
  launch_finish(p, N, partial, chunk_off, n->order, features, components, s);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "feature kernels");
  return GMP_OK;
}

gmp_status gmp_features_backward(const gmp_plan *p, const gmp_batch *b, const gmp_neighbors *n,
                                 const double *components, const void *features, const void *grad_features,
                                 double *grad_pos, double *grad_cell, void *ws, size_t ws_bytes, void *stream) {
  (void)features;  // F is recomputed from the FP64 components
  gmp_status st = check_batch(p, b);
  if (st) return st;
  st = check_nbrs(p, b, n, true);
  if (st) return st;
  const int64_t N = batch_centres(b), NT = b->n_atoms + batch_points(b);
  if (N == 0) {  // no centres: zero gradients
    if (grad_pos && NT > 0) fill_zero(grad_pos, (size_t)NT * 3 * sizeof(double), (hipStream_t)stream);
    if (grad_cell && b->n_structs > 0)
      fill_zero(grad_cell, (size_t)b->n_structs * 9 * sizeof(double), (hipStream_t)stream);
    return GMP_OK;
  }
  if (!components || !grad_features || !grad_pos) return set_error(GMP_E_INVALID, "null backward argument");
  if (!n->reverse && !b->point_offsets) return set_error(GMP_E_INVALID, "backward needs the reverse-pair index");
  if (!ws) return set_error(GMP_E_INVALID, "null workspace");
  hipStream_t s = (hipStream_t)stream;
  WsLayout L = carve(p, b->n_structs, b->n_atoms, batch_points(b), n->capacity, ws, ws_bytes);
  if (L.bytes > ws_bytes) return set_error(GMP_E_NOMEM, "workspace too small");
  BatchDev bt = to_dev(b);
  NbrDev nb = to_dev(n);
  const int64_t pairs = n->n_pairs > 0 && n->n_pairs <= n->capacity ? n->n_pairs : n->capacity;
  if (b->point_offsets && pairs > 0xffffffffLL)
    return set_error(GMP_E_UNSUPPORTED, "at most 2^32-1 pairs in the backward of reference points");
  const int64_t C = adjoint_items(p, pairs, N);
  launch_backward(p, bt, nb, components, grad_features, grad_pos, grad_cell, L, (int)C, pairs, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "adjoint kernels");
  return GMP_OK;
}

gmp_status gmp_feature_jacobian(const gmp_plan *p, const gmp_batch *b, const gmp_neighbors *n,
                                const double *components, void *jac, int64_t ld, void *ws, size_t ws_bytes,
                                void *stream) {
  gmp_status st = check_batch(p, b);
  if (st) return st;
  st = check_nbrs(p, b, n, true);
  if (st) return st;
  const int64_t N = batch_centres(b);
  if (N == 0) return GMP_OK;
  if (!components || !jac) return set_error(GMP_E_INVALID, "null jacobian argument");
  const int64_t pairs = n->n_pairs > 0 && n->n_pairs <= n->capacity ? n->n_pairs : n->capacity;
  if (ld < pairs) return set_error(GMP_E_INVALID, "ld smaller than the pair count (capacity in no-sync use)");
  if (!ws) return set_error(GMP_E_INVALID, "null workspace");
  hipStream_t s = (hipStream_t)stream;
  WsLayout L = carve(p, b->n_structs, b->n_atoms, batch_points(b), n->capacity, ws, ws_bytes);
  if (L.bytes > ws_bytes) return set_error(GMP_E_NOMEM, "workspace too small");
  BatchDev bt = to_dev(b);
  NbrDev nb = to_dev(n);
  const int64_t C = adjoint_items(p, pairs, N);
  launch_jacobian(p, bt, nb, components, jac, ld, L, (int)C, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "jacobian kernels");
  return GMP_OK;
}

gmp_status gmp_profile_begin(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof) { g_event_pool.push_back(r.a); g_event_pool.push_back(r.b); }
  g_prof.clear();
  g_prof_on = true;
  return GMP_OK;
}

gmp_status gmp_profile_end(int32_t max_kernels, int32_t *n_kernels, char *names, int32_t *launches, double *ms) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = false;
  std::vector<std::string> order;
  std::map<std::string, std::pair<int, double>> agg;
  for (auto &r : g_prof) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return hip_error(e, "profile event sync");
    float t = 0.f;
    e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return hip_error(e, "profile elapsed time");
    if (!agg.count(r.name)) order.push_back(r.name);
    agg[r.name].first += 1;
    agg[r.name].second += t;
  }
  for (auto &r : g_prof) { g_event_pool.push_back(r.a); g_event_pool.push_back(r.b); }
  g_prof.clear();
  int k = 0;
  for (auto &nm : order) {
    if (k >= max_kernels) break;
    if (names) { strncpy(names + 64 * k, nm.c_str(), 63); names[64 * k + 63] = 0; }
    if (launches) launches[k] = agg[nm].first;
    if (ms) ms[k] = agg[nm].second;
    ++k;
  }
  if (n_kernels) *n_kernels = k;
  return GMP_OK;
}

}  // extern "C"
