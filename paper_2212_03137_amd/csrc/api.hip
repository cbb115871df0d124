// C ABI of the library: context set-up, host-side precomputation (normal-mode transfer
// matrix and coefficients, SPME influence function, cell stencils), the force pipeline,
// stepping, and state and diagnostic transfers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <set>
#include <unordered_map>
#include <vector>

#include "qhp_internal.h"

hipError_t qtb_build_kernels(qhp_ctx* c);

int qhp_fail(qhp_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

// Events come from a pool that grows on demand and is recycled by qhp_profile_read, so a
// timed loop only records events.
static hipEvent_t pool_event(qhp_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

void prof_begin(qhp_ctx* c, int which, hipEvent_t* ev) {
  *ev = nullptr;
  if (c->prof_which != which) return;
  *ev = pool_event(c);
  if (*ev) (void)hipEventRecord(*ev, c->stream);
}

void prof_end(qhp_ctx* c, int which, hipEvent_t ev) {
  if (c->prof_which != which || !ev) return;
  hipEvent_t e2 = pool_event(c);
  if (!e2) return;
  (void)hipEventRecord(e2, c->stream);
  c->ev_pending.emplace_back(ev, e2);
}

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void**)p, n * sizeof(T));
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int next_pow2(int v) { int p = 1; while (p < v) p *= 2; return p; }

// Free ring-polymer modes: T[j][n] real Fourier basis (column 0 = 1/sqrt(P); pairs of
// cos/sin columns for 1 <= k < P/2 with frequency 2 (P / beta hbar) sin(pi k / P); the
// alternating column last for even P), the eigenvectors of the cyclic second-difference
// matrix of eq. matrix_free_RP in order of increasing frequency.
void normal_modes(int P, double beta, double hbar, std::vector<double>& T, std::vector<double>& w) {
  T.assign((size_t)P * P, 0.0);
  w.assign(P, 0.0);
  const double wP = P / (beta * hbar);
  for (int j = 0; j < P; ++j) T[j * P + 0] = 1.0 / std::sqrt((double)P);
  for (int k = 1; 2 * k < P; ++k) {
    for (int j = 0; j < P; ++j) {
      const double ang = 2.0 * M_PI * j * k / P;
      T[j * P + 2 * k - 1] = std::sqrt(2.0 / P) * std::cos(ang);
      T[j * P + 2 * k] = std::sqrt(2.0 / P) * std::sin(ang);
    }
    w[2 * k - 1] = w[2 * k] = 2.0 * wP * std::sin(M_PI * k / P);
  }
  if (P % 2 == 0 && P > 1) {
    for (int j = 0; j < P; ++j) T[j * P + P - 1] = ((j % 2) ? -1.0 : 1.0) / std::sqrt((double)P);
    w[P - 1] = 2.0 * wP;
  }
}

// Cardinal B-spline M_n at integer points 1..n-1 (recursion of Essmann et al. 1995).
double bspline_at(int n, double x) {
  if (n == 2) return (x >= 0 && x <= 2) ? 1.0 - std::fabs(x - 1.0) : 0.0;
  return x / (n - 1) * bspline_at(n - 1, x) + (n - x) / (n - 1) * bspline_at(n - 1, x - 1.0);
}

// |b(m)|^2 = 1 / |sum_{k=0}^{n-2} M_n(k+1) e^{2 pi i m k / K}|^2; a vanishing denominator
// (odd n, m = K/2) takes the neighbouring value.
std::vector<double> bmod(int K, int n) {
  std::vector<double> out(K);
  for (int m = 0; m < K; ++m) {
    double re = 0, im = 0;
    for (int k = 0; k <= n - 2; ++k) {
      const double Mk = bspline_at(n, k + 1.0);
      re += Mk * std::cos(2.0 * M_PI * m * k / K);
      im += Mk * std::sin(2.0 * M_PI * m * k / K);
    }
    const double den = re * re + im * im;
    out[m] = den < 1e-10 ? out[m > 0 ? m - 1 : 0] : 1.0 / den;
  }
  return out;
}

// n x n matrix in the top-left corner of an m x m zero matrix (row-major)
std::vector<double> embed_square(const std::vector<double>& a, int n, int m) {
  std::vector<double> out((size_t)m * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[(size_t)i * m + j] = a[(size_t)i * n + j];
  return out;
}

void free_all(qhp_ctx* c) {
  void* ptrs[] = {c->T, c->mode_c, c->mode_s_w, c->mode_ws, c->mode_c1, c->mode_c2, c->mode_w2,
                  c->d_type, c->d_mass, c->d_charge, c->d_sqrt_mkT, c->d_sigma, c->d_eps,
                  c->Q, c->Pa, c->x, c->g, c->cent, c->cref, c->coff, c->cwrap, c->xf, c->ctrl,
                  c->cell_of, c->cell_count, c->cell_fill, c->cell_start, c->cell_atoms, c->stencil, c->nbr,
                  c->nnbr, c->bmax, c->grid, c->grid2, c->grid_l1, c->tile_of, c->tile_atoms, c->tile_count, c->tile_fill, c->tile_start, c->influence, c->tw[0], c->tw[1], c->tw[2], c->energy,
                  c->io_a, c->io_b, c->xs, c->gs, c->xfs, c->Cs, c->pa_tmp, c->g_eval, c->pg_dq, c->pg_lj, c->pair_tab,
                  c->hvp_out, c->d_charge_alt, c->d_anchor,
                  c->qtb.gamma, c->qtb.hhat, c->qtb.hker, c->qtb.noise, c->qtb.noise_t, c->qtb.vrec_t,
                  c->qtb.vrec, c->qtb.dsum, c->qtb.dbar, c->qtb.vvsum, c->qtb.vfsum,
                  c->qtb.avg_vv, c->qtb.avg_vf, c->qtb.d_tmass, c->qtb.d_inv_count,
                  c->qtb.tw2, c->qtb.tw4, c->snap, c->snap_ctrl};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  c->step_exec = nullptr;
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  c->stream = nullptr;
  if (c->side) (void)hipStreamDestroy(c->side);
  c->side = nullptr;
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  c->ev_fork = c->ev_join = nullptr;
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
  c->ev_pending.clear();
}

hipError_t upload_twiddles(double2** dst, int L) {
  std::vector<double2> t(L);
  for (int m = 0; m < L; ++m) t[m] = make_double2(std::cos(2.0 * M_PI * m / L), -std::sin(2.0 * M_PI * m / L));
  hipError_t e = dalloc(dst, L);
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, t.data(), L * sizeof(double2), hipMemcpyHostToDevice);
}

// Tables of the FP32 pair kernel, indexed by s = r^2 so that a Coulomb-only interaction
// needs no square root: QHP_PAIR_TAB equal intervals of s, interval k = [k, k + 1) / scale,
// each holding the cubic through four equally spaced points (both ends included) of the
// force kernel (erfc(a r)/r + 2a/sqrt(pi) exp(-a^2 r^2)) / r^2 and of the energy kernel
// erfc(a r)/r, as float4 (c0, c1, c2, c3) of c0 + c1 f + c2 f^2 + c3 f^3, f the position in
// the interval. scale = QHP_PAIR_TAB / (rc^2 (1 + 2^-18)), rounded to FP32: then
// fl(r2 scale) < QHP_PAIR_TAB for every FP32 r2 below the FP32 rc^2, so the interval
// index needs no clamp. FP32 evaluation is accurate to ~1.4e-6 relative from r = 1 A
// (closer pairs take the formula) at rc = 9 A, alpha = 0.35 / A.
float pair_table_scale(double rc) {
  return (float)(QHP_PAIR_TAB / (rc * rc * (1.0 + std::ldexp(1.0, -18))));
}

std::vector<float4> pair_tables(double a, float scale) {
  const int n = QHP_PAIR_TAB;
  const double h = 1.0 / (double)scale, c2a = 2.0 * a / std::sqrt(M_PI);
  std::vector<float4> t(2 * n);
  for (int which = 0; which < 2; ++which)
    for (int k = 0; k < n; ++k) {
      double y[4];
      for (int j = 0; j < 4; ++j) {
        const double r = std::max(std::sqrt((k + j / 3.0) * h), 0.25);
        const double e = std::erfc(a * r) / r;
        y[j] = which == 0 ? (e + c2a * std::exp(-a * a * r * r)) / (r * r) : e;
      }
      // the cubic through (0, y0), (1/3, y1), (2/3, y2), (1, y3) in monomial form
      const double c0 = y[0];
      const double c1 = (-11.0 * y[0] + 18.0 * y[1] - 9.0 * y[2] + 2.0 * y[3]) / 2.0;
      const double c2 = 9.0 * (2.0 * y[0] - 5.0 * y[1] + 4.0 * y[2] - y[3]) / 2.0;
      const double c3 = 27.0 * (-y[0] + 3.0 * y[1] - 3.0 * y[2] + y[3]) / 6.0;
      t[(size_t)which * n + k] = make_float4((float)c0, (float)c1, (float)c2, (float)c3);
    }
  return t;
}

// charges of the alchemical system at electrostatic coupling le: solute charges scaled
void scaled_charges(const qhp_ctx* c, double le, std::vector<double>& out) {
  out.resize(c->N);
  for (int i = 0; i < c->N; ++i) out[i] = c->q_given[i] * (c->soft[c->type[i]] ? le : 1.0);
}

// Ewald self term -C alpha / sqrt(pi) sum q^2
double self_of(const qhp_ctx* c, const std::vector<double>& q) {
  double q2 = 0;
  for (double v : q) q2 += v * v;
  return -c->p.coulomb * c->p.ewald_alpha / std::sqrt(M_PI) * q2;
}

int validate(const qhp_params* p, std::string& why) {
  auto bad = [&](const std::string& s) { why = s; return QHP_EINVAL; };
  if (!p) return bad("null params");
  if (p->n_atoms < 3 || p->n_atoms % 3) return bad("n_atoms must be a positive multiple of 3");
  if (p->n_atoms >= (1 << 26)) return bad("n_atoms must be < 2^26");
  if (p->n_beads < 1 || p->n_beads > 64) return bad("n_beads must be in 1..64");
  if ((long long)p->n_atoms * next_pow2(p->n_beads) > (1ll << 27)) {
    why = "n_atoms * n_beads must be <= 2^27 (32-bit byte offsets of the bead arrays)";
    return QHP_EUNSUPPORTED;
  }
  if (!p->type || !p->mass || !p->charge || !p->lj_sigma || !p->lj_epsilon) return bad("null array");
  if (p->n_types < 1 || p->n_types > QHP_MAX_TYPES) return bad("n_types must be in 1..8");
  for (int d = 0; d < 3; ++d)
    if (!(p->box[d] > 0) || !std::isfinite(p->box[d])) return bad("box edges must be positive");
  const double Lmin = std::min(p->box[0], std::min(p->box[1], p->box[2]));
  if (!(p->cutoff > 0) || !(p->cutoff < 0.5 * Lmin)) return bad("cutoff must be in (0, L/2)");
  if (!(p->skin >= 0)) return bad("skin must be >= 0");
  if (!(p->ewald_alpha > 0) || !(p->coulomb > 0)) return bad("alpha and coulomb must be positive");
  if (p->pme_order != 4 && p->pme_order != 5 && p->pme_order != 6 && p->pme_order != 8) {
    why = "pme_order must be 4, 5, 6 or 8";
    return p->pme_order >= 3 && p->pme_order <= 8 ? QHP_EUNSUPPORTED : QHP_EINVAL;
  }
  for (int d = 0; d < 3; ++d) {
    const int K = p->pme_grid[d];
    // powers of two, or multiples of 8 (the spreading tiles the atoms are binned in) whose
    // prime factors are 2, 3, 5 and 7 (the radices of the plain path's transforms)
    int rest = K;
    for (int f : {2, 3, 5, 7})
      while (rest > 1 && rest % f == 0) rest /= f;
    if (K < 8 || K > 128 || !(pow2(K) || (K % 8 == 0 && rest == 1)))
      return bad("pme_grid must be in 8..128: powers of two, or multiples of 8 with prime "
                 "factors 2, 3, 5, 7");
    if (K < 2 * p->pme_order) return bad("pme_grid must be >= 2 * pme_order");
  }
  if (p->precision != QHP_FP64 && p->precision != QHP_FP32_PAIRS) return bad("precision");
  if (p->exec != QHP_BATCHED && p->exec != QHP_PLAIN) return bad("exec");
  if (p->thermostat != QHP_TRPMD && p->thermostat != QHP_ADQTB) return bad("thermostat");
  if (!(p->dt > 0) || !(p->kT > 0) || !(p->hbar > 0)) return bad("dt, kT and hbar must be positive");
  if (p->thermostat == QHP_TRPMD && (!(p->gamma_centroid >= 0) || !(p->trpmd_c >= 0)))
    return bad("friction must be >= 0");
  for (int i = 0; i < p->n_atoms; ++i) {
    if (p->type[i] < 0 || p->type[i] >= p->n_types) return bad("atom type out of range");
    if (!(p->mass[i] > 0) || !std::isfinite(p->charge[i])) return bad("masses > 0, finite charges");
  }
  if (p->rpc_beads < 0 || p->rpc_beads > p->n_beads)
    return bad("rpc_beads must be in 0..n_beads");
  if (p->respa_nalt < 0 || p->respa_nalt > 64) return bad("respa_nalt must be in 0..64");
  if (p->integrator != QHP_BAOAB && p->integrator != QHP_BCOCB) return bad("integrator");
  if (p->qtb_adapt_scheme != QHP_QTB_SIMPLE && p->qtb_adapt_scheme != QHP_QTB_RATIO)
    return bad("qtb_adapt_scheme");
  for (int z = 0; z < p->n_types; ++z) {
    const int sz = p->qtb_scheme_of ? p->qtb_scheme_of[z] : p->qtb_adapt_scheme;
    const double tz = p->qtb_tau_of ? p->qtb_tau_of[z] : p->qtb_tau;
    if (sz != QHP_QTB_SIMPLE && sz != QHP_QTB_RATIO) return bad("qtb_scheme_of");
    if (p->thermostat == QHP_ADQTB && sz == QHP_QTB_RATIO && !(tz > 0))
      return bad("qtb_tau must be > 0 for RATIO adaptation");
  }
  {
    const int ps = p->rpc_beads > 0 ? p->rpc_beads : p->n_beads;
    const int na = p->respa_nalt > 0 ? p->respa_nalt : 1;
    if ((ps < p->n_beads || na > 1) && (p->exec != QHP_BATCHED || p->thermostat != QHP_TRPMD)) {
      why = "ring-polymer contraction and RESPA need exec = QHP_BATCHED and thermostat = QHP_TRPMD";
      return QHP_EUNSUPPORTED;
    }
  }
  if (!(p->tether_k >= 0) || !std::isfinite(p->tether_k)) return bad("tether_k must be >= 0");
  if (p->tether_k > 0) {
    if (!p->tether_anchor) return bad("tether_k > 0 needs tether_anchor");
    for (int i = 0; i < 3 * p->n_atoms; ++i)
      if (!std::isfinite(p->tether_anchor[i])) return bad("tether_anchor must be finite");
    const int ps = p->rpc_beads > 0 ? p->rpc_beads : p->n_beads;
    if (ps < p->n_beads || p->respa_nalt > 1) {
      why = "the tether is not available with ring-polymer contraction or RESPA";
      return QHP_EUNSUPPORTED;
    }
  }
  if (p->type_soft) {
    for (int t = 0; t < p->n_types; ++t)
      if (p->type_soft[t] != 0 && p->type_soft[t] != 1) return bad("type_soft must be 0 or 1");
    if (!(p->lambda_elec >= 0 && p->lambda_elec <= 1) || !(p->lambda_vdw >= 0 && p->lambda_vdw <= 1))
      return bad("lambda_elec and lambda_vdw must be in [0, 1]");
    if (!(p->sc_alpha >= 0) || !std::isfinite(p->sc_alpha)) return bad("sc_alpha must be >= 0");
  }
  if (p->thermostat == QHP_ADQTB) {
    if (p->n_beads != 1) return bad("adQTB requires n_beads = 1");
    // 16..1024, a multiple of 8 (the segment record keeps eight steps together) with no
    // prime factor above 7 (the transforms' radices)
    int rest = p->qtb_nseg;
    for (int f : {2, 3, 5, 7})
      while (rest > 1 && rest % f == 0) rest /= f;
    if (p->qtb_nseg < 16 || p->qtb_nseg > 1024 || p->qtb_nseg % 8 || rest != 1)
      return bad("qtb_nseg must be a multiple of 8 in 16..1024 with prime factors 2, 3, 5, 7");
    if (!(p->qtb_gamma0 > 0) || !(p->qtb_gamma_min_frac >= 0)) return bad("qtb gamma");
    double tmass[QHP_MAX_TYPES];
    bool seen[QHP_MAX_TYPES] = {};
    for (int i = 0; i < p->n_atoms; ++i) {
      const int t = p->type[i];
      if (!seen[t]) { seen[t] = true; tmass[t] = p->mass[i]; }
      else if (tmass[t] != p->mass[i]) return bad("adQTB needs one mass per atom type");
    }
  }
  return QHP_OK;
}

}  // namespace

#define TRY(call)                                                              \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      std::string m_ = std::string(#call) + ": " + hipGetErrorString(e_);      \
      free_all(c); delete c;                                                   \
      return e_ == hipErrorOutOfMemory ? QHP_ENOMEM : QHP_EDEVICE;             \
    }                                                                          \
  } while (0)

extern "C" int qhp_create(const qhp_params* p, void* stream, qhp_ctx** out) {
  if (!out) return QHP_EINVAL;
  *out = nullptr;
  std::string why;
  int v = validate(p, why);
  if (v != QHP_OK) return v;
  qhp_ctx* c = new (std::nothrow) qhp_ctx();
  if (!c) return QHP_ENOMEM;
  c->p = *p;
  // per-type adaptation: the scheme and running-mean time of every type, kept here (the
  // caller's arrays are read at creation only)
  for (int z = 0; z < p->n_types; ++z) {
    c->qtb.ratio_of[z] = (p->qtb_scheme_of ? p->qtb_scheme_of[z] : p->qtb_adapt_scheme) == QHP_QTB_RATIO;
    c->qtb.tau_of[z] = p->qtb_tau_of ? p->qtb_tau_of[z] : p->qtb_tau;
    c->qtb.any_ratio = c->qtb.any_ratio || c->qtb.ratio_of[z];
  }
  c->p.qtb_scheme_of = nullptr;
  c->p.qtb_tau_of = nullptr;
  c->stream = (hipStream_t)stream;
  if (!c->stream) {
    // a private stream (default priority): the null stream cannot be captured into a graph
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return QHP_EDEVICE;
    }
    c->own_stream = true;
  }
  if (p->exec != QHP_PLAIN) {
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
      free_all(c);
      delete c;
      return QHP_EDEVICE;
    }
  }
  c->use_graph = p->use_graph != 0;
  if (scratch_address(&c->scratch) != hipSuccess) {
    free_all(c);
    delete c;
    return QHP_EDEVICE;
  }
  // a bead count that is not a power of two runs in the lanes of the next power of two:
  // the extra (phantom) beads have zero rows and columns in the transfer matrix, so they
  // stay at the centroid, carry no mode and feel no force, and nothing reports them
  const int N = p->n_atoms, Pb = p->n_beads, P = next_pow2(Pb);
  c->N = N; c->P = P; c->Pb = Pb; c->NW = N / 3; c->Pc = P == 1 ? 1 : P / 2;
  c->type.assign(p->type, p->type + N);
  c->mass.assign(p->mass, p->mass + N);
  c->charge.assign(p->charge, p->charge + N);
  c->q_given = c->charge;
  if (p->type_soft) {
    c->alch = true;
    c->soft.assign(p->type_soft, p->type_soft + p->n_types);
    c->lam_e = p->lambda_elec;
    c->lam_v = p->lambda_vdw;
    scaled_charges(c, c->lam_e, c->charge);
  }
  c->sigma.assign(p->lj_sigma, p->lj_sigma + p->n_types);
  c->eps.assign(p->lj_epsilon, p->lj_epsilon + p->n_types);
  for (int d = 0; d < 3; ++d) c->K[d] = p->pme_grid[d];
  c->spme_generic = !(pow2(c->K[0]) && pow2(c->K[1]) && pow2(c->K[2]));
  const bool plain = p->exec == QHP_PLAIN;
  const int Pc_grid = plain ? 1 : c->Pc;
  if (!c->spme_generic) {
    // every FFT pass must split into whole blocks, for the beads and the contracted beads
    const int ps = p->rpc_beads > 0 ? next_pow2(p->rpc_beads) : P;
    const int pcs[2] = {Pc_grid, ps == 1 ? 1 : ps / 2};
    for (int pc : pcs)
      for (int d = 0; d < 3; ++d) {
        const long series = (long)c->K[0] * c->K[1] * c->K[2] * pc / c->K[d];
        if (series % (QHP_FFT_E / c->K[d])) {
          delete c;
          return QHP_EUNSUPPORTED;
        }
      }
  }

  // ---- normal modes and per-mode coefficients (host, FP64) ----
  std::vector<double> Tb, w;
  normal_modes(Pb, 1.0 / p->kT, p->hbar, Tb, w);
  c->h_omega = w;
  std::vector<double> T = embed_square(Tb, Pb, P);
  w.resize(P, 0.0);
  const double h = 0.5 * p->dt;
  // phantom modes (n >= Pb): no rotation, no friction, no noise: they stay zero
  std::vector<double> mc(P, 1.0), msw(P, h), mws(P, 0.0), mc1(P, 1.0), mc2(P, 0.0), mw2(P, 0.0);
  for (int n = 0; n < Pb; ++n) {
    if (p->integrator == QHP_BCOCB) {
      // Cayley form of the rotation (implicit midpoint rule of the free ring-polymer flow):
      // Q' = ((1 - a^2) Q + h P / m) / (1 + a^2), P' = (-m w^2 h Q + (1 - a^2) P) / (1 + a^2)
      const double a2 = 0.25 * w[n] * w[n] * h * h;
      mc[n] = (1.0 - a2) / (1.0 + a2);
      msw[n] = h / (1.0 + a2);
      mws[n] = w[n] * w[n] * h / (1.0 + a2);
    } else {
      mc[n] = std::cos(w[n] * h);
      msw[n] = w[n] > 0 ? std::sin(w[n] * h) / w[n] : h;
      mws[n] = w[n] * std::sin(w[n] * h);
    }
    const double gam = std::max(p->gamma_centroid, p->trpmd_c * w[n]);
    mc1[n] = std::exp(-gam * p->dt);
    mc2[n] = std::sqrt(1.0 - mc1[n] * mc1[n]);
    mw2[n] = w[n] * w[n];
  }
  auto up = [&](double** dst, const std::vector<double>& src) -> hipError_t {
    hipError_t e = dalloc(dst, src.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice);
  };
  TRY(up(&c->T, T));
  TRY(up(&c->mode_c, mc)); TRY(up(&c->mode_s_w, msw)); TRY(up(&c->mode_ws, mws));
  TRY(up(&c->mode_c1, mc1)); TRY(up(&c->mode_c2, mc2)); TRY(up(&c->mode_w2, mw2));

  // ---- per-atom data ----
  std::vector<double> smkT(N);
  for (int i = 0; i < N; ++i) smkT[i] = std::sqrt(c->mass[i] * p->kT);
  TRY(dalloc(&c->d_type, N));
  TRY(hipMemcpy(c->d_type, c->type.data(), N * sizeof(int), hipMemcpyHostToDevice));
  TRY(up(&c->d_mass, c->mass)); TRY(up(&c->d_charge, c->charge)); TRY(up(&c->d_sqrt_mkT, smkT));
  TRY(up(&c->d_sigma, c->sigma)); TRY(up(&c->d_eps, c->eps));
  if (c->alch) TRY(dalloc(&c->d_charge_alt, N));
  c->self_energy = self_of(c, c->charge);

  // ---- state ----
  const size_t NP3 = (size_t)3 * N * P;
  TRY(dalloc(&c->Q, NP3)); TRY(dalloc(&c->Pa, NP3)); TRY(dalloc(&c->x, NP3)); TRY(dalloc(&c->g, NP3));
  TRY(dalloc(&c->cent, N)); TRY(dalloc(&c->cref, N)); TRY(dalloc(&c->coff, N)); TRY(dalloc(&c->cwrap, N));
  TRY(dalloc(&c->xf, (size_t)N * P));
  TRY(dalloc(&c->io_a, NP3)); TRY(dalloc(&c->io_b, NP3)); TRY(dalloc(&c->g_eval, NP3));
  TRY(dalloc(&c->pg_dq, N)); TRY(dalloc(&c->pg_lj, 2 * QHP_MAX_TYPES));
  if (p->precision == QHP_FP32_PAIRS) {
    c->pair_tab_scale = pair_table_scale(p->cutoff);
    c->pair_tab_kmin = (int)std::ceil(1.0 * (double)c->pair_tab_scale);   // from r = 1 A
    const std::vector<float4> tab = pair_tables(p->ewald_alpha, c->pair_tab_scale);
    TRY(dalloc(&c->pair_tab, tab.size()));
    TRY(hipMemcpy(c->pair_tab, tab.data(), tab.size() * sizeof(float4), hipMemcpyHostToDevice));
  }
  TRY(dalloc(&c->energy, (size_t)P * QHP_NTERMS));
  if (p->tether_k > 0) {           // anchors [N][3] -> [3][N]
    std::vector<double> an((size_t)3 * N);
    for (int i = 0; i < N; ++i)
      for (int d = 0; d < 3; ++d) an[(size_t)d * N + i] = p->tether_anchor[3 * i + d];
    c->tether_k = p->tether_k;
    TRY(dalloc(&c->d_anchor, an.size()));
    TRY(hipMemcpy(c->d_anchor, an.data(), an.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  // ---- multiple time stepping / ring-polymer contraction ----
  c->Psb = p->rpc_beads > 0 ? p->rpc_beads : Pb;
  c->Ps = next_pow2(c->Psb);          // lanes of the contracted set (phantoms as above)
  c->nalt = p->respa_nalt > 0 ? p->respa_nalt : 1;
  c->respa = c->Psb < Pb || c->nalt > 1;
  c->pack_qt = p->exec != QHP_PLAIN && !c->respa;
  if (c->respa) {
    const int Ps = c->Ps;
    TRY(dalloc(&c->xs, (size_t)3 * N * Ps)); TRY(dalloc(&c->gs, (size_t)3 * N * Ps));
    TRY(dalloc(&c->xfs, (size_t)N * Ps)); TRY(dalloc(&c->pa_tmp, NP3));
    // C = the transfer matrix of Ps beads (eq. beads_positions with Ps in place of P): the
    // Ps lowest modes of the full polymer, each with unit weight
    std::vector<double> Tc, wc;
    normal_modes(c->Psb, 1.0 / p->kT, p->hbar, Tc, wc);
    TRY(up(&c->Cs, embed_square(Tc, c->Psb, Ps)));
  }
  TRY(hipMemset(c->energy, 0, (size_t)P * QHP_NTERMS * sizeof(double)));
  TRY(hipMemset(c->cref, 0, N * sizeof(double4)));
  TRY(hipMemset(c->coff, 0, N * sizeof(double4)));

  // ---- neighbour list: cells of edge >= r_list / 2 (a small margin keeps rounding of the
  //      fractional coordinate from skipping a cell) and their distinct neighbour cells
  //      within two cells per axis ----
  c->rlist = p->cutoff + p->skin;
  const double half = 0.5 * c->rlist;
  for (int d = 0; d < 3; ++d) {
    int n = std::max(1, (int)std::floor(p->box[d] / half));
    while (n > 1 && p->box[d] / n < half * (1.0 + 1e-9)) --n;
    c->nc[d] = n;
  }
  c->ncell = c->nc[0] * c->nc[1] * c->nc[2];
  c->nst = 125;
  std::vector<int> st((size_t)c->ncell * c->nst, -1);
  for (int a = 0; a < c->nc[0]; ++a)
    for (int b = 0; b < c->nc[1]; ++b)
      for (int e = 0; e < c->nc[2]; ++e) {
        std::set<int> s;
        for (int da = -2; da <= 2; ++da)
          for (int db = -2; db <= 2; ++db)
            for (int de = -2; de <= 2; ++de) {
              const int ia = ((a + da) % c->nc[0] + c->nc[0]) % c->nc[0];
              const int ib = ((b + db) % c->nc[1] + c->nc[1]) % c->nc[1];
              const int ie = ((e + de) % c->nc[2] + c->nc[2]) % c->nc[2];
              s.insert((ia * c->nc[1] + ib) * c->nc[2] + ie);
            }
        int k = 0;
        const int id = (a * c->nc[1] + b) * c->nc[2] + e;
        for (int v2 : s) st[(size_t)id * c->nst + k++] = v2;
      }
  TRY(dalloc(&c->stencil, st.size()));
  TRY(hipMemcpy(c->stencil, st.data(), st.size() * sizeof(int), hipMemcpyHostToDevice));
  const double V = p->box[0] * p->box[1] * p->box[2];
  if (p->nbr_capacity > 0) {
    c->cap = p->nbr_capacity;
  } else {
    const double expect = 4.0 / 3.0 * M_PI * c->rlist * c->rlist * c->rlist * N / V;
    c->cap = (int)std::ceil(1.4 * expect + 64);
    c->cap = (c->cap + 31) / 32 * 32;
  }
  c->cap = std::min(c->cap, N);
  TRY(dalloc(&c->ctrl, 1));
  c->n_bmax = (N + 255) / 256 * 64;      // >= blocks of the normal-mode kernel for any P
  TRY(dalloc(&c->bmax, c->n_bmax));
  TRY(hipMemset(c->bmax, 0, c->n_bmax * sizeof(double4)));
  TRY(hipMemset(c->ctrl, 0, sizeof(NlCtrl)));
  TRY(dalloc(&c->cell_of, N)); TRY(dalloc(&c->cell_count, c->ncell)); TRY(dalloc(&c->cell_fill, c->ncell));
  TRY(dalloc(&c->cell_start, c->ncell + 1)); TRY(dalloc(&c->cell_atoms, N));
  TRY(hipMemset(c->cell_count, 0, c->ncell * sizeof(int)));   // zero between steps
  TRY(dalloc(&c->nbr, (size_t)c->cap * N)); TRY(dalloc(&c->nnbr, N));
  TRY(hipMemset(c->nnbr, 0, N * sizeof(int)));

  // ---- SPME: influence function G(m) and FFT twiddles ----
  const size_t KKK = (size_t)c->K[0] * c->K[1] * c->K[2];
  TRY(dalloc(&c->grid, KKK * Pc_grid));
  if (!plain && Pc_grid >= 2) TRY(dalloc(&c->grid_l1, KKK * Pc_grid));
  {
    std::vector<double> b0 = bmod(c->K[0], p->pme_order), b1 = bmod(c->K[1], p->pme_order),
                        b2 = bmod(c->K[2], p->pme_order);
    std::vector<double> G(KKK);
    const double a2 = p->ewald_alpha * p->ewald_alpha;
    for (int i = 0; i < c->K[0]; ++i)
      for (int j = 0; j < c->K[1]; ++j)
        for (int k = 0; k < c->K[2]; ++k) {
          const double m0 = (i <= c->K[0] / 2 ? i : i - c->K[0]) / p->box[0];
          const double m1 = (j <= c->K[1] / 2 ? j : j - c->K[1]) / p->box[1];
          const double m2 = (k <= c->K[2] / 2 ? k : k - c->K[2]) / p->box[2];
          const double msq = m0 * m0 + m1 * m1 + m2 * m2;
          G[((size_t)i * c->K[1] + j) * c->K[2] + k] =
              msq > 0 ? p->coulomb / (M_PI * V) * std::exp(-M_PI * M_PI * msq / a2) / msq * b0[i] * b1[j] * b2[k]
                      : 0.0;
        }
    TRY(up(&c->influence, G));
  }
  for (int d = 0; d < 3; ++d) TRY(upload_twiddles(&c->tw[d], c->K[d]));
  {
    // 8^3-point spreading tiles and their distinct neighbours (one tile either way)
    int nt[3];
    for (int d = 0; d < 3; ++d) nt[d] = c->K[d] / 8;
    c->ntiles = nt[0] * nt[1] * nt[2];
    TRY(dalloc(&c->tile_of, N)); TRY(dalloc(&c->tile_atoms, N));
    TRY(dalloc(&c->tile_count, c->ntiles)); TRY(dalloc(&c->tile_fill, c->ntiles));
    TRY(dalloc(&c->tile_start, c->ntiles + 1));
    TRY(hipMemset(c->tile_count, 0, c->ntiles * sizeof(int)));
  }

  // ---- adQTB ----
  if (p->thermostat == QHP_ADQTB) {
    QtbState& q = c->qtb;
    q.nseg = p->qtb_nseg;
    const int nk = p->n_types * (q.nseg + 1);
    TRY(dalloc(&q.gamma, nk)); TRY(dalloc(&q.dsum, nk)); TRY(dalloc(&q.dbar, nk));
    TRY(hipMemset(q.dbar, 0, nk * sizeof(double)));
    if (q.any_ratio) {
      TRY(dalloc(&q.vvsum, nk)); TRY(dalloc(&q.vfsum, nk));
      TRY(dalloc(&q.avg_vv, nk)); TRY(dalloc(&q.avg_vf, nk));
      for (double* z : {q.vvsum, q.vfsum, q.avg_vv, q.avg_vf}) TRY(hipMemset(z, 0, nk * sizeof(double)));
    }
    TRY(dalloc(&q.hhat, (size_t)p->n_types * 4 * q.nseg));
    TRY(dalloc(&q.noise, (size_t)q.nseg * 3 * N));
    TRY(dalloc(&q.vrec, (size_t)q.nseg * 3 * N));
    TRY(dalloc(&q.noise_t, (size_t)q.nseg * 3 * N));
    TRY(dalloc(&q.vrec_t, (size_t)q.nseg * 3 * N));
    TRY(upload_twiddles(&q.tw2, 2 * q.nseg));
    TRY(upload_twiddles(&q.tw4, 4 * q.nseg));
    std::vector<double> tm(p->n_types, 1.0), ic(p->n_types, 0.0);
    for (int z = 0; z < p->n_types; ++z) q.type_count[z] = 0;
    for (int i = 0; i < N; ++i) { tm[c->type[i]] = c->mass[i]; q.type_count[c->type[i]]++; }
    for (int z = 0; z < p->n_types; ++z) ic[z] = q.type_count[z] ? 1.0 / (3.0 * q.type_count[z]) : 0.0;
    TRY(up(&q.d_tmass, tm)); TRY(up(&q.d_inv_count, ic));
    q.c1 = std::exp(-p->qtb_gamma0 * p->dt);
    q.osd = std::sqrt((1.0 - q.c1 * q.c1) * p->dt / (2.0 * p->qtb_gamma0));
  }
  *out = c;
  return QHP_OK;
}

extern "C" int qhp_destroy(qhp_ctx* c) {
  if (!c) return QHP_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
  return QHP_OK;
}

BeadSet full_beads(qhp_ctx* c) {
  return BeadSet{c->P, c->Pc, c->x, c->g, c->xf, c->energy, QHP_TERMS_ALL};
}

// V_f (bonds and angles) on the P beads: initialises c->g
static int fast_forces(qhp_ctx* c, bool energy) {
  BeadSet f{c->P, c->Pc, c->x, c->g, c->xf, c->energy, QHP_TERMS_BONDED};
  QHP_HIP(c, launch_bonded(c, energy, -1, &f));
  return QHP_OK;
}

// Bonded (initialises grad V of the bead set), real space and SPME of a bead set after
// the list stage. The SPME spread and transforms depend only on the positions and the
// tile bins of the list stage, so they run on the side stream while the bonded and pair
// kernels run on the main stream; the gather, which adds into grad V, follows both. When
// kernel classes are being timed one at a time, and in the steps a group captures (whose
// members are already concurrent branches), everything stays on the main stream.
static int batched_forces(qhp_ctx* c, bool energy, const BeadSet* bs) {
  if (!c->side || c->serial_forces || c->prof_which != QHP_PROF_OFF) {
    QHP_HIP(c, launch_bonded(c, energy, -1, bs));
    QHP_HIP(c, launch_tether(c, energy, -1, bs));
    QHP_HIP(c, launch_pair(c, energy, -1, bs));
    QHP_HIP(c, launch_spme(c, energy, -1, bs));
    return QHP_OK;
  }
  QHP_HIP(c, hipEventRecord(c->ev_fork, c->stream));
  QHP_HIP(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
  const hipStream_t main = c->stream;
  c->stream = c->side;               // the launchers queue on c->stream
  hipError_t e = launch_spme(c, energy, -1, bs, SPME_FRONT);
  if (e == hipSuccess) e = hipEventRecord(c->ev_join, c->side);
  c->stream = main;
  QHP_HIP(c, e);
  QHP_HIP(c, launch_bonded(c, energy, -1, bs));
  QHP_HIP(c, launch_tether(c, energy, -1, bs));
  QHP_HIP(c, launch_pair(c, energy, -1, bs));
  QHP_HIP(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  QHP_HIP(c, launch_spme(c, energy, -1, bs, SPME_GATHER));
  return QHP_OK;
}

// V_s (exclusion correction, real space, SPME) on the contracted beads: initialises c->gs.
// Phantom contracted beads (lanes Psb..Ps-1) add their terms to energy rows that belong to
// real beads of the full polymer; those terms are cleared again.
static int slow_forces(qhp_ctx* c, bool energy, bool from_step) {
  QHP_HIP(c, launch_nlist(c, from_step));
  BeadSet sl{c->Ps, c->Ps == 1 ? 1 : c->Ps / 2, c->xs, c->gs, c->xfs, c->energy, QHP_TERMS_EXCL};
  int r = batched_forces(c, energy, &sl);
  if (r || !energy || c->Psb == c->Ps) return r;
  QHP_HIP(c, launch_clear_slow_energy(c, c->Psb, c->Ps));
  return QHP_OK;
}

// Bonded + exclusion (initialise grad V), centroid pair list, real space, SPME.
int forces_all(qhp_ctx* c, bool energy, bool from_step) {
  QHP_HIP(c, launch_nlist(c, from_step));
  if (c->p.exec == QHP_PLAIN) {
    for (int b = 0; b < c->P; ++b) {
      QHP_HIP(c, launch_bonded(c, energy, b));
      QHP_HIP(c, launch_tether(c, energy, b));
      QHP_HIP(c, launch_pair(c, energy, b));
      QHP_HIP(c, launch_spme(c, energy, b));
    }
    return QHP_OK;
  }
  return batched_forces(c, energy, nullptr);
}

static int copy_in(qhp_ctx* c, const double* src, int mem_kind, double* dst_internal) {
  const size_t n = (size_t)c->Pb * c->N * 3;
  if (mem_kind == QHP_MEM_HOST) {
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(src[i])) return qhp_fail(c, QHP_ENONFINITE, "non-finite input");
    QHP_HIP(c, hipMemcpyAsync(c->io_a, src, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    QHP_HIP(c, launch_transpose_in(c, c->io_a, dst_internal));
  } else {
    QHP_HIP(c, launch_transpose_in(c, src, dst_internal));
  }
  return QHP_OK;
}

static int copy_out_energy(qhp_ctx* c, double* energy, int mem_kind) {
  if (!energy) return QHP_OK;
  const size_t n = (size_t)c->Pb * QHP_NTERMS * sizeof(double);
  if (mem_kind == QHP_MEM_HOST) {
    QHP_HIP(c, hipMemcpyAsync(energy, c->energy, n, hipMemcpyDeviceToHost, c->stream));
    QHP_HIP(c, hipStreamSynchronize(c->stream));
  } else {
    QHP_HIP(c, hipMemcpyAsync(energy, c->energy, n, hipMemcpyDeviceToDevice, c->stream));
  }
  return QHP_OK;
}

static int read_ctrl(qhp_ctx* c, NlCtrl* h) {
  QHP_HIP(c, hipMemcpyAsync(h, c->ctrl, sizeof(NlCtrl), hipMemcpyDeviceToHost, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  return QHP_OK;
}

static int ctrl_error(qhp_ctx* c, const NlCtrl& h) {
  if (h.overflow)
    return qhp_fail(c, QHP_ENOMEM, "neighbour capacity " + std::to_string(c->cap) +
                                       " exceeded (max count " + std::to_string(h.max_count) + ")");
  if (h.nonfinite) return qhp_fail(c, QHP_ENONFINITE, "state became non-finite");
  if (h.spread_margin)
    return qhp_fail(c, QHP_EUNSUPPORTED,
                    "a bead is further from its centroid than the SPME tile margin allows");
  return QHP_OK;
}

static int check_ctrl(qhp_ctx* c) {
  NlCtrl h;
  int r = read_ctrl(c, &h);
  return r ? r : ctrl_error(c, h);
}

// A list build found more neighbours than a row holds: grow the rows (at least 1.5 times,
// and to the largest count seen plus a margin; at most N), clear the flag and have the
// next list stage rebuild. Captured steps hold the old list buffer: they are recaptured.
static int grow_list(qhp_ctx* c, int max_count) {
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  int cap = std::max(c->cap + c->cap / 2, max_count + max_count / 4 + 32);
  cap = std::min((cap + 31) / 32 * 32, c->N);
  if (cap <= c->cap) return qhp_fail(c, QHP_ENOMEM, "neighbour rows cannot grow further");
  int* nbr = nullptr;
  hipError_t e = hipMalloc((void**)&nbr, (size_t)cap * c->N * sizeof(int));
  if (e != hipSuccess) return qhp_fail(c, QHP_ENOMEM, "neighbour rows: " + std::string(hipGetErrorString(e)));
  (void)hipFree(c->nbr);
  c->nbr = nbr;
  c->cap = cap;
  c->list_grown += 1;
  NlCtrl h;
  int r = read_ctrl(c, &h);
  if (r) return r;
  h.overflow = 0;
  h.force_build = 1;
  QHP_HIP(c, hipMemcpyAsync(c->ctrl, &h, sizeof(NlCtrl), hipMemcpyHostToDevice, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  c->step_exec = nullptr;
  ++c->graph_epoch;
  return QHP_OK;
}

// Run a stateless evaluation (it builds its own list) until no list row overflows.
template <class F>
static int with_list_growth(qhp_ctx* c, F&& run) {
  for (int attempt = 0;; ++attempt) {
    int r = run();
    if (r) return r;
    NlCtrl h;
    if ((r = read_ctrl(c, &h))) return r;
    if (!h.overflow || attempt >= 16) return ctrl_error(c, h);
    if ((r = grow_list(c, h.max_count))) return r;
  }
}

static int eval_once(qhp_ctx* c, const double* pos, double* energy, double* forces, int mem_kind) {
  int r = copy_in(c, pos, mem_kind, c->x);
  if (r) return r;
  QHP_HIP(c, launch_centroid_of_beads(c));
  // the gradient goes to scratch: c->g holds the propagated state's forces
  std::swap(c->g, c->g_eval);
  r = forces_all(c, energy != nullptr, false);
  std::swap(c->g, c->g_eval);
  if (r) return r;
  if (forces) {
    const size_t n = (size_t)c->Pb * c->N * 3;
    if (mem_kind == QHP_MEM_HOST) {
      QHP_HIP(c, launch_transpose_out(c, c->g_eval, c->io_a, -1.0));
      QHP_HIP(c, hipMemcpyAsync(forces, c->io_a, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    } else {
      QHP_HIP(c, launch_transpose_out(c, c->g_eval, forces, -1.0));
    }
  }
  return copy_out_energy(c, energy, mem_kind);
}

extern "C" int qhp_eval(qhp_ctx* c, const double* pos, const double box[3], double* energy,
                        double* forces, int mem_kind) {
  if (!c || !pos) return qhp_fail(c, QHP_EINVAL, "null argument");
  if (box)
    for (int d = 0; d < 3; ++d)
      if (!(std::fabs(box[d] - c->p.box[d]) <= 1e-12 * c->p.box[d]))
        return qhp_fail(c, QHP_EINVAL, "the box differs from the context's (it is fixed per "
                                       "context: create a context for another box)");
  return with_list_growth(c, [&] { return eval_once(c, pos, energy, forces, mem_kind); });
}

extern "C" int qhp_set_lambda(qhp_ctx* c, double lambda_elec, double lambda_vdw) {
  if (!c) return QHP_EINVAL;
  if (!c->alch) return qhp_fail(c, QHP_EINVAL, "no solute (type_soft was not given)");
  if (!(lambda_elec >= 0 && lambda_elec <= 1) || !(lambda_vdw >= 0 && lambda_vdw <= 1))
    return qhp_fail(c, QHP_EINVAL, "lambda_elec and lambda_vdw must be in [0, 1]");
  // earlier queued work may still read the charges: let it finish before overwriting
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  c->lam_e = lambda_elec;
  c->lam_v = lambda_vdw;
  scaled_charges(c, c->lam_e, c->charge);
  c->self_energy = self_of(c, c->charge);
  QHP_HIP(c, hipMemcpy(c->d_charge, c->charge.data(), (size_t)c->N * sizeof(double),
                       hipMemcpyHostToDevice));
  // the captured step holds the old LJ tables and self energy in its kernel arguments
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  c->step_exec = nullptr;
  ++c->graph_epoch;
  return QHP_OK;
}

extern "C" int qhp_eval_lambda(qhp_ctx* c, const double* pos, double lambda_elec,
                               double lambda_vdw, double* energy, double* forces, int mem_kind) {
  if (!c || !pos) return qhp_fail(c, QHP_EINVAL, "null argument");
  if (!c->alch) return qhp_fail(c, QHP_EINVAL, "no solute (type_soft was not given)");
  if (!(lambda_elec >= 0 && lambda_elec <= 1) || !(lambda_vdw >= 0 && lambda_vdw <= 1))
    return qhp_fail(c, QHP_EINVAL, "lambda_elec and lambda_vdw must be in [0, 1]");
  // the other couplings' charges go to a second buffer (the propagated system's stay in
  // place for captured steps); launches read the couplings when they are queued
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  scaled_charges(c, lambda_elec, c->charge_alt);
  QHP_HIP(c, hipMemcpy(c->d_charge_alt, c->charge_alt.data(), (size_t)c->N * sizeof(double),
                       hipMemcpyHostToDevice));
  const double le = c->lam_e, lv = c->lam_v, self = c->self_energy;
  std::swap(c->d_charge, c->d_charge_alt);
  c->lam_e = lambda_elec;
  c->lam_v = lambda_vdw;
  c->self_energy = self_of(c, c->charge_alt);
  int r = qhp_eval(c, pos, nullptr, energy, forces, mem_kind);
  std::swap(c->d_charge, c->d_charge_alt);
  c->lam_e = le;
  c->lam_v = lv;
  c->self_energy = self;
  if (r) return r;
  // the alternative buffer is reused by the next call: finish reading it here
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  return QHP_OK;
}

extern "C" int qhp_bar(const double* du_a, int64_t n_a, const double* du_b, int64_t n_b,
                       double beta, double* dF, int32_t* iterations) {
  if (!du_a || !du_b || !dF || n_a < 1 || n_b < 1 || !(beta > 0)) return QHP_EINVAL;
  double lo = du_a[0], hi = du_a[0];
  for (int64_t k = 0; k < n_a; ++k) {
    if (!std::isfinite(du_a[k])) return QHP_ENONFINITE;
    lo = std::min(lo, du_a[k]); hi = std::max(hi, du_a[k]);
  }
  for (int64_t k = 0; k < n_b; ++k) {
    if (!std::isfinite(du_b[k])) return QHP_ENONFINITE;
    lo = std::min(lo, du_b[k]); hi = std::max(hi, du_b[k]);
  }
  // The pair of equations holds exactly when the self-consistent constant C solves
  // h(C) = sum_B f(C - du) - sum_A f(du - C) = 0, with f(x) = 1 / (1 + e^{beta x}):
  // h falls monotonically from n_b to -n_a, so its root is unique. Newton steps on h,
  // kept inside a bracket that shrinks with every evaluation (bisection when a step
  // would leave it).
  auto fermi = [beta](double x) {                 // both tails to full relative accuracy
    const double y = beta * x, e = std::exp(-std::fabs(y));
    return y > 0 ? e / (1.0 + e) : 1.0 / (1.0 + e);
  };
  auto eval = [&](double C, double& h, double& dh) {
    h = 0.0; dh = 0.0;
    for (int64_t k = 0; k < n_b; ++k) {
      const double f = fermi(C - du_b[k]);
      h += f; dh -= beta * f * (1.0 - f);
    }
    for (int64_t k = 0; k < n_a; ++k) {
      const double f = fermi(du_a[k] - C);
      h -= f; dh -= beta * f * (1.0 - f);
    }
  };
  lo -= 40.0 / beta;
  hi += 40.0 / beta;
  double C = 0.5 * (lo + hi);
  for (int it = 1; it <= 500; ++it) {
    double h, dh;
    eval(C, h, dh);
    if (h > 0) lo = C; else hi = C;
    double next = dh < 0 ? C - h / dh : 0.5 * (lo + hi);
    if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
    const bool done = std::fabs(next - C) <= 1e-13 * std::max(1.0, std::fabs(C)) || h == 0.0 ||
                      !(0.5 * (lo + hi) > lo && 0.5 * (lo + hi) < hi);
    C = h == 0.0 ? C : next;
    if (done) {
      *dF = C - std::log((double)n_b / (double)n_a) / beta;
      if (iterations) *iterations = it;
      return std::isfinite(*dF) ? QHP_OK : QHP_ENONFINITE;
    }
  }
  return QHP_ENONFINITE;
}

extern "C" int qhp_set_launch(qhp_ctx* c, int32_t spread_beads, int32_t spread_ztiles,
                              int32_t fft_slots, int32_t pair_atoms) {
  if (!c) return QHP_EINVAL;
  auto p2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
  if (!(spread_beads == 0 || (p2(spread_beads) && spread_beads <= 16)))
    return qhp_fail(c, QHP_EINVAL, "spread_beads must be 0 or a power of two <= 16");
  if (!(spread_ztiles == 0 || (p2(spread_ztiles) && spread_ztiles <= 8)))
    return qhp_fail(c, QHP_EINVAL, "spread_ztiles must be 0 or a power of two <= 8");
  if (!(fft_slots == 0 || fft_slots == -1 || (p2(fft_slots) && fft_slots <= 8)))
    return qhp_fail(c, QHP_EINVAL, "fft_slots must be -1, 0 or a power of two <= 8");
  if (!(pair_atoms == 0 || pair_atoms == 2 || pair_atoms == 4 || pair_atoms == 8))
    return qhp_fail(c, QHP_EINVAL, "pair_atoms must be 0, 2, 4 or 8");
  c->pair_wpb = pair_atoms;
  c->spread_gb = spread_beads;
  c->spread_z = spread_ztiles;
  c->fft_nb = fft_slots;
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  c->step_exec = nullptr;
  ++c->graph_epoch;
  return QHP_OK;
}

extern "C" int qhp_autotune(qhp_ctx* c, int32_t reps, int32_t* spread_beads,
                            int32_t* spread_ztiles, int32_t* fft_slots, int32_t* pair_atoms) {
  if (!c) return QHP_EINVAL;
  if (reps < 1) return qhp_fail(c, QHP_EINVAL, "reps must be >= 1");
  if (!c->have_state) return qhp_fail(c, QHP_EINVAL, "no state set");
  if (c->p.exec == QHP_PLAIN) {          // one bead per launch: keep the default tile
    if (spread_beads) *spread_beads = 1;
    if (spread_ztiles) *spread_ztiles = 1;
    if (fft_slots) *fft_slots = 0;
    if (pair_atoms) *pair_atoms = 0;
    return QHP_OK;
  }
  // the reciprocal-space pass of the propagated beads (the contracted ones under RESPA),
  // its gradient sent to scratch so that the state is untouched
  BeadSet B = c->respa ? BeadSet{c->Ps, c->Ps == 1 ? 1 : c->Ps / 2, c->xs, c->g_eval, c->xfs,
                                 c->energy, QHP_TERMS_EXCL}
                       : full_beads(c);
  B.g = c->g_eval;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  QHP_HIP(c, hipEventCreate(&t0));
  QHP_HIP(c, hipEventCreate(&t1));
  int best_gb = 0, best_z = 0;
  float best_ms = 0.f;
  hipError_t e = hipSuccess;
  const int nt2 = c->K[2] / QHP_TB;
  for (int gb = 1; gb <= 16 && gb <= B.P && e == hipSuccess; gb *= 2)
    for (int z = 1; z <= 8 && z <= nt2 && gb * z <= 16 && e == hipSuccess; z *= 2) {
      c->spread_gb = gb;
      c->spread_z = z;
      e = launch_spme(c, false, -1, &B);                   // warm
      if (e == hipSuccess) e = hipEventRecord(t0, c->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_spme(c, false, -1, &B);
      if (e == hipSuccess) e = hipEventRecord(t1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e == hipSuccess && (best_gb == 0 || ms < best_ms)) { best_gb = gb; best_z = z; best_ms = ms; }
    }
  c->spread_gb = best_gb;
  c->spread_z = best_z;
  // then the reciprocal transforms: the y-z plane kernel with 1, 2, 4 or 8 slots per
  // block (square 32^2 or 64^2 planes; up to 2 slots at 64) or five one-axis passes
  int best_nb = 0;
  best_ms = 0.f;
  const bool planes = c->K[1] == c->K[2] && (c->K[1] == 32 || c->K[1] == 64);
  const int cap = c->K[1] == 64 ? 2 : 8;
  for (int nb = -1; nb <= 8 && e == hipSuccess; nb = nb < 0 ? 1 : 2 * nb) {
    if (nb > 0 && (!planes || nb > cap || nb > B.Pc)) continue;
    c->fft_nb = nb;
    e = launch_spme(c, false, -1, &B);
    if (e == hipSuccess) e = hipEventRecord(t0, c->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_spme(c, false, -1, &B);
    if (e == hipSuccess) e = hipEventRecord(t1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess && (best_nb == 0 || ms < best_ms)) { best_nb = nb; best_ms = ms; }
  }
  c->fft_nb = best_nb;
  // then the FP32 pair kernel of the same beads: 2, 4 or 8 atoms (wavefronts) per block
  // (FP64 pairs have one shape)
  int best_w = 0;
  const double Lmin = std::min(c->p.box[0], std::min(c->p.box[1], c->p.box[2]));
  if (c->p.precision == QHP_FP32_PAIRS && 2.0 * (c->p.cutoff + c->p.skin) < Lmin) {
    best_ms = 0.f;
    for (int w = 2; w <= 8 && e == hipSuccess; w *= 2) {
      c->pair_wpb = w;
      e = launch_pair(c, false, -1, &B);
      if (e == hipSuccess) e = hipEventRecord(t0, c->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_pair(c, false, -1, &B);
      if (e == hipSuccess) e = hipEventRecord(t1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e == hipSuccess && (best_w == 0 || ms < best_ms)) { best_w = w; best_ms = ms; }
    }
    c->pair_wpb = best_w;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  QHP_HIP(c, e);
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  c->step_exec = nullptr;
  ++c->graph_epoch;
  if (spread_beads) *spread_beads = best_gb;
  if (spread_ztiles) *spread_ztiles = best_z;
  if (fft_slots) *fft_slots = best_nb;
  if (pair_atoms) *pair_atoms = best_w;
  return QHP_OK;
}

extern "C" int qhp_param_grad(qhp_ctx* c, const double* pos, double* dq, double* deps,
                              double* dsig, int mem_kind) {
  if (!c || !pos || !dq || !deps || !dsig) return qhp_fail(c, QHP_EINVAL, "null argument");
  if (c->p.exec == QHP_PLAIN)
    return qhp_fail(c, QHP_EUNSUPPORTED, "parameter gradients need exec = QHP_BATCHED");
  if (c->alch)
    return qhp_fail(c, QHP_EUNSUPPORTED, "parameter gradients of an alchemical system");
  if (c->tether_k > 0)
    return qhp_fail(c, QHP_EUNSUPPORTED, "parameter gradients with the test tether");
  if (c->Pb != c->P)
    return qhp_fail(c, QHP_EUNSUPPORTED, "parameter gradients need a power-of-two bead count");
  auto run = [&]() -> int {
    int r = copy_in(c, pos, mem_kind, c->x);
    if (r) return r;
    QHP_HIP(c, launch_centroid_of_beads(c));
    QHP_HIP(c, launch_zero(c, c->pg_dq, (size_t)c->N * sizeof(double)));
    QHP_HIP(c, launch_zero(c, c->pg_lj, 2 * QHP_MAX_TYPES * sizeof(double)));
    // forces go to scratch (c->g holds the propagated state's); the pair terms always take
    // the FP64 kernel here
    std::swap(c->g, c->g_eval);
    BeadSet B = full_beads(c);
    B.pgrad = 1;
    hipError_t e = launch_nlist(c, false);
    if (e == hipSuccess) e = launch_bonded(c, false, -1, &B);
    if (e == hipSuccess) e = launch_pair(c, false, -1, &B);
    if (e == hipSuccess) e = launch_spme(c, false, -1, &B);
    std::swap(c->g, c->g_eval);
    QHP_HIP(c, e);
    return QHP_OK;
  };
  int r = with_list_growth(c, run);
  if (r) return r;
  const int T = c->p.n_types;
  const hipMemcpyKind k = mem_kind == QHP_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  QHP_HIP(c, hipMemcpyAsync(dq, c->pg_dq, (size_t)c->N * sizeof(double), k, c->stream));
  QHP_HIP(c, hipMemcpyAsync(deps, c->pg_lj, T * sizeof(double), k, c->stream));
  QHP_HIP(c, hipMemcpyAsync(dsig, c->pg_lj + QHP_MAX_TYPES, T * sizeof(double), k, c->stream));
  if (mem_kind == QHP_MEM_HOST) QHP_HIP(c, hipStreamSynchronize(c->stream));
  return QHP_OK;
}

extern "C" int qhp_hvp(qhp_ctx* c, const double* pos, const double* dir, double* out,
                       double* dq, double* deps, double* dsig, int mem_kind) {
  if (!c || !pos || !dir || !out) return qhp_fail(c, QHP_EINVAL, "null argument");
  const bool mix = dq != nullptr;
  if (mix && (!deps || !dsig)) return qhp_fail(c, QHP_EINVAL, "dq, deps and dsig go together");
  if (c->p.exec == QHP_PLAIN)
    return qhp_fail(c, QHP_EUNSUPPORTED, "Hessian-vector products need exec = QHP_BATCHED");
  if (c->alch)
    return qhp_fail(c, QHP_EUNSUPPORTED, "Hessian-vector products of an alchemical system");
  if (c->tether_k > 0)
    return qhp_fail(c, QHP_EUNSUPPORTED, "Hessian-vector products with the test tether");
  if (c->Pb != c->P)
    return qhp_fail(c, QHP_EUNSUPPORTED, "Hessian-vector products need a power-of-two bead count");
  const size_t n = (size_t)c->Pb * c->N * 3;
  if (!c->hvp_out) QHP_HIP(c, hipMalloc((void**)&c->hvp_out, n * sizeof(double)));
  auto run = [&]() -> int {
    int r = copy_in(c, dir, mem_kind, c->io_b);
    if (!r) r = copy_in(c, pos, mem_kind, c->x);
    if (r) return r;
    QHP_HIP(c, launch_centroid_of_beads(c));
    // the potential grid of these positions (and forces, into scratch)
    std::swap(c->g, c->g_eval);
    r = forces_all(c, false, false);
    std::swap(c->g, c->g_eval);
    if (r) return r;
    if (mix) {
      QHP_HIP(c, launch_zero(c, c->pg_dq, (size_t)c->N * sizeof(double)));
      QHP_HIP(c, launch_zero(c, c->pg_lj, 2 * QHP_MAX_TYPES * sizeof(double)));
    }
    QHP_HIP(c, launch_bonded_hvp(c, c->io_b, c->hvp_out, mix));
    BeadSet B = full_beads(c);
    B.g = c->hvp_out;
    B.hvp_u = c->io_b;
    B.pgrad = mix ? 1 : 0;
    QHP_HIP(c, launch_pair(c, false, -1, &B));
    QHP_HIP(c, launch_spme_hvp(c, c->io_b, c->hvp_out, mix));
    return QHP_OK;
  };
  int r = with_list_growth(c, run);
  if (r) return r;
  const hipMemcpyKind k = mem_kind == QHP_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (mix) {
    const int T = c->p.n_types;
    QHP_HIP(c, hipMemcpyAsync(dq, c->pg_dq, (size_t)c->N * sizeof(double), k, c->stream));
    QHP_HIP(c, hipMemcpyAsync(deps, c->pg_lj, T * sizeof(double), k, c->stream));
    QHP_HIP(c, hipMemcpyAsync(dsig, c->pg_lj + QHP_MAX_TYPES, T * sizeof(double), k, c->stream));
  }
  if (mem_kind == QHP_MEM_HOST) {
    QHP_HIP(c, launch_transpose_out(c, c->hvp_out, c->io_a, 1.0));
    QHP_HIP(c, hipMemcpyAsync(out, c->io_a, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    QHP_HIP(c, hipStreamSynchronize(c->stream));
    return QHP_OK;
  }
  QHP_HIP(c, launch_transpose_out(c, c->hvp_out, out, 1.0));
  return QHP_OK;
}

extern "C" int qhp_set_state(qhp_ctx* c, const double* pos, const double* vel, int64_t step, int mem_kind) {
  if (!c || !pos || !vel) return qhp_fail(c, QHP_EINVAL, "null argument");
  if (step < 0) return qhp_fail(c, QHP_EINVAL, "step must be >= 0");
  if (c->p.thermostat == QHP_ADQTB && step % c->qtb.nseg)
    return qhp_fail(c, QHP_EINVAL, "adQTB state must start at a segment boundary");
  // everything from the inputs on is repeated if a list row overflows (the rows then grow)
  auto run = [&]() -> int {
    // bead positions and velocities in the bead-innermost layout, whatever exec is
    const int exec = c->p.exec;
    c->p.exec = QHP_BATCHED;
    int r = copy_in(c, pos, mem_kind, c->io_b);
    if (!r) r = copy_in(c, vel, mem_kind, c->g);
    c->p.exec = exec;
    if (r) return r;
    QHP_HIP(c, launch_beads_to_modes(c, c->io_b, c->g));
    // bead positions in the context's layout for the first force evaluation
    r = copy_in(c, pos, mem_kind, c->x);
    if (r) return r;
    if (c->respa) {
      // V_f on the beads, V_s on the contracted beads; Pa = P - (dt/2) f_f - (n dt/2) f_s
      QHP_HIP(c, launch_contract(c));
      if ((r = fast_forces(c, false))) return r;
      if ((r = slow_forces(c, false, false))) return r;
      QHP_HIP(c, launch_kick_back(c));
      QHP_HIP(c, launch_kick_slow(c, c->Pa, c->Pa, -0.5 * c->nalt * c->p.dt));
    } else {
      QHP_HIP(c, launch_centroid_of_beads(c));
      if ((r = forces_all(c, false, false))) return r;
      QHP_HIP(c, launch_kick_back(c));          // store Pa = P - (dt/2) f
    }
    return QHP_OK;
  };
  int r = with_list_growth(c, run);
  if (r) return r;
  c->step = step;
  {
    long long st = step;
    QHP_HIP(c, hipMemcpyAsync(&c->ctrl->step, &st, sizeof(st), hipMemcpyHostToDevice, c->stream));
    QHP_HIP(c, hipStreamSynchronize(c->stream));
  }
  if (c->p.thermostat == QHP_ADQTB) {
    QHP_HIP(c, qtb_reset_gamma(c));
    QHP_HIP(c, launch_qtb_generate(c, step / c->qtb.nseg));
  }
  c->have_state = true;
  return check_ctrl(c);
}

extern "C" int qhp_get_state(qhp_ctx* c, double* pos, double* vel, int64_t* step, int mem_kind) {
  if (!c) return QHP_EINVAL;
  if (!c->have_state) return qhp_fail(c, QHP_EINVAL, "no state set");
  if (step) *step = c->step;
  if (!pos && !vel) return QHP_OK;
  const size_t n = (size_t)c->Pb * c->N * 3;
  const double* pa = c->Pa;
  if (c->respa) {          // momenta with the pending slow kick (n dt/2) f_s
    QHP_HIP(c, launch_kick_slow(c, c->pa_tmp, c->Pa, 0.5 * c->nalt * c->p.dt));
    pa = c->pa_tmp;
  }
  if (mem_kind == QHP_MEM_HOST) {
    QHP_HIP(c, launch_state_out(c, pos ? c->io_a : nullptr, vel ? c->io_b : nullptr, pa));
    if (pos) QHP_HIP(c, hipMemcpyAsync(pos, c->io_a, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (vel) QHP_HIP(c, hipMemcpyAsync(vel, c->io_b, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    QHP_HIP(c, hipStreamSynchronize(c->stream));
  } else {
    QHP_HIP(c, launch_state_out(c, pos, vel, pa));
  }
  return QHP_OK;
}

// One propagation step: B A O A (normal modes), then bonded, list check/rebuild, pairs
// and SPME at the new beads. Under RESPA / contraction one outer step: n inner steps
// (kick with dt f_f, plus n dt f_s in the first; A O A; V_f at the new beads), then V_s
// at the contracted beads of the last.
static int one_step(qhp_ctx* c, bool energy) {
  hipEvent_t ev = nullptr;
  if (!c->respa) {
    prof_begin(c, QHP_PROF_NM, &ev);
    QHP_HIP(c, launch_nm_step(c, 0, 0.0, true));
    prof_end(c, QHP_PROF_NM, ev);
    return forces_all(c, energy, true);
  }
  for (int k = 0; k < c->nalt; ++k) {
    const bool last = k == c->nalt - 1;
    prof_begin(c, QHP_PROF_NM, &ev);
    QHP_HIP(c, launch_nm_step(c, k, k == 0 ? c->nalt * c->p.dt : 0.0, last));
    prof_end(c, QHP_PROF_NM, ev);
    int r = fast_forces(c, energy && last);
    if (r) return r;
  }
  return slow_forces(c, energy, true);
}

// Capture one step (without energies) as a HIP graph on the context's stream.
static int capture_step(qhp_ctx* c) {
  hipGraph_t g = nullptr;
  QHP_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int r = one_step(c, false);
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (r) { if (g) (void)hipGraphDestroy(g); return r; }
  if (e != hipSuccess) return qhp_fail(c, QHP_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&c->step_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->step_exec = nullptr;
    return qhp_fail(c, QHP_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  return QHP_OK;
}

// The propagated state a call to qhp_step starts from, kept on the device so that the call
// can be repeated when a list build overflows its rows: modes, momenta, gradients, the
// control block (step counter, build bookkeeping) and the adQTB adaptation state. The
// coloured noise of the segment and the recorded velocities are rewritten by the repeat.
static int snapshot(qhp_ctx* c, bool save) {
  const size_t NP3 = (size_t)3 * c->N * c->P;
  const size_t NS3 = c->respa ? (size_t)3 * c->N * c->Ps : 0;
  const size_t nk = c->p.thermostat == QHP_ADQTB ? (size_t)c->p.n_types * (c->qtb.nseg + 1) : 0;
  double* parts[] = {c->Q, c->Pa, c->g, c->gs, c->qtb.gamma, c->qtb.dbar, c->qtb.avg_vv,
                     c->qtb.avg_vf};
  const size_t sizes[] = {NP3, NP3, NP3, NS3, nk, nk, c->qtb.avg_vv ? nk : 0,
                          c->qtb.avg_vf ? nk : 0};
  size_t total = 0;
  for (size_t z : sizes) total += z;
  if (!c->snap) {
    if (!save) return QHP_OK;
    QHP_HIP(c, hipMalloc((void**)&c->snap, total * sizeof(double)));
    QHP_HIP(c, hipMalloc((void**)&c->snap_ctrl, sizeof(NlCtrl)));
  }
  size_t off = 0;
  for (int k = 0; k < 8; ++k) {
    if (sizes[k] == 0) continue;
    void* dst = save ? (void*)(c->snap + off) : (void*)parts[k];
    const void* src = save ? (const void*)parts[k] : (const void*)(c->snap + off);
    QHP_HIP(c, hipMemcpyAsync(dst, src, sizes[k] * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    off += sizes[k];
  }
  QHP_HIP(c, hipMemcpyAsync(save ? (void*)c->snap_ctrl : (void*)c->ctrl,
                            save ? (const void*)c->ctrl : (const void*)c->snap_ctrl,
                            sizeof(NlCtrl), hipMemcpyDeviceToDevice, c->stream));
  return QHP_OK;
}

static int run_steps(qhp_ctx* c, int32_t nsteps, bool want_energy) {
  const bool qtb = c->p.thermostat == QHP_ADQTB;
  for (int s = 0; s < nsteps; ++s) {
    const bool want_e = want_energy && s == nsteps - 1;
    const bool graph = c->use_graph && !want_e && c->prof_which == QHP_PROF_OFF;
    if (graph) {
      if (!c->step_exec) {
        int r = capture_step(c);
        if (r) return r;
      }
      QHP_HIP(c, hipGraphLaunch(c->step_exec, c->stream));
    } else {
      int r = one_step(c, want_e);
      if (r) return r;
    }
    c->step += c->nalt;
    if (qtb && c->step % c->qtb.nseg == 0) {
      QHP_HIP(c, launch_qtb_adapt(c));
      QHP_HIP(c, launch_qtb_generate(c, c->step / c->qtb.nseg));
    }
  }
  return QHP_OK;
}

extern "C" int qhp_step(qhp_ctx* c, int32_t nsteps, double* energy, int mem_kind) {
  if (!c) return QHP_EINVAL;
  if (!c->have_state) return qhp_fail(c, QHP_EINVAL, "no state set");
  if (nsteps < 0) return qhp_fail(c, QHP_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return check_ctrl(c);
  // rows of N entries cannot overflow; otherwise keep the starting state for a repeat
  const bool guard = c->cap < c->N;
  const int64_t step0 = c->step;
  if (guard) {
    int r = snapshot(c, true);
    if (r) return r;
  }
  for (int attempt = 0;; ++attempt) {
    int r = run_steps(c, nsteps, energy != nullptr);
    if (r) return r;
    NlCtrl h;
    if ((r = read_ctrl(c, &h))) return r;
    if (!h.overflow || !guard || attempt >= 16) {
      if ((r = ctrl_error(c, h))) return r;
      break;
    }
    // a build ran out of row space: back to the starting state, larger rows, again
    if ((r = snapshot(c, false))) return r;
    c->step = step0;
    if ((r = grow_list(c, h.max_count))) return r;
    if (c->p.thermostat == QHP_ADQTB) QHP_HIP(c, launch_qtb_generate(c, step0 / c->qtb.nseg));
  }
  return copy_out_energy(c, energy, mem_kind);
}

extern "C" int qhp_mode_energies(qhp_ctx* c, double* kinetic, double* spring) {
  if (!c || !kinetic || !spring) return QHP_EINVAL;
  if (!c->have_state) return qhp_fail(c, QHP_EINVAL, "no state set");
  QHP_HIP(c, launch_zero(c, c->io_a, 2 * sizeof(double)));
  const double* pa = c->Pa;
  if (c->respa) {
    QHP_HIP(c, launch_kick_slow(c, c->pa_tmp, c->Pa, 0.5 * c->nalt * c->p.dt));
    pa = c->pa_tmp;
  }
  QHP_HIP(c, launch_mode_energies(c, c->io_a, pa));
  double h[2];
  QHP_HIP(c, hipMemcpyAsync(h, c->io_a, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  *kinetic = h[0];
  *spring = h[1];
  return QHP_OK;
}

extern "C" int qhp_mode_energies_noalloc(qhp_ctx* c, double* out) {
  if (!c || !out) return QHP_EINVAL;
  if (!c->have_state) return qhp_fail(c, QHP_EINVAL, "no state set");
  if (mode_energy_parts(c) > QHP_SCRATCH_DOUBLES)
    return qhp_fail(c, QHP_ENOMEM, "the partial sums of " + std::to_string(mode_energy_parts(c) / 2) +
                                       " blocks exceed the 1 MiB scratch (65,536 blocks)");
  const double* pa = c->Pa;
  if (c->respa) {
    QHP_HIP(c, launch_kick_slow(c, c->pa_tmp, c->Pa, 0.5 * c->nalt * c->p.dt));
    pa = c->pa_tmp;
  }
  QHP_HIP(c, launch_mode_energies_noalloc(c, out, pa));
  return QHP_OK;
}

extern "C" int qhp_nlist_export(qhp_ctx* c, int32_t* pairs, int64_t capacity, int64_t* npairs) {
  if (!c || !npairs) return QHP_EINVAL;
  const int N = c->N;
  std::vector<int> nn(N), nb((size_t)c->cap * N);
  QHP_HIP(c, hipMemcpyAsync(nn.data(), c->nnbr, N * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  QHP_HIP(c, hipMemcpyAsync(nb.data(), c->nbr, nb.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<std::pair<int, int>> out;
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < nn[i]; ++k) {
      const int j = nb[(size_t)i * c->cap + k] & 0x3FFFFFF;
      if (j > i) out.emplace_back(i, j);
    }
  std::sort(out.begin(), out.end());
  *npairs = (int64_t)out.size();
  if (!pairs) return QHP_OK;
  if ((int64_t)out.size() > capacity) return qhp_fail(c, QHP_ENOMEM, "pairs buffer too small");
  for (size_t k = 0; k < out.size(); ++k) { pairs[2 * k] = out[k].first; pairs[2 * k + 1] = out[k].second; }
  return QHP_OK;
}

extern "C" int qhp_nlist_stats(qhp_ctx* c, int64_t* builds, int32_t* max_count, int32_t* capacity) {
  if (!c || !builds || !max_count || !capacity) return QHP_EINVAL;
  NlCtrl h;
  QHP_HIP(c, hipMemcpyAsync(&h, c->ctrl, sizeof(NlCtrl), hipMemcpyDeviceToHost, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  *builds = h.n_builds;
  *max_count = h.max_count;
  *capacity = c->cap;
  return QHP_OK;
}

extern "C" int qhp_noise_export(qhp_ctx* c, int32_t stream, int64_t step, double* out) {
  if (!c || !out) return QHP_EINVAL;
  if (stream != 5 && stream != 6) return qhp_fail(c, QHP_EINVAL, "stream must be 5 or 6");
  if (stream == 5 && step < 0) return qhp_fail(c, QHP_EINVAL, "step must be >= 0");
  if (stream == 6 && step + c->p.qtb_nseg < 0)
    return qhp_fail(c, QHP_EINVAL, "white-noise step must be >= -N_seg");
  const size_t n = (size_t)(stream == 5 ? c->Pb : 1) * c->N * 3;
  QHP_HIP(c, launch_noise_export(c, stream, step, c->io_a));
  QHP_HIP(c, hipMemcpyAsync(out, c->io_a, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  return QHP_OK;
}

extern "C" int qhp_qtb_get_gamma(qhp_ctx* c, double* gamma) {
  if (!c || !gamma) return QHP_EINVAL;
  if (c->p.thermostat != QHP_ADQTB) return qhp_fail(c, QHP_EINVAL, "not an adQTB context");
  const size_t n = (size_t)c->p.n_types * (c->qtb.nseg + 1) * sizeof(double);
  QHP_HIP(c, hipMemcpyAsync(gamma, c->qtb.gamma, n, hipMemcpyDeviceToHost, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  return QHP_OK;
}

extern "C" int qhp_qtb_set_gamma(qhp_ctx* c, const double* gamma) {
  if (!c || !gamma) return QHP_EINVAL;
  if (c->p.thermostat != QHP_ADQTB) return qhp_fail(c, QHP_EINVAL, "not an adQTB context");
  const size_t n = (size_t)c->p.n_types * (c->qtb.nseg + 1) * sizeof(double);
  QHP_HIP(c, hipMemcpyAsync(c->qtb.gamma, gamma, n, hipMemcpyHostToDevice, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  if (c->have_state) QHP_HIP(c, launch_qtb_generate(c, c->step / c->qtb.nseg));
  return QHP_OK;
}

extern "C" int qhp_qtb_get_noise(qhp_ctx* c, double* noise) {
  if (!c || !noise) return QHP_EINVAL;
  if (c->p.thermostat != QHP_ADQTB) return qhp_fail(c, QHP_EINVAL, "not an adQTB context");
  // device layout [t][3][N] -> boundary [t][N][3]
  const int N = c->N, S = c->qtb.nseg;
  std::vector<double> tmp((size_t)S * 3 * N);
  QHP_HIP(c, hipMemcpyAsync(tmp.data(), c->qtb.noise, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  for (int t = 0; t < S; ++t)
    for (int a = 0; a < N; ++a)
      for (int d = 0; d < 3; ++d) noise[((size_t)t * N + a) * 3 + d] = tmp[((size_t)t * 3 + d) * N + a];
  return QHP_OK;
}

extern "C" int qhp_qtb_get_delta(qhp_ctx* c, double* delta) {
  if (!c || !delta) return QHP_EINVAL;
  if (c->p.thermostat != QHP_ADQTB) return qhp_fail(c, QHP_EINVAL, "not an adQTB context");
  const size_t n = (size_t)c->p.n_types * (c->qtb.nseg + 1) * sizeof(double);
  QHP_HIP(c, hipMemcpyAsync(delta, c->qtb.dbar, n, hipMemcpyDeviceToHost, c->stream));
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  return QHP_OK;
}

extern "C" int qhp_profile(qhp_ctx* c, int which) {
  if (!c) return QHP_EINVAL;
  if (which < 0 || which > QHP_PROF_NM) return qhp_fail(c, QHP_EINVAL, "profile class");
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  c->ev_pending.clear();
  c->ev_used = 0;
  c->prof_which = which;
  c->prof_ms = 0;
  c->prof_launches = 0;
  return QHP_OK;
}

extern "C" int qhp_profile_read(qhp_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return QHP_EINVAL;
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  for (auto& pr : c->ev_pending) {
    float t = 0;
    if (hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) c->prof_ms += t;
    c->prof_launches += 1;
  }
  c->ev_pending.clear();
  c->ev_used = 0;
  *ms = c->prof_ms;
  *launches = c->prof_launches;
  return QHP_OK;
}

extern "C" int qhp_sync(qhp_ctx* c) {
  if (!c) return QHP_EINVAL;
  QHP_HIP(c, hipStreamSynchronize(c->stream));
  return QHP_OK;
}

extern "C" const char* qhp_last_error(qhp_ctx* c) { return c ? c->err.c_str() : "null context"; }

// ------------------------------- groups of contexts ------------------------------------
struct qhp_group {
  std::vector<qhp_ctx*> m;
  std::vector<int64_t> epoch;        // members' graph epochs at the last capture
  std::vector<hipEvent_t> ev;        // [0] fork, [1..n-1] joins
  hipGraphExec_t exec = nullptr;
  std::string err;
};

static int group_fail(qhp_group* g, int code, const std::string& msg) {
  g->err = msg;
  return code;
}

static void group_free(qhp_group* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  g->exec = nullptr;
  for (hipEvent_t e : g->ev)
    if (e) (void)hipEventDestroy(e);
  g->ev.clear();
}

extern "C" int qhp_group_create(qhp_ctx* const* members, int32_t n, qhp_group** out) {
  if (!out) return QHP_EINVAL;
  *out = nullptr;
  if (!members || n < 1) return QHP_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!members[i]) return QHP_EINVAL;
    for (int j = 0; j < i; ++j)
      if (members[j] == members[i]) return QHP_EINVAL;
    if (members[i]->p.thermostat != QHP_TRPMD) return QHP_EUNSUPPORTED;
  }
  qhp_group* g = new (std::nothrow) qhp_group();
  if (!g) return QHP_ENOMEM;
  g->m.assign(members, members + n);
  g->epoch.assign(n, -1);
  g->ev.assign(n, nullptr);
  for (int i = 0; i < n; ++i)
    if (hipEventCreateWithFlags(&g->ev[i], hipEventDisableTiming) != hipSuccess) {
      group_free(g);
      delete g;
      return QHP_EDEVICE;
    }
  *out = g;
  return QHP_OK;
}

extern "C" int qhp_group_destroy(qhp_group* g) {
  if (!g) return QHP_EINVAL;
  group_free(g);
  delete g;
  return QHP_OK;
}

extern "C" const char* qhp_group_last_error(qhp_group* g) { return g ? g->err.c_str() : "null group"; }

// Copy every node of a captured step graph (kernel, memcpy and empty nodes; anything else
// is refused) into `dst` with the same edges, so that the copies form a branch of `dst`
// with no dependence on its other nodes.
static hipError_t graph_append(hipGraph_t dst, hipGraph_t src) {
  size_t nn = 0, ne = 0;
  hipError_t e = hipGraphGetNodes(src, nullptr, &nn);
  if (e == hipSuccess) e = hipGraphGetEdges(src, nullptr, nullptr, &ne);
  if (e != hipSuccess) return e;
  std::vector<hipGraphNode_t> nodes(nn), from(ne), to(ne), copy(nn, nullptr);
  if (nn) e = hipGraphGetNodes(src, nodes.data(), &nn);
  if (e == hipSuccess && ne) e = hipGraphGetEdges(src, from.data(), to.data(), &ne);
  if (e != hipSuccess) return e;
  std::unordered_map<hipGraphNode_t, size_t> index;
  for (size_t k = 0; k < nn; ++k) index[nodes[k]] = k;
  std::vector<std::vector<size_t>> deps(nn);
  for (size_t k = 0; k < ne; ++k) deps[index.at(to[k])].push_back(index.at(from[k]));
  // nodes in an order where every node follows its dependencies
  std::vector<int> state(nn, 0);
  std::vector<size_t> order;
  order.reserve(nn);
  for (size_t r = 0; r < nn; ++r) {
    if (state[r]) continue;
    std::vector<std::pair<size_t, size_t>> st{{r, 0}};
    state[r] = 1;
    while (!st.empty()) {
      auto& [v, i] = st.back();
      if (i < deps[v].size()) {
        const size_t u = deps[v][i++];
        if (state[u] == 1) return hipErrorInvalidValue;   // not acyclic
        if (!state[u]) { state[u] = 1; st.push_back({u, 0}); }
      } else {
        state[v] = 2;
        order.push_back(v);
        st.pop_back();
      }
    }
  }
  for (size_t v : order) {
    std::vector<hipGraphNode_t> d;
    for (size_t u : deps[v]) d.push_back(copy[u]);
    hipGraphNodeType type;
    e = hipGraphNodeGetType(nodes[v], &type);
    if (e != hipSuccess) return e;
    if (type == hipGraphNodeTypeKernel) {
      hipKernelNodeParams kp;
      e = hipGraphKernelNodeGetParams(nodes[v], &kp);
      if (e == hipSuccess) e = hipGraphAddKernelNode(&copy[v], dst, d.data(), d.size(), &kp);
    } else if (type == hipGraphNodeTypeMemcpy) {
      hipMemcpy3DParms mp;
      e = hipGraphMemcpyNodeGetParams(nodes[v], &mp);
      if (e == hipSuccess) e = hipGraphAddMemcpyNode(&copy[v], dst, d.data(), d.size(), &mp);
    } else if (type == hipGraphNodeTypeEmpty) {
      e = hipGraphAddEmptyNode(&copy[v], dst, d.data(), d.size());
    } else {
      return hipErrorNotSupported;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One step of every member as one graph: each member's step is captured on its own stream
// (the member's stream is the origin of that capture) and its nodes are copied into the
// group graph with their edges, so that the members form independent branches of one flat
// graph; no capture is nested inside another. The members' forces stay on their own
// stream: with each member's SPME work as a further branch, the 16-window group stepped
// 1.83 ms instead of 1.21 ms (copies of the nodes, not child-graph nodes: those ran the
// members one after another, 3.06 ms).
static int group_capture(qhp_group* g) {
  const int n = (int)g->m.size();
  hipGraph_t graph = nullptr;
  hipError_t e = hipGraphCreate(&graph, 0);
  if (e != hipSuccess) return group_fail(g, QHP_EDEVICE, std::string("graph create: ") + hipGetErrorString(e));
  for (int i = 0; i < n; ++i) {
    qhp_ctx* c = g->m[i];
    hipGraph_t gi = nullptr;
    e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    int r = QHP_OK;
    if (e == hipSuccess) {
      c->serial_forces = true;
      r = one_step(c, false);
      c->serial_forces = false;
      e = hipStreamEndCapture(c->stream, &gi);
    }
    if (!r && e == hipSuccess) e = graph_append(graph, gi);
    if (gi) (void)hipGraphDestroy(gi);
    if (r || e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      if (r) return group_fail(g, r, "member " + std::to_string(i) + ": " + c->err);
      return group_fail(g, QHP_EDEVICE, "member " + std::to_string(i) + " capture: " + hipGetErrorString(e));
    }
  }
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g->exec = nullptr;
    return group_fail(g, QHP_EDEVICE, std::string("group instantiate: ") + hipGetErrorString(e));
  }
  for (int i = 0; i < n; ++i) g->epoch[i] = g->m[i]->graph_epoch;
  return QHP_OK;
}

extern "C" int qhp_group_step(qhp_group* g, int32_t nsteps) {
  if (!g) return QHP_EINVAL;
  if (nsteps < 0) return group_fail(g, QHP_EINVAL, "nsteps must be >= 0");
  const int n = (int)g->m.size();
  for (int i = 0; i < n; ++i) {
    qhp_ctx* c = g->m[i];
    if (!c->have_state) return group_fail(g, QHP_EINVAL, "member " + std::to_string(i) + " has no state");
    if (!c->use_graph) return group_fail(g, QHP_EINVAL, "members need use_graph = 1");
    if (c->prof_which != QHP_PROF_OFF) return group_fail(g, QHP_EINVAL, "members must not be profiling");
  }
  if (nsteps == 0) return QHP_OK;
  // if any member's rows can overflow, every member keeps its starting state: a repeat
  // restarts all of them
  bool guard = false;
  for (int i = 0; i < n; ++i) guard = guard || g->m[i]->cap < g->m[i]->N;
  std::vector<int64_t> step0(n);
  for (int i = 0; i < n; ++i) {
    qhp_ctx* c = g->m[i];
    step0[i] = c->step;
    if (guard) {
      int r = snapshot(c, true);
      if (r) return group_fail(g, r, "member " + std::to_string(i) + ": " + c->err);
    }
  }
  for (int attempt = 0;; ++attempt) {
    for (int i = 0; i < n; ++i)
      if (g->epoch[i] != g->m[i]->graph_epoch && g->exec) {
        (void)hipGraphExecDestroy(g->exec);
        g->exec = nullptr;
      }
    // the members' own queued work must be done before the origin stream runs the graph
    for (int i = 1; i < n; ++i) {
      hipError_t e = hipEventRecord(g->ev[i], g->m[i]->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(g->m[0]->stream, g->ev[i], 0);
      if (e != hipSuccess) return group_fail(g, QHP_EDEVICE, hipGetErrorString(e));
    }
    if (!g->exec) {
      int r = group_capture(g);
      if (r) return r;
    }
    for (int s = 0; s < nsteps; ++s) {
      hipError_t e = hipGraphLaunch(g->exec, g->m[0]->stream);
      if (e != hipSuccess) return group_fail(g, QHP_EDEVICE, std::string("group launch: ") + hipGetErrorString(e));
      for (int i = 0; i < n; ++i) g->m[i]->step += g->m[i]->nalt;
    }
    // later work queued on a member's own stream follows the group's steps
    hipError_t e = hipEventRecord(g->ev[0], g->m[0]->stream);
    for (int i = 1; i < n && e == hipSuccess; ++i) e = hipStreamWaitEvent(g->m[i]->stream, g->ev[0], 0);
    if (e != hipSuccess) return group_fail(g, QHP_EDEVICE, hipGetErrorString(e));
    bool again = false;
    std::vector<NlCtrl> h(n);
    for (int i = 0; i < n; ++i) {
      int r = read_ctrl(g->m[i], &h[i]);
      if (r) return group_fail(g, r, "member " + std::to_string(i) + ": " + g->m[i]->err);
      if (h[i].overflow && guard && attempt < 16) again = true;
    }
    if (!again) {
      for (int i = 0; i < n; ++i) {
        int r = ctrl_error(g->m[i], h[i]);
        if (r) return group_fail(g, r, "member " + std::to_string(i) + ": " + g->m[i]->err);
      }
      return QHP_OK;
    }
    // a member's list build ran out of row space: every member back to its starting
    // state, larger rows where needed, the group step recaptured and repeated
    for (int i = 0; i < n; ++i) {
      qhp_ctx* c = g->m[i];
      int r = snapshot(c, false);
      c->step = step0[i];
      if (!r && h[i].overflow) r = grow_list(c, h[i].max_count);
      if (r) return group_fail(g, r, "member " + std::to_string(i) + ": " + c->err);
    }
  }
}
