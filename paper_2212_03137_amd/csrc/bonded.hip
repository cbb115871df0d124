// Intramolecular terms of the flexible 3-site water and the Ewald corrections that do not
// involve other molecules: harmonic O-H bonds, harmonic H-O-H angle, and removal of the
// screened interaction of the three excluded intramolecular pairs,
// -C q_a q_b erf(alpha r) / r, that the reciprocal sum contains. This kernel *initialises*
// grad V of every bead of its bead set; the pair and SPME kernels add to it. Under
// multiple time stepping the bonds and angles (V_f) and the exclusion correction (with
// the rest of V_s) run on different bead sets: TERMS selects which.
// Lane (w, b): water w at bead b; 256 / P waters per block.
#include "qhp_internal.h"

namespace {

constexpr int NT = 256;

struct BondArgs {
  int N, NW;
  const double* x; double* g;
  const double* charge;
  double L[3], invL[3];
  double r0, kb, th0, kth, alpha, coulomb;
  double* energy;
  double* dq;              // parameter gradients: d/d charge (exclusion and self terms)
};

template <int P>
QHP_DEV void reduce_energy_by_bead(double* sred, int tid, double v, double* dst) {
  constexpr int AT = NT / P;
  sred[tid] = v;
  __syncthreads();
  for (int s = AT / 2; s > 0; s >>= 1) {
    if (tid / P < s) sred[tid] += sred[tid + s * P];
    __syncthreads();
  }
  if (tid < P) atomicAdd(dst + tid * QHP_NTERMS, sred[tid]);
  __syncthreads();
}

// PG: also add the charge derivatives of the exclusion correction (-C q_b erf(alpha r)/r
// for atom a of each excluded pair, and symmetrically) and of the self term
// (-2 C alpha / sqrt(pi) q per bead), summed over the beads of each water.
template <int P, bool ENERGY, int TERMS, bool PG = false>
__global__ __launch_bounds__(NT) void k_bonded(BondArgs A) {
  constexpr int AT = NT / P;
  __shared__ double sred[NT];
  const int tid = threadIdx.x, b = tid % P;
  const int w = blockIdx.x * AT + tid / P;
  double eb = 0, ea = 0, ex = 0;
  double pq[3] = {0.0, 0.0, 0.0};
  if (w < A.NW) {
    const int N = A.N;
    double X[3][3], G[3][3];
    for (int k = 0; k < 3; ++k)
      for (int d = 0; d < 3; ++d) {
        X[k][d] = A.x[(d * N + 3 * w + k) * P + b];
        G[k][d] = 0.0;
      }
    double u[2][3], r[2];
    if (TERMS & QHP_TERMS_BONDED) {
    for (int h = 0; h < 2; ++h) {
      double dd[3];
      for (int d = 0; d < 3; ++d) {
        dd[d] = X[h + 1][d] - X[0][d];
        dd[d] -= A.L[d] * rint(dd[d] * A.invL[d]);
      }
      r[h] = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
      const double dr = r[h] - A.r0;
      if (ENERGY) eb += 0.5 * A.kb * dr * dr;
      const double s = A.kb * dr / r[h];
      for (int d = 0; d < 3; ++d) {
        u[h][d] = dd[d] / r[h];
        G[h + 1][d] += s * dd[d];
        G[0][d] -= s * dd[d];
      }
    }
    double cs = u[0][0] * u[1][0] + u[0][1] * u[1][1] + u[0][2] * u[1][2];
    cs = fmin(1.0, fmax(-1.0, cs));
    const double th = acos(cs), sn = sqrt(1.0 - cs * cs);
    const double dth = th - A.th0;
    if (ENERGY) ea = 0.5 * A.kth * dth * dth;
    const double de = A.kth * dth;
    for (int d = 0; d < 3; ++d) {
      const double g1 = -de / (r[0] * sn) * (u[1][d] - cs * u[0][d]);
      const double g2 = -de / (r[1] * sn) * (u[0][d] - cs * u[1][d]);
      G[1][d] += g1;
      G[2][d] += g2;
      G[0][d] -= g1 + g2;
    }
    }
    if (TERMS & QHP_TERMS_EXCL) {
    const double c2a = 2.0 * A.alpha / sqrt(M_PI);
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    for (int e = 0; e < 3; ++e) {
      double dd[3];
      for (int d = 0; d < 3; ++d) {
        dd[d] = X[pb[e]][d] - X[pa[e]][d];
        dd[d] -= A.L[d] * rint(dd[d] * A.invL[d]);
      }
      const double r2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
      const double rr = sqrt(r2);
      const double qq = A.coulomb * A.charge[3 * w + pa[e]] * A.charge[3 * w + pb[e]];
      const double erfv = erf(A.alpha * rr);
      if (ENERGY) ex += -qq * erfv / rr;
      if (PG) {
        pq[pa[e]] += -A.coulomb * A.charge[3 * w + pb[e]] * erfv / rr;
        pq[pb[e]] += -A.coulomb * A.charge[3 * w + pa[e]] * erfv / rr;
      }
      const double dEdr = -qq * (c2a * exp(-A.alpha * A.alpha * r2) / rr - erfv / r2);
      const double s = dEdr / rr;
      for (int d = 0; d < 3; ++d) {
        G[pb[e]][d] += s * dd[d];
        G[pa[e]][d] -= s * dd[d];
      }
    }
    }
    for (int k = 0; k < 3; ++k)
      for (int d = 0; d < 3; ++d) A.g[(d * N + 3 * w + k) * P + b] = G[k][d];
    if (PG)
      for (int k = 0; k < 3; ++k) pq[k] += -2.0 * A.coulomb * A.alpha / sqrt(M_PI) * A.charge[3 * w + k];
  }
  if (PG) {                          // sum over the P bead lanes of the water
    for (int o = 1; o < P; o <<= 1)
      for (int k = 0; k < 3; ++k) pq[k] += __shfl_xor(pq[k], o);
    if (w < A.NW && b == 0)
      for (int k = 0; k < 3; ++k) A.dq[3 * w + k] += pq[k];
  }
  if (ENERGY && (TERMS & QHP_TERMS_BONDED)) {
    reduce_energy_by_bead<P>(sred, tid, eb, A.energy + QHP_E_BOND);
    reduce_energy_by_bead<P>(sred, tid, ea, A.energy + QHP_E_ANGLE);
  }
  if (ENERGY && (TERMS & QHP_TERMS_EXCL)) reduce_energy_by_bead<P>(sred, tid, ex, A.energy + QHP_E_COUL_EXCL);
}

// zero [rows][NTERMS] and put the self term on the first self_rows rows
// ---- Hessian-vector products of the intramolecular terms by forward differentiation ----
// A dual number (v, d) carries a value and its derivative along the direction u; running
// the gradient of the bond, angle and exclusion terms on dual positions x + eps u gives
// the gradient's derivative along u, H u, exactly (no truncation).
struct Dual {
  double v, d;
};
QHP_DEV Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
QHP_DEV Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
QHP_DEV Dual operator-(Dual a) { return {-a.v, -a.d}; }
QHP_DEV Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
QHP_DEV Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
QHP_DEV Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
QHP_DEV Dual dsqrt(Dual a) {
  const double s = sqrt(a.v);
  return {s, 0.5 * a.d / s};
}
QHP_DEV Dual dacos(Dual a) { return {acos(a.v), -a.d / sqrt(1.0 - a.v * a.v)}; }
QHP_DEV Dual derf(Dual a) { return {erf(a.v), a.d * (2.0 / sqrt(M_PI)) * exp(-a.v * a.v)}; }
QHP_DEV Dual dexp(Dual a) {
  const double e = exp(a.v);
  return {e, a.d * e};
}

// With A.dq set, also add the exclusion term's part of d(u . grad E)/dq: the derivative
// along u of -C q_b erf(alpha r)/r (and symmetrically), summed over the beads.
template <int P>
__global__ __launch_bounds__(NT) void k_bonded_hvp(BondArgs A, const double* u, double* hu) {
  constexpr int AT = NT / P;
  const int tid = threadIdx.x, b = tid % P;
  const int w = blockIdx.x * AT + tid / P;
  double mq[3] = {0.0, 0.0, 0.0};
  if (w < A.NW) {
  const int N = A.N;
  Dual X[3][3], G[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) {
      const size_t i = (size_t)(d * N + 3 * w + k) * P + b;
      X[k][d] = {A.x[i], u[i]};
      G[k][d] = {0.0, 0.0};
    }
  auto sep = [&](int a0, int a1, Dual* dd) {   // minimum-image difference X[a1] - X[a0]
    for (int d = 0; d < 3; ++d) {
      dd[d] = X[a1][d] - X[a0][d];
      dd[d].v -= A.L[d] * rint(dd[d].v * A.invL[d]);   // the shift is locally constant
    }
  };
  Dual uu[2][3], r[2];
  for (int h = 0; h < 2; ++h) {                     // O-H bonds
    Dual dd[3];
    sep(0, h + 1, dd);
    r[h] = dsqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
    const Dual s = A.kb * ((r[h] - Dual{A.r0, 0.0}) / r[h]);
    for (int d = 0; d < 3; ++d) {
      uu[h][d] = dd[d] / r[h];
      G[h + 1][d] = G[h + 1][d] + s * dd[d];
      G[0][d] = G[0][d] - s * dd[d];
    }
  }
  {                                                 // H-O-H angle
    Dual cs = uu[0][0] * uu[1][0] + uu[0][1] * uu[1][1] + uu[0][2] * uu[1][2];
    const Dual th = dacos(cs), sn = dsqrt(Dual{1.0, 0.0} - cs * cs);
    const Dual de = A.kth * (th - Dual{A.th0, 0.0});
    for (int d = 0; d < 3; ++d) {
      const Dual g1 = -(de / (r[0] * sn)) * (uu[1][d] - cs * uu[0][d]);
      const Dual g2 = -(de / (r[1] * sn)) * (uu[0][d] - cs * uu[1][d]);
      G[1][d] = G[1][d] + g1;
      G[2][d] = G[2][d] + g2;
      G[0][d] = G[0][d] - (g1 + g2);
    }
  }
  const double c2a = 2.0 * A.alpha / sqrt(M_PI);
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int e = 0; e < 3; ++e) {                     // exclusion correction
    Dual dd[3];
    sep(pa[e], pb[e], dd);
    const Dual r2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
    const Dual rr = dsqrt(r2);
    const double qq = A.coulomb * A.charge[3 * w + pa[e]] * A.charge[3 * w + pb[e]];
    const Dual erfv = derf(A.alpha * rr);
    const Dual dEdr = (-qq) * (c2a * (dexp((-A.alpha * A.alpha) * r2) / rr) - erfv / r2);
    const Dual s = dEdr / rr;
    for (int d = 0; d < 3; ++d) {
      G[pb[e]][d] = G[pb[e]][d] + s * dd[d];
      G[pa[e]][d] = G[pa[e]][d] - s * dd[d];
    }
    const double dh = (erfv / rr).d;                 // d/dh of erf(alpha r)/r along u
    mq[pa[e]] += -A.coulomb * A.charge[3 * w + pb[e]] * dh;
    mq[pb[e]] += -A.coulomb * A.charge[3 * w + pa[e]] * dh;
  }
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) hu[(size_t)(d * N + 3 * w + k) * P + b] = G[k][d].d;
  }
  if (A.dq) {                          // sum over the P bead lanes of the water
    for (int o = 1; o < P; o <<= 1)
      for (int k = 0; k < 3; ++k) mq[k] += __shfl_xor(mq[k], o);
    if (w < A.NW && b == 0)
      for (int k = 0; k < 3; ++k) A.dq[3 * w + k] += mq[k];
  }
}

__global__ void k_energy_init(double* energy, int rows, int self_rows, double self) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows * QHP_NTERMS)
    energy[i] = (i % QHP_NTERMS == QHP_E_COUL_SELF && i / QHP_NTERMS < self_rows) ? self : 0.0;
}

// zero the terms evaluated on the contracted beads (all but bonds and angles) in rows
// [r0, r1) of the energy table
__global__ void k_clear_slow_energy(double* energy, int r0, int r1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = r0 + i / QHP_NTERMS, t = i % QHP_NTERMS;
  if (row < r1 && t != QHP_E_BOND && t != QHP_E_ANGLE) energy[(size_t)row * QHP_NTERMS + t] = 0.0;
}

__global__ void k_zero(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace

#define QHP_SWITCH_P(P, CALL)                          \
  switch (P) {                                         \
    case 1: { constexpr int PP = 1; CALL; } break;     \
    case 2: { constexpr int PP = 2; CALL; } break;     \
    case 4: { constexpr int PP = 4; CALL; } break;     \
    case 8: { constexpr int PP = 8; CALL; } break;     \
    case 16: { constexpr int PP = 16; CALL; } break;   \
    case 32: { constexpr int PP = 32; CALL; } break;   \
    case 64: { constexpr int PP = 64; CALL; } break;   \
    default: return hipErrorInvalidValue;              \
  }

// Test-only harmonic tether of every atom at every bead: grad V += k (x - a), and with
// energies k/2 |x - a|^2 added to the bead's bond term. x, g: [3][N][P] (one bead of the
// plain layout: P = 1 on the bead's slices); a: [3][N].
__global__ __launch_bounds__(256) void k_tether(int N, int P, const double* x, double* g,
                                                const double* anchor, double k,
                                                double* energy) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * P) return;
  const int a = t / P, b = t % P;
  double e = 0.0;
  for (int d = 0; d < 3; ++d) {
    const size_t i = ((size_t)d * N + a) * P + b;
    const double dd = x[i] - anchor[(size_t)d * N + a];
    g[i] += k * dd;
    e += dd * dd;
  }
  if (energy) atomicAdd(energy + (size_t)b * QHP_NTERMS + QHP_E_BOND, 0.5 * k * e);
}

hipError_t launch_tether(qhp_ctx* c, bool energy, int bead, const BeadSet* bs) {
  if (!(c->tether_k > 0)) return hipSuccess;
  const int N = c->N;
  const bool plain = bead >= 0;
  const BeadSet B = bs ? *bs : full_beads(c);
  const int P = plain ? 1 : B.P;
  const double* x = plain ? c->x + (size_t)bead * 3 * N : B.x;
  double* g = plain ? c->g + (size_t)bead * 3 * N : B.g;
  double* e = energy ? (plain ? c->energy + (size_t)bead * QHP_NTERMS : B.energy) : nullptr;
  const unsigned nb = (unsigned)(((size_t)N * P + 255) / 256);
  hipLaunchKernelGGL(k_tether, nb, 256, 0, c->stream, N, P, x, g, c->d_anchor, c->tether_k, e);
  return hipGetLastError();
}

hipError_t launch_bonded(qhp_ctx* c, bool energy, int bead, const BeadSet* bs) {
  BondArgs A;
  const int N = c->N;
  const bool plain = bead >= 0;
  const BeadSet B = bs ? *bs : full_beads(c);
  A.N = N; A.NW = c->NW;
  A.x = plain ? c->x + (size_t)bead * 3 * N : B.x;
  A.g = plain ? c->g + (size_t)bead * 3 * N : B.g;
  A.charge = c->d_charge;
  for (int d = 0; d < 3; ++d) { A.L[d] = c->p.box[d]; A.invL[d] = 1.0 / c->p.box[d]; }
  A.r0 = c->p.bond_r0; A.kb = c->p.bond_k; A.th0 = c->p.angle_theta0; A.kth = c->p.angle_k;
  A.alpha = c->p.ewald_alpha; A.coulomb = c->p.coulomb;
  A.energy = (plain ? c->energy : B.energy) + (plain ? (size_t)bead * QHP_NTERMS : 0);
  A.dq = c->pg_dq;
  const int P = plain ? 1 : B.P;
  const int terms = plain ? QHP_TERMS_ALL : B.terms;
  // the launch that carries the bonds initialises the energy rows of the whole step; under
  // contraction the self term belongs to the contracted beads only
  if (energy && bead <= 0 && (terms & QHP_TERMS_BONDED)) {
    const int rows = plain ? c->P : B.P;
    const int self_rows = terms == QHP_TERMS_ALL ? (plain ? c->Pb : B.P) : c->Psb;
    hipLaunchKernelGGL(k_energy_init, (rows * QHP_NTERMS + 511) / 512, 512, 0, c->stream,
                       plain ? c->energy : B.energy, rows, self_rows, c->self_energy);
  }
  const unsigned nb = (unsigned)((c->NW + NT / P - 1) / (NT / P));
#define BONDED_CALL(TT)                                                                           \
  QHP_SWITCH_P(P, if (energy) hipLaunchKernelGGL((k_bonded<PP, true, TT>), nb, NT, 0, c->stream, A); \
               else hipLaunchKernelGGL((k_bonded<PP, false, TT>), nb, NT, 0, c->stream, A))
  if (!plain && B.pgrad && terms == QHP_TERMS_ALL) {
    QHP_SWITCH_P(P, hipLaunchKernelGGL((k_bonded<PP, false, QHP_TERMS_ALL, true>), nb, NT, 0, c->stream, A));
  } else if (terms == QHP_TERMS_BONDED) { BONDED_CALL(QHP_TERMS_BONDED); }
  else if (terms == QHP_TERMS_EXCL) { BONDED_CALL(QHP_TERMS_EXCL); }
  else { BONDED_CALL(QHP_TERMS_ALL); }
#undef BONDED_CALL
  return hipGetLastError();
}

hipError_t launch_bonded_hvp(qhp_ctx* c, const double* u, double* hu, bool mix) {
  BondArgs A;
  A.N = c->N; A.NW = c->NW; A.x = c->x; A.g = nullptr; A.charge = c->d_charge;
  for (int d = 0; d < 3; ++d) { A.L[d] = c->p.box[d]; A.invL[d] = 1.0 / c->p.box[d]; }
  A.r0 = c->p.bond_r0; A.kb = c->p.bond_k; A.th0 = c->p.angle_theta0; A.kth = c->p.angle_k;
  A.alpha = c->p.ewald_alpha; A.coulomb = c->p.coulomb; A.energy = nullptr;
  A.dq = mix ? c->pg_dq : nullptr;
  const int P = c->P;
  const unsigned nb = (unsigned)((c->NW + NT / P - 1) / (NT / P));
  QHP_SWITCH_P(P, hipLaunchKernelGGL((k_bonded_hvp<PP>), nb, NT, 0, c->stream, A, u, hu));
  return hipGetLastError();
}

hipError_t launch_clear_slow_energy(qhp_ctx* c, int r0, int r1) {
  const int n = (r1 - r0) * QHP_NTERMS;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_slow_energy, (n + 255) / 256, 256, 0, c->stream, c->energy, r0, r1);
  return hipGetLastError();
}

hipError_t launch_zero(qhp_ctx* c, void* ptr, size_t bytes) {
  const size_t n = bytes / sizeof(double);
  const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero, nb, 256, 0, c->stream, (double*)ptr, n);
  return hipGetLastError();
}
