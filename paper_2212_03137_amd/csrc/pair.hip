// Real-space part of the bead potential: Ewald-screened Coulomb C q_i q_j erfc(alpha r)/r
// and Lennard-Jones 4 eps ((s/r)^12 - (s/r)^6) over centroid-list pairs whose *bead*
// distance is below the cutoff (plain truncation), for every bead at once.
//
// Lane layout: a 64-lane wavefront covers 64/P atoms i and all P beads; lane (i, b) walks
// the full neighbour list of atom i (each j index is shared by the P lanes of i) and owns
// grad_i at bead b, so no atomics are needed. Each pair is evaluated from both ends.
//
// FP32-pair mode: the displacement is formed in FP64 as (wrapped centroid difference +
// stored image shift), rounded once to FP32, and the per-bead offsets from the centroids
// (kept in FP32) are added; distances, erfc/exp and the force scalar are FP32; forces are
// summed in FP32 over chunks of 32 neighbours and then in FP64; energies in FP64.
// The stored shift is the bead's minimum image for every pair within the cutoff whenever
// 2 (rc + skin) < L (see the rebuild rule in the neighbour list); otherwise the FP64 path
// is used. The FP64 path takes each bead's own minimum image.
#include "qhp_internal.h"

namespace {

constexpr int NT = 256;

struct PairArgs {
  int N, cap;
  const double* x;        // [3][N][P] (or one bead's [3][N] with P = 1)
  double* g;
  const double4* cwrap;
  const float4* xf;
  const int* nbr; const int* nnbr;
  const double* charge; const int* type;
  double L[3], invL[3];
  double rc2, alpha, coulomb;
  double lj_s6[QHP_MAX_TYPES * QHP_MAX_TYPES];
  double lj_e4[QHP_MAX_TYPES * QHP_MAX_TYPES];
  int ntypes;
  double* energy;         // [P][NTERMS] (plain: the bead's row)
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

template <int P, bool ENERGY>
__global__ __launch_bounds__(NT) void k_pair64(PairArgs A) {
  constexpr int AT = NT / P;
  __shared__ double sred[NT];
  const int tid = threadIdx.x, b = tid % P;
  const int i = blockIdx.x * AT + tid / P;
  const bool live = i < A.N;
  double gx = 0, gy = 0, gz = 0, ec = 0, elj = 0;
  if (live) {
    const int N = A.N;
    const double xi = A.x[(0 * N + i) * P + b], yi = A.x[(1 * N + i) * P + b],
                 zi = A.x[(2 * N + i) * P + b];
    const double qi = A.coulomb * A.charge[i];
    const int ti = A.type[i];
    const double c2a = 2.0 * A.alpha / sqrt(M_PI);
    const int nn = A.nnbr[i];
    for (int k = 0; k < nn; ++k) {
      const unsigned e = (unsigned)A.nbr[(size_t)k * N + i];
      const int j = e & 0x3FFFFFF;
      double dx = A.x[(0 * N + j) * P + b] - xi;
      double dy = A.x[(1 * N + j) * P + b] - yi;
      double dz = A.x[(2 * N + j) * P + b] - zi;
      dx -= A.L[0] * rint(dx * A.invL[0]);
      dy -= A.L[1] * rint(dy * A.invL[1]);
      dz -= A.L[2] * rint(dz * A.invL[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < A.rc2) {
        const double r = sqrt(r2), ir = 1.0 / r, ir2 = ir * ir;
        const double qq = qi * A.charge[j];
        const double erfcv = erfc(A.alpha * r);
        double s = qq * (erfcv * ir + c2a * exp(-A.alpha * A.alpha * r2)) * ir2;
        if (ENERGY) ec += qq * erfcv * ir;
        const int tp = ti * A.ntypes + A.type[j];
        const double e4 = A.lj_e4[tp];
        if (e4 != 0.0) {
          const double s6 = A.lj_s6[tp] * ir2 * ir2 * ir2;
          s += e4 * (12.0 * s6 * s6 - 6.0 * s6) * ir2;
          if (ENERGY) elj += e4 * (s6 * s6 - s6);
        }
        gx += s * dx; gy += s * dy; gz += s * dz;
      }
    }
    A.g[(0 * N + i) * P + b] += gx;
    A.g[(1 * N + i) * P + b] += gy;
    A.g[(2 * N + i) * P + b] += gz;
  }
  if (ENERGY) {
    reduce_energy_by_bead<P>(sred, tid, 0.5 * ec, A.energy + QHP_E_COUL_REAL);
    reduce_energy_by_bead<P>(sred, tid, 0.5 * elj, A.energy + QHP_E_LJ);
  }
}

template <int P, bool ENERGY>
__global__ __launch_bounds__(NT) void k_pair32(PairArgs A) {
  constexpr int AT = NT / P;
  __shared__ double sred[NT];
  const int tid = threadIdx.x, b = tid % P;
  const int i = blockIdx.x * AT + tid / P;
  const bool live = i < A.N;
  double gx = 0, gy = 0, gz = 0, ec = 0, elj = 0;
  if (live) {
    const int N = A.N;
    const float4 oi = A.xf[(size_t)i * P + b];
    const double4 ci = A.cwrap[i];
    const float qi = (float)(A.coulomb * A.charge[i]);
    const int ti = A.type[i];
    const float alpha = (float)A.alpha, a2 = (float)(A.alpha * A.alpha);
    const float c2a = (float)(2.0 * A.alpha / sqrt(M_PI));
    const float rc2 = (float)A.rc2;
    const int nn = A.nnbr[i];
    for (int k0 = 0; k0 < nn; k0 += 32) {
      float fx = 0.f, fy = 0.f, fz = 0.f;
      const int k1 = min(nn, k0 + 32);
      for (int k = k0; k < k1; ++k) {
        const unsigned e = (unsigned)A.nbr[(size_t)k * N + i];
        const int j = e & 0x3FFFFFF;
        const double4 cj = A.cwrap[j];
        const float cx = (float)((cj.x - ci.x) + A.L[0] * (double)((int)((e >> 26) & 3) - 1));
        const float cy = (float)((cj.y - ci.y) + A.L[1] * (double)((int)((e >> 28) & 3) - 1));
        const float cz = (float)((cj.z - ci.z) + A.L[2] * (double)((int)((e >> 30) & 3) - 1));
        const float4 oj = A.xf[(size_t)j * P + b];
        const float dx = cx + (oj.x - oi.x), dy = cy + (oj.y - oi.y), dz = cz + (oj.z - oi.z);
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < rc2) {
          const float ir = rsqrtf(r2), ir2 = ir * ir;
          const float r = r2 * ir;
          const float qq = qi * oj.w;
          const float erfcv = erfcf(alpha * r);
          float s = qq * (erfcv * ir + c2a * expf(-a2 * r2)) * ir2;
          if (ENERGY) ec += (double)(qq * erfcv * ir);
          const int tp = ti * A.ntypes + A.type[j];
          const float e4 = (float)A.lj_e4[tp];
          if (e4 != 0.f) {
            const float s6 = (float)A.lj_s6[tp] * ir2 * ir2 * ir2;
            s += e4 * (12.f * s6 * s6 - 6.f * s6) * ir2;
            if (ENERGY) elj += (double)(e4 * (s6 * s6 - s6));
          }
          fx += s * dx; fy += s * dy; fz += s * dz;
        }
      }
      gx += (double)fx; gy += (double)fy; gz += (double)fz;
    }
    A.g[(0 * N + i) * P + b] += gx;
    A.g[(1 * N + i) * P + b] += gy;
    A.g[(2 * N + i) * P + b] += gz;
  }
  if (ENERGY) {
    reduce_energy_by_bead<P>(sred, tid, 0.5 * ec, A.energy + QHP_E_COUL_REAL);
    reduce_energy_by_bead<P>(sred, tid, 0.5 * elj, A.energy + QHP_E_LJ);
  }
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

hipError_t launch_pair(qhp_ctx* c, bool energy, int bead) {
  PairArgs A;
  const int N = c->N;
  A.N = N; A.cap = c->cap;
  const bool plain = bead >= 0;
  A.x = plain ? c->x + (size_t)bead * 3 * N : c->x;
  A.g = plain ? c->g + (size_t)bead * 3 * N : c->g;
  A.cwrap = c->cwrap; A.xf = c->xf; A.nbr = c->nbr; A.nnbr = c->nnbr;
  A.charge = c->d_charge; A.type = c->d_type;
  for (int d = 0; d < 3; ++d) { A.L[d] = c->p.box[d]; A.invL[d] = 1.0 / c->p.box[d]; }
  A.rc2 = c->p.cutoff * c->p.cutoff; A.alpha = c->p.ewald_alpha; A.coulomb = c->p.coulomb;
  A.ntypes = c->p.n_types;
  for (int a = 0; a < c->p.n_types; ++a)
    for (int b = 0; b < c->p.n_types; ++b) {
      const double s = 0.5 * (c->sigma[a] + c->sigma[b]);
      const double e = sqrt(c->eps[a] * c->eps[b]);
      A.lj_s6[a * A.ntypes + b] = s * s * s * s * s * s;
      A.lj_e4[a * A.ntypes + b] = 4.0 * e;
    }
  A.energy = c->energy + (plain ? (size_t)bead * QHP_NTERMS : 0);
  const int P = plain ? 1 : c->P;
  const unsigned nb = (unsigned)((N + NT / P - 1) / (NT / P));
  const double Lmin = fmin(c->p.box[0], fmin(c->p.box[1], c->p.box[2]));
  const bool minimg = !(2.0 * (c->p.cutoff + c->p.skin) < Lmin);
  const bool f32 = c->p.precision == QHP_FP32_PAIRS && !plain && !minimg;
  hipEvent_t ev = nullptr;
  prof_begin(c, QHP_PROF_PAIR, &ev);
  if (f32) {
    QHP_SWITCH_P(P, if (energy) hipLaunchKernelGGL((k_pair32<PP, true>), nb, NT, 0, c->stream, A);
                 else hipLaunchKernelGGL((k_pair32<PP, false>), nb, NT, 0, c->stream, A));
  } else {
    QHP_SWITCH_P(P, if (energy) hipLaunchKernelGGL((k_pair64<PP, true>), nb, NT, 0, c->stream, A);
                 else hipLaunchKernelGGL((k_pair64<PP, false>), nb, NT, 0, c->stream, A));
  }
  prof_end(c, QHP_PROF_PAIR, ev);
  return hipGetLastError();
}
