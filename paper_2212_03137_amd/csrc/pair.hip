// Real-space part of the bead potential: Ewald-screened Coulomb C q_i q_j erfc(alpha r)/r
// and Lennard-Jones 4 eps ((s/r)^12 - (s/r)^6) over centroid-list pairs whose *bead*
// distance is below the cutoff (plain truncation), for every bead at once.
//
// Lane layout: one wavefront per atom i. Its 64 lanes are S = 64/P neighbour slots times
// the P beads; lane (s, b) takes neighbours s, s+S, ... of atom i at bead b and owns
// grad_i at bead b, so no atomics are needed (each pair is evaluated from both ends).
// The neighbour row is consumed 64 entries at a time: lane l decodes entry l once (index,
// type, charge, FP64 centroid difference with the stored image shift) into LDS, and the
// bead lanes then read it from there, so the per-pair FP64 work is not repeated per bead.
// The decode drops pairs whose centroids are further apart than rc plus both atoms'
// largest bead-centroid distances (no bead can then be in range) and stores the pairs
// with an LJ term first, so that the LJ arithmetic runs on those pairs only. With one
// bead (64 slots, one interaction per lane per chunk) there is nothing to share: each
// lane evaluates its own decoded entry in place.
//
// FP32-pair mode: the displacement is the FP64 wrapped-centroid difference plus image
// shift, rounded once to FP32, plus the FP32 bead offsets from the centroids; distance
// and force scalar are FP32; each lane sums forces in FP32 over one chunk of neighbours,
// then in FP64; energies in FP64. The screened Coulomb kernels come from cubic tables in
// r^2; below 1 A they are evaluated directly, erfc(x) = exp(-x^2) t Q(t) with
// t = 1/(1 + p x) (Hastings' form; p and Q fitted by gen_erfc_fit.py, relative error
// 3e-8), sharing exp(-x^2) with the force term. The stored shift is the bead's minimum
// image for every pair within the cutoff whenever 2 (rc + skin) < L (neighbour-list
// rebuild rule); otherwise the FP64 path is used, which takes each bead's own minimum
// image.
//
// Blocks are remapped so that each of the 8 XCDs works on a contiguous range of atoms
// (a slab of the box in lattice order), keeping its neighbours' data in its own L2.
#include "qhp_internal.h"

namespace {

constexpr int NT = 256;
constexpr int WPB = NT / 64;      // atoms (wavefronts) per block
#ifndef QHP_PAIR_PF
#define QHP_PAIR_PF 1
#endif
#ifndef QHP_ONE_ACC
#define QHP_ONE_ACC 8
#endif

// p = 0.418649012, max relative error of exp(x^2) erfc(x) on [0, 6]: 2.94e-08
constexpr float ERFC_P = 0.418649012f;
constexpr float ERFC_Q[8] = {0.235933458f, 0.240632992f, 0.183633505f, 0.301421722f,
                             -0.189258145f, 0.502240173f, -0.351184483f, 0.0765808055f};

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
  double lj_a[QHP_MAX_TYPES * QHP_MAX_TYPES];     // soft-core alpha (1 - lambda_vdw), 0 = plain
  double lj_sig[QHP_MAX_TYPES * QHP_MAX_TYPES];   // sigma_ij (parameter gradients)
  double eps_of[QHP_MAX_TYPES];                    // epsilon of each type
  double* dq; double* deps; double* dsig;          // parameter-gradient outputs (FP64 path)
  const double* u; double* hu;                     // Hessian-vector product: direction, output
  int mix;                                         // HVP: also d(u . grad E)/d(q, eps, sigma)
  const float4* tab;      // FP32 pairs: force and energy kernel tables ([2][QHP_PAIR_TAB])
  float tab_scale;        // intervals per A^2 of r^2 (fl(r2 tab_scale) < QHP_PAIR_TAB in range)
  int tab_kmin;           // first interval the tables are used for (closer: the formula)
  int nblocks;            // logical blocks
  int pack_qt;            // centroid records carry charge, type and spread (see qhp_internal.h)
  const NlCtrl* ctrl;     // max_db: largest bead-centroid distance this step
  double* energy;         // [P][NTERMS] (plain: the bead's row)
};

QHP_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// physical block -> logical block so that XCD k (blocks k, k+8, ...) gets a contiguous range
QHP_DEV int xcd_block(int bid, int nphys) { return (bid & 7) * (nphys >> 3) + (bid >> 3); }

// sum over the S slots of a wavefront; lanes 0..P-1 end up with their bead's total
template <int P>
QHP_DEV double slot_sum(double v) {
#pragma unroll
  for (int o = P; o < 64; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

template <int P, bool ENERGY>
QHP_DEV void flush(const PairArgs& A, int i, int lane, double gx, double gy, double gz,
                   double ec, double elj) {
  gx = slot_sum<P>(gx); gy = slot_sum<P>(gy); gz = slot_sum<P>(gz);
  if (ENERGY) { ec = slot_sum<P>(ec); elj = slot_sum<P>(elj); }
  if (lane < P) {
    const int N = A.N;
    A.g[(0 * (size_t)N + i) * P + lane] += gx;
    A.g[(1 * (size_t)N + i) * P + lane] += gy;
    A.g[(2 * (size_t)N + i) * P + lane] += gz;
    if (ENERGY) {
      atomicAdd(A.energy + lane * QHP_NTERMS + QHP_E_COUL_REAL, 0.5 * ec);
      atomicAdd(A.energy + lane * QHP_NTERMS + QHP_E_LJ, 0.5 * elj);
    }
  }
}

// PG: also accumulate the derivatives of the summed bead energies with respect to the
// charge of atom i (C q_j erfc(alpha r)/r per in-range pair, visited from i's end) and to
// the LJ epsilon and sigma of i's type (the i-side halves of d e_ij and d s_ij; the j side
// is added when the pair is visited from j).
// HVP: instead of the gradient, add M (u_i - u_j) per in-range pair to hu_i, with
// M = phi'' r^ r^T + (phi'/r)(I - r^ r^T) the pair's Hessian block (phi the screened
// Coulomb plus LJ pair potential of r).
// SOFT: pairs with lj_a != 0 take the soft-core LJ form. With s6 = (sigma/r)^6 and
// d = 1 + a s6, the soft-core term e4 [1/D^2 - 1/D] (D = a + (r/sigma)^6, e4 = 4 eps
// lambda) is e4 (u^2 - u) with u = s6 / d, and -(dE/dr)/r = 6 e4 u (2u - 1) / (d r^2);
// a = 0 gives plain LJ.
// F32 (parameter gradients and Hessian-vector products with FP32 pairs): the displacement
// and r^2 stay FP64; r, 1/r, erfc(alpha r) (the Hastings form of the FP32 force kernel) and
// exp(-alpha^2 r^2) are FP32 values; every product and sum after them is FP64.
template <int P, bool ENERGY, bool PG = false, bool HVP = false, bool SOFT = false,
          bool F32 = false>
__global__ __launch_bounds__(NT) void k_pair64(PairArgs A) {
  static_assert(!SOFT || (!PG && !HVP), "soft-core pairs have forces and energies only");
  static_assert(!F32 || PG || HVP, "FP32 pair forces have their own kernel");
  constexpr int S = 64 / P;
  __shared__ int sj[WPB][64];
  __shared__ double sq[WPB][64];
  __shared__ double2 slj[WPB][64];
  __shared__ double ssa[SOFT ? WPB : 1][SOFT ? 64 : 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, s = lane / P, b = lane % P;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int i = lb * WPB + wv;
  if (lb >= A.nblocks || i >= A.N) return;       // whole wavefront leaves together
  const int N = A.N;
  const double xi = A.x[(0 * (size_t)N + i) * P + b], yi = A.x[(1 * (size_t)N + i) * P + b],
               zi = A.x[(2 * (size_t)N + i) * P + b];
  const double qi = A.coulomb * A.charge[i];
  const int ti = A.type[i];
  const double c2a = 2.0 * A.alpha / sqrt(M_PI);
  const int nn = A.nnbr[i];
  const int* row = A.nbr + (size_t)i * A.cap;
  double gx = 0, gy = 0, gz = 0, ec = 0, elj = 0;
  double pq = 0, pe = 0, ps = 0;                  // parameter gradients (PG)
  double uix = 0, uiy = 0, uiz = 0;
  if (HVP) {
    uix = A.u[(0 * (size_t)N + i) * P + b];
    uiy = A.u[(1 * (size_t)N + i) * P + b];
    uiz = A.u[(2 * (size_t)N + i) * P + b];
  }
  __shared__ double ssig[PG || HVP ? WPB : 1][PG || HVP ? 64 : 1];
  const double half_over_eps = (PG || HVP) && A.eps_of[ti] > 0.0 ? 0.5 / A.eps_of[ti] : 0.0;
  const bool mix = HVP && A.mix;
  for (int k0 = 0; k0 < nn; k0 += 64) {
    const int cnt = min(64, nn - k0);
    if (lane < cnt) {
      const int j = row[k0 + lane] & 0x3FFFFFF;
      sj[wv][lane] = j;
      sq[wv][lane] = qi * A.charge[j];
      const int tp = ti * A.ntypes + A.type[j];
      slj[wv][lane] = make_double2(A.lj_e4[tp], A.lj_s6[tp]);
      if (SOFT) ssa[wv][lane] = A.lj_a[tp];
      if (PG || HVP) ssig[wv][lane] = A.lj_sig[tp];
    }
    wave_sync();
    for (int t = s; t < cnt; t += S) {
      const int j = sj[wv][t];
      double dx = A.x[(0 * (size_t)N + j) * P + b] - xi;
      double dy = A.x[(1 * (size_t)N + j) * P + b] - yi;
      double dz = A.x[(2 * (size_t)N + j) * P + b] - zi;
      dx -= A.L[0] * rint(dx * A.invL[0]);
      dy -= A.L[1] * rint(dy * A.invL[1]);
      dz -= A.L[2] * rint(dz * A.invL[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < A.rc2) {
        double r, ir, erfcv, ex2;
        if constexpr (F32) {
          const float r2f = (float)r2;
          const float irf = __builtin_amdgcn_rsqf(r2f), rf = r2f * irf;
          const float tt = __builtin_amdgcn_rcpf(1.0f + ERFC_P * ((float)A.alpha * rf));
          float qf = ERFC_Q[7];
#pragma unroll
          for (int m = 6; m >= 0; --m) qf = qf * tt + ERFC_Q[m];
          const float exf = __builtin_amdgcn_exp2f(
              (float)(-A.alpha * A.alpha * 1.4426950408889634) * r2f);
          r = (double)rf; ir = (double)irf;
          ex2 = (double)exf; erfcv = (double)(tt * qf * exf);
        } else {
          r = sqrt(r2); ir = 1.0 / r;
          erfcv = erfc(A.alpha * r); ex2 = exp(-A.alpha * A.alpha * r2);
        }
        const double ir2 = ir * ir;
        const double qq = sq[wv][t];
        double sc = qq * (erfcv * ir + c2a * ex2) * ir2;
        if (ENERGY) ec += qq * erfcv * ir;
        if (PG) pq += A.coulomb * A.charge[j] * erfcv * ir;
        const double2 lj = slj[wv][t];
        const double e4 = lj.x;
        if (SOFT && e4 != 0.0) {
          const double s6 = lj.y * ir2 * ir2 * ir2;
          const double rd = 1.0 / (1.0 + ssa[wv][t] * s6), u = s6 * rd;
          sc += 6.0 * e4 * u * (2.0 * u - 1.0) * rd * ir2;
          if (ENERGY) elj += e4 * (u * u - u);
        } else if (e4 != 0.0) {
          const double s6 = lj.y * ir2 * ir2 * ir2;
          sc += e4 * (12.0 * s6 * s6 - 6.0 * s6) * ir2;
          if (ENERGY) elj += e4 * (s6 * s6 - s6);
          if (PG) {
            pe += (s6 * s6 - s6) * e4 * half_over_eps;            // dE/de_ij * e_ij / (2 eps_i)
            ps += 0.5 * e4 * (12.0 * s6 * s6 - 6.0 * s6) / ssig[wv][t];
          }
        }
        if (HVP) {
          // phi' and phi'' of the pair: -sc r is phi'; phi'' below
          double d1 = -sc * r;
          double d2 = qq * (2.0 * erfcv * ir2 * ir + c2a * ex2 * (2.0 * ir2 + 2.0 * A.alpha * A.alpha));
          if (e4 != 0.0) {
            const double s6 = lj.y * ir2 * ir2 * ir2;
            d2 += e4 * (156.0 * s6 * s6 - 42.0 * s6) * ir2;
          }
          const double ux = uix - A.u[(0 * (size_t)N + j) * P + b];
          const double uy = uiy - A.u[(1 * (size_t)N + j) * P + b];
          const double uz = uiz - A.u[(2 * (size_t)N + j) * P + b];
          const double dd = dx * ux + dy * uy + dz * uz;
          const double c1 = (d2 - d1 * ir) * ir2 * dd, c0 = d1 * ir;
          gx += c1 * dx + c0 * ux; gy += c1 * dy + c0 * uy; gz += c1 * dz + c0 * uz;
          if (mix) {
            // d r / dh along u is r^ . (u_j - u_i) = -dd / r; the i-side parameter terms
            const double drdh = -dd * ir;
            pq += A.coulomb * A.charge[j] * -(erfcv * ir2 + c2a * ex2 * ir) * drdh;
            if (e4 != 0.0) {
              const double s6 = lj.y * ir2 * ir2 * ir2;
              pe += (-12.0 * s6 * s6 + 6.0 * s6) * ir * e4 * half_over_eps * drdh;
              ps += 0.5 * e4 * (-144.0 * s6 * s6 + 36.0 * s6) * ir / ssig[wv][t] * drdh;
            }
          }
        } else {
          gx += sc * dx; gy += sc * dy; gz += sc * dz;
        }
      }
    }
    wave_sync();
  }
  if (HVP) {
    gx = slot_sum<P>(gx); gy = slot_sum<P>(gy); gz = slot_sum<P>(gz);
    if (lane < P) {
      A.hu[(0 * (size_t)N + i) * P + lane] += gx;
      A.hu[(1 * (size_t)N + i) * P + lane] += gy;
      A.hu[(2 * (size_t)N + i) * P + lane] += gz;
    }
    if (!mix) return;
  }
  if (!HVP) flush<P, ENERGY>(A, i, lane, gx, gy, gz, ec, elj);
  if (PG || mix) {
    for (int o = 1; o < 64; o <<= 1) {
      pq += __shfl_xor(pq, o);
      pe += __shfl_xor(pe, o);
      ps += __shfl_xor(ps, o);
    }
    if (lane == 0) {
      A.dq[i] += pq;
      if (pe != 0.0) atomicAdd(A.deps + ti, pe);
      if (ps != 0.0) atomicAdd(A.dsig + ti, ps);
    }
  }
}

// Constants of the FP32 interaction, set once per atom.
struct Pair32K {
  float4 oi;              // the lane's bead offset from atom i's centroid
  float rc2, tscale, alpha, kexp, c2a;
  int kmin;
  const float4* stab;     // the block's kernel tables
};

// One pair at the lane's bead: cd = FP32 centroid difference and q_i q_j C, oj = atom j's
// bead offset, lj = (4 eps_ij, sigma_ij^6), a = soft-core alpha (1 - lambda); adds the
// force on atom i to (fx, fy, fz) and the energies to ec, elj.
template <bool ENERGY, bool LJ, bool SOFT>
QHP_DEV void interact32(const Pair32K& K, const float4 cd, const float4 oj, const float2 lj,
                        const float a, float& fx, float& fy, float& fz, double& ec,
                        double& elj) {
  const float4 oi = K.oi;
  const float rc2 = K.rc2, tscale = K.tscale, alpha = K.alpha, kexp = K.kexp, c2a = K.c2a;
  const int kmin = K.kmin;
  const float4* stab = K.stab;
  const float dx = cd.x + (oj.x - oi.x), dy = cd.y + (oj.y - oi.y), dz = cd.z + (oj.z - oi.z);
  const float r2 = dx * dx + dy * dy + dz * dz;
  if (r2 < rc2) {
    const float u = r2 * tscale;
    const int k = (int)u;              // < QHP_PAIR_TAB for r2 < rc2 (see tab_scale)
    float sc;
    if (k >= kmin) {
      const float f = __builtin_amdgcn_fractf(u);
      const float4 c = stab[k];
      sc = cd.w * fmaf(fmaf(fmaf(c.w, f, c.z), f, c.y), f, c.x);
      if (ENERGY) {
        const float4 d = stab[QHP_PAIR_TAB + k];
        ec += (double)(cd.w * fmaf(fmaf(fmaf(d.w, f, d.z), f, d.y), f, d.x));
      }
    } else {
      const float ir = __builtin_amdgcn_rsqf(r2), ir2 = ir * ir;
      const float x = alpha * (r2 * ir);
      const float tt = __builtin_amdgcn_rcpf(1.0f + ERFC_P * x);
      float q = ERFC_Q[7];
#pragma unroll
      for (int m = 6; m >= 0; --m) q = q * tt + ERFC_Q[m];
      const float ex = __builtin_amdgcn_exp2f(kexp * r2);     // exp(-alpha^2 r^2)
      const float tq = tt * q;                                 // erfc(alpha r) / ex
      sc = cd.w * ir2 * ex * (tq * ir + c2a);
      if (ENERGY) ec += (double)(cd.w * tq * ex * ir);
    }
    const float ir2 = LJ ? __builtin_amdgcn_rcpf(r2) : 0.f;
    if (LJ && SOFT) {
      const float s6 = lj.y * ir2 * ir2 * ir2;
      const float rd = __builtin_amdgcn_rcpf(1.0f + a * s6), u = s6 * rd;
      sc += 6.f * lj.x * u * (2.f * u - 1.f) * rd * ir2;
      if (ENERGY) elj += (double)(lj.x * (u * u - u));
    } else if (LJ) {
      const float s6 = lj.y * ir2 * ir2 * ir2;
      sc += lj.x * (12.f * s6 * s6 - 6.f * s6) * ir2;
      if (ENERGY) elj += (double)(lj.x * (s6 * s6 - s6));
    }
    fx += sc * dx; fy += sc * dy; fz += sc * dz;
  }
}

// Compacted neighbours t0 + s, t0 + s + S, ... < cnt for the lane (slot s, bead b).
// LJ = false for neighbours without an LJ term (a wavefront-uniform choice).
// SOFT: the LJ neighbours' soft-core alpha (1 - lambda) is in sa (the k_pair64 form).
// The screened Coulomb force and energy kernels come from cubic tables in r^2 (stab: force,
// stab + QHP_PAIR_TAB: energy), so a pair without an LJ term takes no square root or
// reciprocal; pairs closer than the tables' first used interval (1 A; none in liquid
// water) take the erfc fit instead.
template <int P, bool ENERGY, bool LJ, bool SOFT = false>
QHP_DEV void chunk(const PairArgs& A, const float4* scd, const float2* slj, const float* sa,
                   const unsigned* sj, const float4* stab, int t0, int cnt, int s,
                   unsigned boff, float4 oi, float rc2, float alpha, float kexp, float c2a,
                   float& fx, float& fy, float& fz, double& ec, double& elj) {
  constexpr int S = 64 / P;
  const char* xf = reinterpret_cast<const char*>(A.xf);
  const float tscale = A.tab_scale;
  const int kmin = A.tab_kmin;
  // one bead: the bead is its centroid and its stored offset is exactly zero
  auto load = [&](int t) {
    if constexpr (P == 1) return make_float4(0.f, 0.f, 0.f, 0.f);
    else return *reinterpret_cast<const float4*>(xf + (sj[t] + boff));
  };
  const Pair32K K{oi, rc2, tscale, alpha, kexp, c2a, kmin, stab};
  auto interact = [&](const float4 cd, const float4 oj, const float2 lj, const float a) {
    interact32<ENERGY, LJ, SOFT>(K, cd, oj, lj, a, fx, fy, fz, ec, elj);
  };
  // four neighbours per lane per iteration: their loads are all issued before the math;
  // the trip count is the same for every lane (a scalar loop), the remainder follows
  int tt = t0;
  for (; tt + 4 * S <= cnt; tt += 4 * S) {
    const int t = tt + s;
    const float4 o0 = load(t), o1 = load(t + S), o2 = load(t + 2 * S), o3 = load(t + 3 * S);
    interact(scd[t], o0, slj[t], SOFT ? sa[t] : 0.f);
    interact(scd[t + S], o1, slj[t + S], SOFT ? sa[t + S] : 0.f);
    interact(scd[t + 2 * S], o2, slj[t + 2 * S], SOFT ? sa[t + 2 * S] : 0.f);
    interact(scd[t + 3 * S], o3, slj[t + 3 * S], SOFT ? sa[t + 3 * S] : 0.f);
  }
  for (int t = tt + s; t < cnt; t += S) interact(scd[t], load(t), slj[t], SOFT ? sa[t] : 0.f);
}

// One bead (P = 1): a lane's list entry is its only interaction in a chunk of 64, so the
// decoded entry is evaluated in place (no staging, no compaction). The centroid records of
// the next PF chunks are kept in flight and the list entries one chunk further (PF = 1, 2
// and 3 measured the same on the 21,952-water box).
template <bool SOFT, int W, int PF>
__global__ __launch_bounds__(64 * W) void k_pair32_one(PairArgs A) {
  __shared__ float4 stab[QHP_PAIR_TAB];
  __shared__ float2 sljt[QHP_MAX_TYPES * QHP_MAX_TYPES];   // (4 eps, sigma^6) per type pair
  __shared__ float slja[SOFT ? QHP_MAX_TYPES * QHP_MAX_TYPES : 1];
  for (int k = threadIdx.x; k < QHP_PAIR_TAB; k += 64 * W) stab[k] = A.tab[k];
  for (int k = threadIdx.x; k < A.ntypes * A.ntypes; k += 64 * W) {
    sljt[k] = make_float2((float)A.lj_e4[k], (float)A.lj_s6[k]);
    if (SOFT) slja[k] = (float)A.lj_a[k];
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int i = lb * W + wv;
  if (lb >= A.nblocks || i >= A.N) return;       // whole wavefront leaves together
  const double4 ci = A.cwrap[i];
  const double qi = A.coulomb * A.charge[i];
  const int ti = A.type[i];
  const float alpha = (float)A.alpha;
  const float kexp = (float)(-A.alpha * A.alpha * 1.4426950408889634);  // -alpha^2 log2(e)
  const float c2a = (float)(2.0 * A.alpha / sqrt(M_PI));
  const float rc2 = (float)A.rc2;
  const float reach2 = (float)((sqrt(A.rc2) + 1e-3) * (sqrt(A.rc2) + 1e-3));
  const int nn = A.nnbr[i];
  const int* row = A.nbr + (size_t)i * A.cap;
  const Pair32K K{make_float4(0.f, 0.f, 0.f, 0.f), rc2, A.tab_scale, alpha, kexp, c2a,
                  A.tab_kmin, stab};
  // ring of prefetched chunks: centroid records of chunks k .. k + PF - 1, the list entry
  // of chunk k + PF
  unsigned e[PF + 1];
  double4 cj[PF];
  double qj[PF];
  int tj[PF];
#pragma unroll
  for (int p = 0; p <= PF; ++p) e[p] = p * 64 + lane < nn ? (unsigned)row[p * 64 + lane] : 0u;
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    cj[p] = make_double4(0.0, 0.0, 0.0, 0.0); qj[p] = 0.0; tj[p] = 0;
    if (p * 64 + lane < nn) {
      const int j = e[p] & 0x3FFFFFF;
      cj[p] = A.cwrap[j];
      if (!A.pack_qt) { qj[p] = A.charge[j]; tj[p] = A.type[j]; }
    }
  }
  // each lane sums its forces in FP32 over QHP_ONE_ACC chunks (one interaction each), then
  // in FP64
  double gx = 0, gy = 0, gz = 0, ec = 0, elj = 0;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  for (int k0 = 0; k0 < nn; k0 += 64) {
    const unsigned ec0 = e[0];
    const double4 c = cj[0];
    const double qq = A.pack_qt ? (double)qhp::packed_charge(c.w) : qj[0];
    const int tt = A.pack_qt ? qhp::packed_type(c.w) : tj[0];
#pragma unroll
    for (int p = 0; p < PF; ++p) e[p] = e[p + 1];
#pragma unroll
    for (int p = 0; p + 1 < PF; ++p) { cj[p] = cj[p + 1]; qj[p] = qj[p + 1]; tj[p] = tj[p + 1]; }
    // chunk k + PF from the entry loaded one chunk ago; the entry of chunk k + PF + 1
    {
      const int t = k0 + PF * 64 + lane;
      cj[PF - 1] = make_double4(0.0, 0.0, 0.0, 0.0); qj[PF - 1] = 0.0; tj[PF - 1] = 0;
      if (t < nn) {
        const int j = e[PF - 1] & 0x3FFFFFF;
        cj[PF - 1] = A.cwrap[j];
        if (!A.pack_qt) { qj[PF - 1] = A.charge[j]; tj[PF - 1] = A.type[j]; }
      }
      e[PF] = t + 64 < nn ? (unsigned)row[t + 64] : 0u;
    }
    if (k0 + lane < nn) {
      const float cx = (float)((c.x - ci.x) + A.L[0] * (double)((int)((ec0 >> 26) & 3) - 1));
      const float cy = (float)((c.y - ci.y) + A.L[1] * (double)((int)((ec0 >> 28) & 3) - 1));
      const float cz = (float)((c.z - ci.z) + A.L[2] * (double)((int)((ec0 >> 30) & 3) - 1));
      if (cx * cx + cy * cy + cz * cz < reach2) {
        const int tp = ti * A.ntypes + tt;
        const float2 ljv = sljt[tp];
        const float av = SOFT ? slja[tp] : 0.f;
        interact32<false, true, SOFT>(K, make_float4(cx, cy, cz, (float)(qi * qq)),
                                      make_float4(0.f, 0.f, 0.f, 0.f), ljv, av, fx, fy, fz,
                                      ec, elj);
      }
    }
    if (((k0 >> 6) & (QHP_ONE_ACC - 1)) == QHP_ONE_ACC - 1) {    // same chunk for every lane
      gx += (double)fx; gy += (double)fy; gz += (double)fz;
      fx = fy = fz = 0.f;
    }
  }
  gx += (double)fx; gy += (double)fy; gz += (double)fz;
  flush<1, false>(A, i, lane, gx, gy, gz, ec, elj);
}

// W atoms (wavefronts) per block: the launch shape the autotuner picks
template <int P, bool ENERGY, bool SOFT = false, int W = WPB>
__global__ __launch_bounds__(64 * W) void k_pair32(PairArgs A) {
  constexpr int S = 64 / P;
  __shared__ float4 scd[W][64];     // centroid difference (x, y, z) and q_i q_j C
  __shared__ float2 slj[W][64];     // 4 eps_ij and sigma_ij^6 of the pair
  __shared__ float ssa[SOFT ? W : 1][SOFT ? 64 : 1];   // soft-core alpha (1 - lambda)
  __shared__ unsigned sj[W][64];    // byte offset of atom j's bead-0 FP32 offset
  __shared__ float4 stab[(ENERGY ? 2 : 1) * QHP_PAIR_TAB];   // kernel tables
  __shared__ float2 sljt[QHP_MAX_TYPES * QHP_MAX_TYPES];   // (4 eps, sigma^6) per type pair
  __shared__ float slja[SOFT ? QHP_MAX_TYPES * QHP_MAX_TYPES : 1];
  for (int k = threadIdx.x; k < (ENERGY ? 2 : 1) * QHP_PAIR_TAB; k += 64 * W) stab[k] = A.tab[k];
  for (int k = threadIdx.x; k < A.ntypes * A.ntypes; k += 64 * W) {
    sljt[k] = make_float2((float)A.lj_e4[k], (float)A.lj_s6[k]);
    if (SOFT) slja[k] = (float)A.lj_a[k];
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, s = lane / P, b = lane % P;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int i = lb * W + wv;
  if (lb >= A.nblocks || i >= A.N) return;       // whole wavefront leaves together
  const float4 oi = A.xf[(size_t)i * P + b];
  const double4 ci = A.cwrap[i];
  const double qi = A.coulomb * A.charge[i];
  const int ti = A.type[i];
  const unsigned boff = (unsigned)b * (unsigned)sizeof(float4);
  const float alpha = (float)A.alpha;
  const float kexp = (float)(-A.alpha * A.alpha * 1.4426950408889634);  // -alpha^2 log2(e)
  const float c2a = (float)(2.0 * A.alpha / sqrt(M_PI));
  const float rc2 = (float)A.rc2;
  // no bead of a pair whose centroids are further apart than rc + d_i + d_j can be within
  // the cutoff, d = an atom's largest bead-centroid distance this step (kept in the w of
  // its centroid record); small margin for the FP32 rounding of the difference
  const double di = P == 1 ? 0.0 : (A.pack_qt ? (double)qhp::packed_spread(ci.w) : ci.w);
  const double reach_i = sqrt(A.rc2) + di + 1e-3;
  const int nn = A.nnbr[i];
  const int* row = A.nbr + (size_t)i * A.cap;
  double gx = 0, gy = 0, gz = 0, ec = 0, elj = 0;
  // list entries of the next chunk are loaded while the current one is processed; with
  // one bead (a chunk is one interaction per lane) also the next chunk's centroid
  // records, charges and types, and the list entries two chunks ahead
  unsigned e_next = lane < nn ? (unsigned)row[lane] : 0u;
  double4 cj_n = make_double4(0.0, 0.0, 0.0, 0.0);
  double qj_n = 0.0;
  int tj_n = 0;
  unsigned e_nn = 0u;
  if constexpr (P == 1) {
    if (lane < nn) {
      const int j = e_next & 0x3FFFFFF;
      cj_n = A.cwrap[j]; qj_n = A.charge[j]; tj_n = A.type[j];
    }
    if (64 + lane < nn) e_nn = (unsigned)row[64 + lane];
  }
  for (int k0 = 0; k0 < nn; k0 += 64) {
    bool keep = false, haslj = false;
    float4 cdv;
    float2 ljv;
    float av = 0.f;
    unsigned jp = 0;
    const unsigned e_cur = e_next;
    double4 cj_p = cj_n;
    double qj_p = qj_n;
    int tj_p = tj_n;
    if constexpr (P == 1) {
      e_next = e_nn;
      if (k0 + 64 + lane < nn) {
        const int jn = e_next & 0x3FFFFFF;
        cj_n = A.cwrap[jn]; qj_n = A.charge[jn]; tj_n = A.type[jn];
      }
      if (k0 + 128 + lane < nn) e_nn = (unsigned)row[k0 + 128 + lane];
    } else if (k0 + 64 + lane < nn) {
      e_next = (unsigned)row[k0 + 64 + lane];
    }
    if (k0 + lane < nn) {
      const unsigned e = e_cur;
      const int j = e & 0x3FFFFFF;
      if constexpr (P != 1) {
        cj_p = A.cwrap[j];
        if (A.pack_qt) { qj_p = (double)qhp::packed_charge(cj_p.w); tj_p = qhp::packed_type(cj_p.w); }
        else { qj_p = A.charge[j]; tj_p = A.type[j]; }
      }
      const double4 cj = cj_p;
      const float cx = (float)((cj.x - ci.x) + A.L[0] * (double)((int)((e >> 26) & 3) - 1));
      const float cy = (float)((cj.y - ci.y) + A.L[1] * (double)((int)((e >> 28) & 3) - 1));
      const float cz = (float)((cj.z - ci.z) + A.L[2] * (double)((int)((e >> 30) & 3) - 1));
      const float reach = (float)(reach_i + (P == 1 ? 0.0 : (A.pack_qt ? (double)qhp::packed_spread(cj.w) : cj.w)));
      keep = cx * cx + cy * cy + cz * cz < reach * reach;
      cdv = make_float4(cx, cy, cz, (float)(qi * qj_p));
      const int tp = ti * A.ntypes + tj_p;
      ljv = sljt[tp];
      if (SOFT) av = slja[tp];
      haslj = ljv.x != 0.f;
      jp = (unsigned)j * (unsigned)(P * sizeof(float4));
    }
    if constexpr (P == 1) {
      // one bead: a lane's decoded entry is its only interaction in the chunk, so it is
      // evaluated in place (no staging; the LJ term of a pair without LJ is zero)
      float fx = 0.f, fy = 0.f, fz = 0.f;
      if (keep) {
        const Pair32K K{oi, rc2, A.tab_scale, alpha, kexp, c2a, A.tab_kmin, stab};
        interact32<ENERGY, true, SOFT>(K, cdv, make_float4(0.f, 0.f, 0.f, 0.f), ljv, av,
                                       fx, fy, fz, ec, elj);
      }
      gx += (double)fx; gy += (double)fy; gz += (double)fz;
      continue;
    }
    // compaction with the LJ pairs first: [0, nlj) carry LJ, [nlj, cnt) do not
    const unsigned long long bl = __ballot(keep && haslj), bn = __ballot(keep && !haslj);
    const int nlj = __popcll(bl), cnt = nlj + __popcll(bn);
    if (keep) {
      const unsigned long long below = (1ull << lane) - 1ull;
      const int slot = haslj ? __popcll(bl & below) : nlj + __popcll(bn & below);
      scd[wv][slot] = cdv;
      slj[wv][slot] = ljv;
      if (SOFT) ssa[wv][slot] = av;
      sj[wv][slot] = jp;
    }
    wave_sync();
    float fx = 0.f, fy = 0.f, fz = 0.f;
    if (nlj > 0)
      chunk<P, ENERGY, true, SOFT>(A, scd[wv], slj[wv], ssa[SOFT ? wv : 0], sj[wv], stab, 0,
                                   nlj, s, boff, oi, rc2, alpha, kexp, c2a, fx, fy, fz, ec,
                                   elj);
    chunk<P, ENERGY, false>(A, scd[wv], slj[wv], nullptr, sj[wv], stab, nlj, cnt, s, boff, oi,
                            rc2, alpha, kexp, c2a, fx, fy, fz, ec, elj);
    gx += (double)fx; gy += (double)fy; gz += (double)fz;
    wave_sync();
  }
  flush<P, ENERGY>(A, i, lane, gx, gy, gz, ec, elj);
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

hipError_t launch_pair(qhp_ctx* c, bool energy, int bead, const BeadSet* bs) {
  PairArgs A;
  const int N = c->N;
  A.N = N; A.cap = c->cap;
  const bool plain = bead >= 0;
  const BeadSet B = bs ? *bs : full_beads(c);
  A.x = plain ? c->x + (size_t)bead * 3 * N : B.x;
  A.g = plain ? c->g + (size_t)bead * 3 * N : B.g;
  A.cwrap = c->cwrap; A.xf = B.xf; A.nbr = c->nbr; A.nnbr = c->nnbr;
  A.charge = c->d_charge; A.type = c->d_type;
  for (int d = 0; d < 3; ++d) { A.L[d] = c->p.box[d]; A.invL[d] = 1.0 / c->p.box[d]; }
  A.rc2 = c->p.cutoff * c->p.cutoff; A.alpha = c->p.ewald_alpha; A.coulomb = c->p.coulomb;
  A.ntypes = c->p.n_types;
  // solute-solvent pairs of an alchemical system: epsilon scaled by lambda_vdw and the
  // soft-core alpha (1 - lambda_vdw) (the current couplings, read at launch)
  bool soft = false;
  for (int a = 0; a < c->p.n_types; ++a)
    for (int b = 0; b < c->p.n_types; ++b) {
      const double s = 0.5 * (c->sigma[a] + c->sigma[b]);
      const double e = sqrt(c->eps[a] * c->eps[b]);
      const bool mixed = c->alch && c->soft[a] != c->soft[b];
      const double lam = mixed ? c->lam_v : 1.0;
      const double sa = mixed ? c->p.sc_alpha * (1.0 - c->lam_v) : 0.0;
      A.lj_s6[a * A.ntypes + b] = s * s * s * s * s * s;
      A.lj_e4[a * A.ntypes + b] = 4.0 * e * lam;
      A.lj_a[a * A.ntypes + b] = sa;
      A.lj_sig[a * A.ntypes + b] = s;
      soft = soft || (sa != 0.0 && e * lam != 0.0);
    }
  for (int a = 0; a < c->p.n_types; ++a) A.eps_of[a] = c->eps[a];
  A.dq = c->pg_dq; A.deps = c->pg_lj; A.dsig = c->pg_lj + QHP_MAX_TYPES;
  A.tab = c->pair_tab;
  A.tab_scale = c->pair_tab_scale;
  A.tab_kmin = c->pair_tab_kmin;

  A.energy = plain ? c->energy + (size_t)bead * QHP_NTERMS : B.energy;
  A.ctrl = c->ctrl;
  A.pack_qt = c->pack_qt ? 1 : 0;
  const int P = plain ? 1 : B.P;
  A.nblocks = (N + WPB - 1) / WPB;
  const unsigned nb = (unsigned)((A.nblocks + 7) / 8 * 8);
  // FP32 force launches: c->pair_wpb atoms per block (2, 4 or 8)
  const int w = c->pair_wpb == 2 || c->pair_wpb == 8 ? c->pair_wpb : WPB;
  const int nlw = (N + w - 1) / w;
  const unsigned nbw = (unsigned)((nlw + 7) / 8 * 8);
  const double Lmin = fmin(c->p.box[0], fmin(c->p.box[1], c->p.box[2]));
  const bool minimg = !(2.0 * (c->p.cutoff + c->p.skin) < Lmin);
  const bool pg = bs && bs->pgrad;     // parameter gradients: the k_pair64 kernels
  const bool hvp = bs && bs->hvp_u;    // Hessian-vector product: the k_pair64 kernels
  const bool f32 = c->p.precision == QHP_FP32_PAIRS && !plain && !minimg && !pg && !hvp;
  A.mix = 0;
  if (hvp) { A.u = bs->hvp_u; A.hu = bs->g; A.mix = bs->pgrad; }
  hipEvent_t ev = nullptr;
  prof_begin(c, QHP_PROF_PAIR, &ev);
  if (f32 && soft && !energy) {
    A.nblocks = nlw;
    QHP_SWITCH_P(P, if (w == 2) hipLaunchKernelGGL((k_pair32<PP, false, true, 2>), nbw, 128, 0, c->stream, A);
                 else if (w == 8) hipLaunchKernelGGL((k_pair32<PP, false, true, 8>), nbw, 512, 0, c->stream, A);
                 else hipLaunchKernelGGL((k_pair32<PP, false, true>), nb, NT, 0, c->stream, A));
  } else if (f32 && soft) {
    QHP_SWITCH_P(P, hipLaunchKernelGGL((k_pair32<PP, true, true>), nb, NT, 0, c->stream, A));
  } else if (f32 && !energy && P == 1) {
    A.nblocks = nlw;
    if (w == 2) hipLaunchKernelGGL((k_pair32_one<false, 2, QHP_PAIR_PF>), nbw, 128, 0, c->stream, A);
    else if (w == 8) hipLaunchKernelGGL((k_pair32_one<false, 8, QHP_PAIR_PF>), nbw, 512, 0, c->stream, A);
    else hipLaunchKernelGGL((k_pair32_one<false, 4, QHP_PAIR_PF>), nb, NT, 0, c->stream, A);
  } else if (f32 && !energy) {
    A.nblocks = nlw;
    QHP_SWITCH_P(P, if (w == 2) hipLaunchKernelGGL((k_pair32<PP, false, false, 2>), nbw, 128, 0, c->stream, A);
                 else if (w == 8) hipLaunchKernelGGL((k_pair32<PP, false, false, 8>), nbw, 512, 0, c->stream, A);
                 else hipLaunchKernelGGL((k_pair32<PP, false>), nb, NT, 0, c->stream, A));
  } else if (f32) {
    QHP_SWITCH_P(P, hipLaunchKernelGGL((k_pair32<PP, true>), nb, NT, 0, c->stream, A));
  } else if (soft) {
    if (pg || hvp) return hipErrorInvalidValue;     // rejected by the entry points
    QHP_SWITCH_P(P, if (energy) hipLaunchKernelGGL((k_pair64<PP, true, false, false, true>), nb, NT, 0, c->stream, A);
                 else hipLaunchKernelGGL((k_pair64<PP, false, false, false, true>), nb, NT, 0, c->stream, A));
  } else if (c->p.precision == QHP_FP32_PAIRS && (pg || hvp)) {
    QHP_SWITCH_P(P, if (hvp) hipLaunchKernelGGL((k_pair64<PP, false, false, true, false, true>), nb, NT, 0, c->stream, A);
                 else hipLaunchKernelGGL((k_pair64<PP, false, true, false, false, true>), nb, NT, 0, c->stream, A));
  } else {
    QHP_SWITCH_P(P, if (hvp) hipLaunchKernelGGL((k_pair64<PP, false, false, true>), nb, NT, 0, c->stream, A);
                 else if (pg) hipLaunchKernelGGL((k_pair64<PP, false, true>), nb, NT, 0, c->stream, A);
                 else if (energy) hipLaunchKernelGGL((k_pair64<PP, true>), nb, NT, 0, c->stream, A);
                 else hipLaunchKernelGGL((k_pair64<PP, false>), nb, NT, 0, c->stream, A));
  }
  prof_end(c, QHP_PROF_PAIR, ev);
  return hipGetLastError();
}
