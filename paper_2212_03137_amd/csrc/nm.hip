// Normal-mode propagation of the ring polymer (Sec. "Integration Scheme"): the fused
// B A O A kernel with the mode -> bead transform (eq. beads_positions) and the projection
// of bead forces on modes (eq. force_normal_modes), plus the state conversions at the
// boundary.
//
// Lane layout: a 256-thread block holds 256/P atoms; lane (a, n) owns mode n of atom a
// for x, y and z. The bead-axis contractions (T^T g and T Q, both P x P) go through LDS:
// at P = 32 they are 2 x 3 x 32 FMAs per lane, fed by paired (16-byte) LDS reads, and the
// kernel stays bound by HBM.
//
// Persistent state between steps: Q, Pa (momenta after the A-O-A of the last step, i.e.
// before its final half kick) and g = grad V at the current beads. A step therefore
// starts with P = Pa + dt * f(g): the previous step's final B and this step's first B,
// which use the same forces.
#include <mutex>

#include "qhp_internal.h"

namespace {

constexpr int NT = 256;

struct NmArgs {
  int N;
  double* Q; double* Pa; double* x; const double* g;
  const double* T; const double* cc; const double* csw; const double* cws;
  const double* c1; const double* c2;
  const double* mass; const double* sqrt_mkT; const double* charge;
  const int* type; int pack_qt;   // packed centroid records: charge, type and spread in w
  double4* cent; const double4* cref; const double4* coff; double4* cwrap; float4* xf;
  NlCtrl* ctrl;
  double4* bmax;
  double KoL[3];
  int K[3], order;
  double dt, h;
  uint64_t seed;
  // adQTB
  const double* noise; double* vrec; int nseg; double qc1, qosd;
  // multiple time stepping / ring-polymer contraction
  const double* gs;        // [3][N][Ps] grad V_s at the contracted beads
  const double* Cs;        // [Ps][Ps] contraction matrix C[j][n]
  double* xs;              // [3][N][Ps] contracted beads (written when emit)
  float4* xfs;             // [N][Ps]
  int Ps, step_off, emit;     // Ps: lanes of the contracted set (phantoms beyond Psb)
  double sP, rsP, sPs, rsPs;  // sqrt and 1/sqrt of the real bead counts Pb and Psb
  double slow_h;           // factor of the slow kick this inner step (0: none)
  qhp::BinGeom bins;       // SPME tile and list cell of every centroid (when emitting)
};

template <int P, bool BEADMAJOR>
QHP_DEV int gidx(int N, int d, int a, int b) {
  return BEADMAJOR ? (b * 3 + d) * N + a : (d * N + a) * P + b;
}

QHP_DEV double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// out[d] = sum_i m_i v[d][i] for the three Cartesian rows v[d] of one atom, where m is the
// lane's vector of matrix entries stored in pairs (m_2j, m_2j+1) at M2[j * P + n]. One paired
// LDS read of m serves all three rows; the rows are read in pairs too, at the same address
// for every lane of the atom (a broadcast).
template <int P>
QHP_DEV void contract3(const double2* M2, const double (*v)[P + 2], int n, double* out) {
  if constexpr (P == 1) {
    for (int d = 0; d < 3; ++d) out[d] = reinterpret_cast<const double*>(M2)[0] * v[d][0];
  } else {
    double s[3][2] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll 4
    for (int j = 0; j < P / 2; ++j) {
      const double2 t = M2[j * P + n];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double2 w = *reinterpret_cast<const double2*>(&v[d][2 * j]);
        s[d][0] += t.x * w.x;
        s[d][1] += t.y * w.y;
      }
    }
    for (int d = 0; d < 3; ++d) out[d] = s[d][0] + s[d][1];
  }
}

// RESPA: the kick adds slow_h * f_s on the modes n < Ps (f_s = -C^T g_s / sqrt(Ps)), the
// noise counter is the outer step's plus step_off, x is written for the bonded terms, and
// only when emit are the contracted beads, their FP32 offsets, the centroids and the
// block maxima (of the contracted beads) written.
template <int P, bool QTB, bool BEADMAJOR, bool F32, bool RESPA = false>
__global__ __launch_bounds__(NT) void k_nm_step(NmArgs A) {
  constexpr int AT = NT / P;
  constexpr int PP = P + 2;          // row stride: 16-byte aligned rows; the atoms of a
                                     // wavefront read different banks
  constexpr int PH = P > 1 ? P / 2 : 1;
  __shared__ double2 sTc[PH * P];    // (T[2j][n], T[2j+1][n]) at j * P + n: column n of T
  __shared__ double2 sTr[PH * P];    // (T[n][2j], T[n][2j+1]) at j * P + n: row n, T[n][0] -> 0
  __shared__ __align__(16) double sh[AT][3][PP];
  __shared__ double sC[RESPA ? P * P : 1];       // C[j][n] at j * Ps + n
  __shared__ double sgs[RESPA ? AT : 1][3][RESPA ? P : 1];
  const int tid = threadIdx.x;
  const int al = tid / P, n = tid % P;
  const int a = blockIdx.x * AT + al;
  const int Ps = RESPA ? A.Ps : P;
  if (RESPA) {
    for (int k = tid; k < Ps * Ps; k += NT) sC[k] = A.Cs[k];
    if (A.slow_h != 0.0)
      for (int d = 0; d < 3; ++d)
        sgs[al][d][n] = (a < A.N && n < Ps) ? A.gs[(d * A.N + a) * Ps + n] : 0.0;
  }
  for (int k = tid; k < PH * P; k += NT) {
    const int j = k / P, m = k % P;
    if (P == 1) {
      sTc[0] = make_double2(A.T[0], 0.0);
      sTr[0] = make_double2(0.0, 0.0);
    } else {
      sTc[k] = make_double2(A.T[(2 * j) * P + m], A.T[(2 * j + 1) * P + m]);
      sTr[k] = make_double2(j == 0 ? 0.0 : A.T[m * P + 2 * j], A.T[m * P + 2 * j + 1]);
    }
  }
  const bool live = a < A.N;
  // advanced by the list check (by the inner steps of an outer step under RESPA)
  const uint64_t step = (uint64_t)A.ctrl->step + (RESPA ? (uint64_t)A.step_off : 0ull);
  double gv[3] = {0, 0, 0}, q0[3] = {0, 0, 0}, p0[3] = {0, 0, 0};
  if (live)
    for (int d = 0; d < 3; ++d) {
      const int gi = (d * A.N + a) * P + n;
      gv[d] = A.g[gidx<P, BEADMAJOR>(A.N, d, a, n)];
      q0[d] = A.Q[gi];
      p0[d] = A.Pa[gi];
    }
  for (int d = 0; d < 3; ++d) sh[al][d][n] = gv[d];
  __syncthreads();
  double fT[3];
  contract3<P>(sTc, sh[al], n, fT);
  const double rsP = A.rsP;
  double fsl[3] = {0.0, 0.0, 0.0};
  if (RESPA && A.slow_h != 0.0 && n < Ps) {
    const double rsPs = A.rsPs;
    for (int d = 0; d < 3; ++d) {
      double acc = 0.0;
      for (int j = 0; j < Ps; ++j) acc += sC[j * Ps + n] * sgs[al][d][j];
      fsl[d] = -acc * rsPs * A.slow_h;
    }
  }
  double q[3], p[3];
  double m = 1.0, cc = A.cc[n], csw = A.csw[n], cws = A.cws[n];
  int bad = 0;
  if (live) {
    m = A.mass[a];
    const double im = 1.0 / m;
    double xi[3] = {0, 0, 0};
    if (!QTB) qhp::gauss3(A.seed, qhp::STREAM_RPMD_O, step, (uint64_t)a, (uint64_t)n, xi);
    for (int d = 0; d < 3; ++d) {
      const double f = -fT[d] * rsP;
      const int gi = (d * A.N + a) * P + n;
      double pp = p0[d] + A.dt * f;
      if (RESPA) pp += fsl[d];
      double qq = q0[d];
      // A(h): exact free ring-polymer evolution of mode n
      double q1 = cc * qq + csw * im * pp;
      double p1 = -m * cws * qq + cc * pp;
      // O(dt)
      if (QTB) {
        const int ni = ((int)(step % (uint64_t)A.nseg) * 3 + d) * A.N + a;
        const double pb = p1;
        p1 = A.qc1 * p1 + A.qosd * A.noise[ni];
        A.vrec[ni] = 0.5 * (pb + p1) * im;
      } else {
        p1 = A.c1[n] * p1 + A.c2[n] * A.sqrt_mkT[a] * xi[d];
      }
      // A(h)
      q[d] = cc * q1 + csw * im * p1;
      p[d] = -m * cws * q1 + cc * p1;
      A.Q[gi] = q[d];
      A.Pa[gi] = p[d];
      if (!isfinite(q[d]) || !isfinite(p[d])) bad = 1;
    }
  }
  __syncthreads();
  if (live)
    for (int d = 0; d < 3; ++d) sh[al][d][n] = q[d];
  __syncthreads();

  // beads from modes: lane index n now stands for bead i = n
  double db2 = 0, dc2 = 0, cen[3] = {0.0, 0.0, 0.0};
  int moff = 0, mbad = 0;
  const bool emit = !RESPA || A.emit;
  if (live) {
    const double sP = A.sP;
    double xb[3], c[3], sx[3];
    // x_n = Q_0 + sqrt(P) sum_{k>=1} T[n][k] Q_k (the k = 0 term enters as Q_0 itself)
    contract3<P>(sTr, sh[al], n, sx);
    for (int d = 0; d < 3; ++d) {
      const double s = sx[d];
      c[d] = sh[al][d][0];
      xb[d] = c[d] + sP * s;
      A.x[gidx<P, BEADMAJOR>(A.N, d, a, n)] = xb[d];
      if (!isfinite(xb[d])) bad = 1;
    }
    // the bead set of the slow forces: the beads themselves, or (RESPA) lanes j < Ps hold
    // the contracted beads x~_j = Q_0 + sqrt(Ps) sum_{k=1}^{Ps-1} C[j][k] Q_k
    bool own = emit;
    if (RESPA && emit) {
      own = n < Ps;
      if (own) {
        const double sPs = A.sPs;
        for (int d = 0; d < 3; ++d) {
          double acc = 0.0;
          for (int k = 1; k < Ps; ++k) acc += sC[n * Ps + k] * sh[al][d][k];
          xb[d] = c[d] + sPs * acc;
          A.xs[(d * A.N + a) * Ps + n] = xb[d];
          if (!isfinite(xb[d])) bad = 1;
        }
      }
    }
    if (own) {
      const double dx = xb[0] - c[0], dy = xb[1] - c[1], dz = xb[2] - c[2];
      db2 = dx * dx + dy * dy + dz * dz;
      for (int d = 0; d < 3; ++d) {
        const int dl = qhp::base_diff(qhp::base_of(xb[d], A.KoL[d], A.K[d]),
                                      qhp::base_of(c[d], A.KoL[d], A.K[d]), A.K[d]);
        moff = max(moff, dl < 0 ? -dl : dl);
        if (dl > QHP_TB || dl < A.order - 1 - QHP_TB) mbad = 1;
      }
      const float4 o4 = make_float4((float)dx, (float)dy, (float)dz, (float)A.charge[a]);
      if (F32 && !RESPA) A.xf[a * P + n] = o4;
      if (F32 && RESPA) A.xfs[a * Ps + n] = o4;
    }
    cen[0] = c[0]; cen[1] = c[1]; cen[2] = c[2];
  }
  // largest bead-centroid distance of each atom (over its P lanes): the pair kernel's
  // per-pair reach; stored in the w components of the centroid records
  double adb2 = db2;
  for (int o = 1; o < P; o <<= 1) adb2 = fmax(adb2, __shfl_xor(adb2, o));
  if (live && emit && n == 0) {
    const double adb = sqrt(adb2);
    A.cent[a] = make_double4(cen[0], cen[1], cen[2], adb);
    qhp::write_bins(A.bins, a, cen[0], cen[1], cen[2]);
    const double4 o = A.coff[a];
    A.cwrap[a] = make_double4(cen[0] - o.x, cen[1] - o.y, cen[2] - o.z,
                              A.pack_qt ? qhp::pack_record(A.charge[a], A.type[a], adb) : adb);
    const double4 r = A.cref[a];
    const double ex = cen[0] - r.x, ey = cen[1] - r.y, ez = cen[2] - r.z;
    dc2 = ex * ex + ey * ey + ez * ez;
  }
  if (!emit) {                       // an inner step without slow forces after it
    if (bad) A.ctrl->nonfinite = 1;
    return;
  }
  // block maxima for the neighbour-list check and the SPME tile margin (no atomics)
  __shared__ double sm[4][NT / 64];
  db2 = wave_max(db2);
  dc2 = wave_max(dc2);
  const double mo = wave_max((double)moff), mb = wave_max((double)mbad);
  if ((tid & 63) == 0) { sm[0][tid >> 6] = dc2; sm[1][tid >> 6] = db2; sm[2][tid >> 6] = mo; sm[3][tid >> 6] = mb; }
  __syncthreads();
  if (tid == 0) {
    double a0 = sm[0][0], a1 = sm[1][0], a2 = sm[2][0], a3 = sm[3][0];
    for (int w = 1; w < NT / 64; ++w) {
      a0 = fmax(a0, sm[0][w]); a1 = fmax(a1, sm[1][w]); a2 = fmax(a2, sm[2][w]); a3 = fmax(a3, sm[3][w]);
    }
    A.bmax[blockIdx.x] = make_double4(a0, a1, a2, a3);
  }
  if (bad) A.ctrl->nonfinite = 1;
}

// Q = T^T x / sqrt(P), Pm = m T^T v / sqrt(P); inputs bead-innermost [3][N][P].
template <int P>
__global__ __launch_bounds__(NT) void k_to_modes(int N, double rsP, const double* xb,
                                                 const double* vb, const double* T,
                                                 const double* mass, double* Q, double* Pm) {
  constexpr int AT = NT / P;
  __shared__ double sT[P * P];
  __shared__ double sx[AT][6][P];
  const int tid = threadIdx.x, al = tid / P, n = tid % P, a = blockIdx.x * AT + al;
  for (int k = tid; k < P * P; k += NT) sT[k] = T[k];
  const bool live = a < N;
  for (int d = 0; d < 3; ++d) {
    sx[al][d][n] = live ? xb[(d * N + a) * P + n] : 0.0;
    sx[al][3 + d][n] = live ? vb[(d * N + a) * P + n] : 0.0;
  }
  __syncthreads();
  if (!live) return;
  const double m = mass[a];
  for (int d = 0; d < 3; ++d) {
    double sq = 0, sv = 0;
    for (int i = 0; i < P; ++i) {
      sq += sT[i * P + n] * sx[al][d][i];
      sv += sT[i * P + n] * sx[al][3 + d][i];
    }
    Q[(d * N + a) * P + n] = sq * rsP;
    Pm[(d * N + a) * P + n] = m * sv * rsP;
  }
}

// Pa += s * f with f = -T^T g / sqrt(P) (g in the context's layout).
template <int P, bool BEADMAJOR>
__global__ __launch_bounds__(NT) void k_kick(int N, double rsP, double* Pa, const double* g,
                                             const double* T, double s) {
  constexpr int AT = NT / P;
  __shared__ double sT[P * P];
  __shared__ double sg[AT][3][P];
  const int tid = threadIdx.x, al = tid / P, n = tid % P, a = blockIdx.x * AT + al;
  for (int k = tid; k < P * P; k += NT) sT[k] = T[k];
  const bool live = a < N;
  for (int d = 0; d < 3; ++d) sg[al][d][n] = live ? g[gidx<P, BEADMAJOR>(N, d, a, n)] : 0.0;
  __syncthreads();
  if (!live) return;
  for (int d = 0; d < 3; ++d) {
    double f = 0;
    for (int i = 0; i < P; ++i) f += sT[i * P + n] * sg[al][d][i];
    Pa[(d * N + a) * P + n] += s * (-f * rsP);
  }
}

// Bead positions and velocities [P][N][3] from (Q, Pa + h f).
template <int P, bool BEADMAJOR>
__global__ __launch_bounds__(NT) void k_state_out(int N, int Pb, double rsP, const double* Q,
                                                  const double* Pa, const double* g,
                                                  const double* T, const double* mass, double h,
                                                  double* xo, double* vo) {
  constexpr int AT = NT / P;
  __shared__ double sT[P * P];
  __shared__ double sh[AT][6][P];
  const int tid = threadIdx.x, al = tid / P, n = tid % P, a = blockIdx.x * AT + al;
  for (int k = tid; k < P * P; k += NT) sT[k] = T[k];
  const bool live = a < N;
  for (int d = 0; d < 3; ++d) sh[al][3 + d][n] = live ? g[gidx<P, BEADMAJOR>(N, d, a, n)] : 0.0;
  __syncthreads();
  const double sP = 1.0 / rsP;
  double pn[3] = {0, 0, 0}, qn[3] = {0, 0, 0};
  if (live)
    for (int d = 0; d < 3; ++d) {
      double f = 0;
      for (int i = 0; i < P; ++i) f += sT[i * P + n] * sh[al][3 + d][i];
      pn[d] = Pa[(d * N + a) * P + n] + h * (-f * rsP);
      qn[d] = Q[(d * N + a) * P + n];
    }
  __syncthreads();
  for (int d = 0; d < 3; ++d) { sh[al][d][n] = qn[d]; sh[al][3 + d][n] = pn[d]; }
  __syncthreads();
  if (!live || n >= Pb) return;      // phantom beads are not reported
  const double im = 1.0 / mass[a];
  for (int d = 0; d < 3; ++d) {
    double sx = 0, sv = 0;
    for (int k = 0; k < P; ++k) {
      sx += sT[n * P + k] * sh[al][d][k];
      sv += sT[n * P + k] * sh[al][3 + d][k];
    }
    if (xo) xo[((size_t)n * N + a) * 3 + d] = sP * sx;
    if (vo) vo[((size_t)n * N + a) * 3 + d] = sP * sv * im;
  }
}

// kinetic sum (Pa + h f)^2 / 2m and spring sum m w^2 Q^2 / 2 -> out[0], out[1]
template <int P, bool BEADMAJOR>
__global__ __launch_bounds__(NT) void k_mode_energy(int N, double rsP, const double* Q,
                                                    const double* Pa, const double* g,
                                                    const double* T, const double* mass,
                                                    const double* w2, double h, double* out) {
  constexpr int AT = NT / P;
  __shared__ double sT[P * P];
  __shared__ double sg[AT][3][P];
  const int tid = threadIdx.x, al = tid / P, n = tid % P, a = blockIdx.x * AT + al;
  for (int k = tid; k < P * P; k += NT) sT[k] = T[k];
  const bool live = a < N;
  for (int d = 0; d < 3; ++d) sg[al][d][n] = live ? g[gidx<P, BEADMAJOR>(N, d, a, n)] : 0.0;
  __syncthreads();
  double ek = 0, es = 0;
  if (live) {
    const double m = mass[a];
    for (int d = 0; d < 3; ++d) {
      double f = 0;
      for (int i = 0; i < P; ++i) f += sT[i * P + n] * sg[al][d][i];
      const double pn = Pa[(d * N + a) * P + n] + h * (-f * rsP);
      const double qn = Q[(d * N + a) * P + n];
      ek += pn * pn / (2.0 * m);
      es += 0.5 * m * w2[n] * qn * qn;
    }
  }
  for (int o = 32; o > 0; o >>= 1) { ek += __shfl_xor(ek, o); es += __shfl_xor(es, o); }
  if ((tid & 63) == 0) { atomicAdd(out, ek); atomicAdd(out + 1, es); }
}

// The same sums without atomics: each block writes its two partial sums to parts[2 b],
// parts[2 b + 1]; k_sum_parts adds them in block order (the result does not depend on the
// order in which blocks ran).
template <int P, bool BEADMAJOR>
__global__ __launch_bounds__(NT) void k_mode_energy_parts(int N, double rsP, const double* Q,
                                                          const double* Pa, const double* g,
                                                          const double* T, const double* mass,
                                                          const double* w2, double h,
                                                          double* parts) {
  constexpr int AT = NT / P;
  __shared__ double sT[P * P];
  __shared__ double sg[AT][3][P];
  __shared__ double sred[2][NT / 64];
  const int tid = threadIdx.x, al = tid / P, n = tid % P, a = blockIdx.x * AT + al;
  for (int k = tid; k < P * P; k += NT) sT[k] = T[k];
  const bool live = a < N;
  for (int d = 0; d < 3; ++d) sg[al][d][n] = live ? g[gidx<P, BEADMAJOR>(N, d, a, n)] : 0.0;
  __syncthreads();
  double ek = 0, es = 0;
  if (live) {
    const double m = mass[a];
    for (int d = 0; d < 3; ++d) {
      double f = 0;
      for (int i = 0; i < P; ++i) f += sT[i * P + n] * sg[al][d][i];
      const double pn = Pa[(d * N + a) * P + n] + h * (-f * rsP);
      const double qn = Q[(d * N + a) * P + n];
      ek += pn * pn / (2.0 * m);
      es += 0.5 * m * w2[n] * qn * qn;
    }
  }
  for (int o = 32; o > 0; o >>= 1) { ek += __shfl_xor(ek, o); es += __shfl_xor(es, o); }
  if ((tid & 63) == 0) { sred[0][tid >> 6] = ek; sred[1][tid >> 6] = es; }
  __syncthreads();
  if (tid == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int w = 0; w < NT / 64; ++w) { a0 += sred[0][w]; a1 += sred[1][w]; }
    parts[2 * blockIdx.x] = a0;
    parts[2 * blockIdx.x + 1] = a1;
  }
}

// out[0..1] = sums of the nparts partial pairs (one block, fixed order)
__global__ __launch_bounds__(256) void k_sum_parts(const double* parts, int nparts, double* out) {
  __shared__ double s[2][256];
  double a0 = 0.0, a1 = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) { a0 += parts[2 * k]; a1 += parts[2 * k + 1]; }
  s[0][threadIdx.x] = a0;
  s[1][threadIdx.x] = a1;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s[0][threadIdx.x] += s[0][threadIdx.x + st];
      s[1][threadIdx.x] += s[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = s[0][0]; out[1] = s[1][0]; }
}

// dst = src + s * f_s on the modes n < Ps, f_s = -(1/sqrt(Ps)) sum_j C[j][n] g_s(j) (the slow
// forces of ring-polymer contraction); the other modes are copied.
template <int P>
__global__ __launch_bounds__(NT) void k_kick_slow(int N, int Ps, double rsPs, double* dst,
                                                  const double* src, const double* gs,
                                                  const double* C, double s) {
  constexpr int AT = NT / P;
  __shared__ double sC[P * P];
  __shared__ double sg[AT][3][P];
  const int tid = threadIdx.x, al = tid / P, n = tid % P, a = blockIdx.x * AT + al;
  for (int k = tid; k < Ps * Ps; k += NT) sC[k] = C[k];
  const bool live = a < N;
  for (int d = 0; d < 3; ++d) sg[al][d][n] = (live && n < Ps) ? gs[(d * N + a) * Ps + n] : 0.0;
  __syncthreads();
  if (!live) return;
  for (int d = 0; d < 3; ++d) {
    double f = 0.0;
    if (n < Ps)
      for (int j = 0; j < Ps; ++j) f += sC[j * Ps + n] * sg[al][d][j];
    const int i = (d * N + a) * P + n;
    dst[i] = src[i] + s * (-f * rsPs);
  }
}

// centroid of given beads (bead-innermost or bead-major x): beads summed in order, / P;
// also the block maxima of the bead-centroid distance and grid-base offset
struct CentArgs {
  int N;
  int Pb;                   // real beads (the centroid is their mean; the others are phantoms)
  double sPs;               // k_contract: sqrt of the real contracted bead count
  const double* x; double4* cent; float4* xf; const double* charge;
  double4* bmax;
  double KoL[3];
  int K[3], order;
  qhp::BinGeom bins;
};

template <int P, bool BEADMAJOR>
__global__ __launch_bounds__(128) void k_centroid_beads(CentArgs A) {
  __shared__ double sm[3][2];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  double db2 = 0;
  int moff = 0, mbad = 0;
  if (a < A.N) {
    double c[3];
    for (int d = 0; d < 3; ++d) {
      double s = A.x[gidx<P, BEADMAJOR>(A.N, d, a, 0)];
      for (int b = 1; b < A.Pb; ++b) s = s + A.x[gidx<P, BEADMAJOR>(A.N, d, a, b)];
      c[d] = s / (double)A.Pb;
    }
    qhp::write_bins(A.bins, a, c[0], c[1], c[2]);
    for (int b = 0; b < P; ++b) {
      double xb[3];
      for (int d = 0; d < 3; ++d) xb[d] = A.x[gidx<P, BEADMAJOR>(A.N, d, a, b)];
      const double dx = xb[0] - c[0], dy = xb[1] - c[1], dz = xb[2] - c[2];
      db2 = fmax(db2, dx * dx + dy * dy + dz * dz);
      if (A.xf) A.xf[a * P + b] = make_float4((float)dx, (float)dy, (float)dz, (float)A.charge[a]);
      if (!BEADMAJOR)
        for (int d = 0; d < 3; ++d) {
          const int dl = qhp::base_diff(qhp::base_of(xb[d], A.KoL[d], A.K[d]),
                                        qhp::base_of(c[d], A.KoL[d], A.K[d]), A.K[d]);
          moff = max(moff, dl < 0 ? -dl : dl);
          if (dl > QHP_TB || dl < A.order - 1 - QHP_TB) mbad = 1;
        }
    }
    A.cent[a] = make_double4(c[0], c[1], c[2], sqrt(db2));
  }
  db2 = wave_max(db2);
  const double mo = wave_max((double)moff), mb = wave_max((double)mbad);
  if ((threadIdx.x & 63) == 0) { sm[0][threadIdx.x >> 6] = db2; sm[1][threadIdx.x >> 6] = mo; sm[2][threadIdx.x >> 6] = mb; }
  __syncthreads();
  if (threadIdx.x == 0)
    A.bmax[blockIdx.x] = make_double4(0.0, fmax(sm[0][0], sm[0][1]), fmax(sm[1][0], sm[1][1]),
                                      fmax(sm[2][0], sm[2][1]));
}

// Contracted beads of the state (modes A.x = Q): x~_j = Q_0 + sqrt(Ps) sum_{k>=1} C[j][k] Q_k,
// their FP32 offsets, the centroids Q_0 and the block maxima of the contracted beads (the
// same bookkeeping as the emitting step of the normal-mode kernel).
template <int P>
__global__ __launch_bounds__(NT) void k_contract(CentArgs A, int Ps, const double* C, double* xs) {
  constexpr int AT = NT / P;
  __shared__ double sC[P * P];
  __shared__ double sq[AT][3][P];
  __shared__ double sm[3][NT / 64];
  const int tid = threadIdx.x, al = tid / P, n = tid % P, a = blockIdx.x * AT + al;
  for (int k = tid; k < Ps * Ps; k += NT) sC[k] = C[k];
  const bool live = a < A.N;
  for (int d = 0; d < 3; ++d) sq[al][d][n] = live ? A.x[(d * A.N + a) * P + n] : 0.0;
  __syncthreads();
  double db2 = 0;
  int moff = 0, mbad = 0;
  if (live && n < Ps) {
    const double sPs = A.sPs;
    double xb[3], c[3];
    for (int d = 0; d < 3; ++d) {
      double acc = 0.0;
      for (int k = 1; k < Ps; ++k) acc += sC[n * Ps + k] * sq[al][d][k];
      c[d] = sq[al][d][0];
      xb[d] = c[d] + sPs * acc;
      xs[(d * A.N + a) * Ps + n] = xb[d];
    }
    const double dx = xb[0] - c[0], dy = xb[1] - c[1], dz = xb[2] - c[2];
    db2 = dx * dx + dy * dy + dz * dz;
    if (A.xf) A.xf[a * Ps + n] = make_float4((float)dx, (float)dy, (float)dz, (float)A.charge[a]);
    for (int d = 0; d < 3; ++d) {
      const int dl = qhp::base_diff(qhp::base_of(xb[d], A.KoL[d], A.K[d]),
                                    qhp::base_of(c[d], A.KoL[d], A.K[d]), A.K[d]);
      moff = max(moff, dl < 0 ? -dl : dl);
      if (dl > QHP_TB || dl < A.order - 1 - QHP_TB) mbad = 1;
    }
    if (n == 0) qhp::write_bins(A.bins, a, c[0], c[1], c[2]);
  }
  double adb2 = db2;                   // the atom's largest contracted-bead distance
  for (int o = 1; o < P; o <<= 1) adb2 = fmax(adb2, __shfl_xor(adb2, o));
  if (live && n == 0)
    A.cent[a] = make_double4(sq[al][0][0], sq[al][1][0], sq[al][2][0], sqrt(adb2));
  db2 = wave_max(db2);
  const double mo = wave_max((double)moff), mb = wave_max((double)mbad);
  if ((tid & 63) == 0) { sm[0][tid >> 6] = db2; sm[1][tid >> 6] = mo; sm[2][tid >> 6] = mb; }
  __syncthreads();
  if (tid == 0) {
    double b0 = sm[0][0], b1 = sm[1][0], b2 = sm[2][0];
    for (int w = 1; w < NT / 64; ++w) { b0 = fmax(b0, sm[0][w]); b1 = fmax(b1, sm[1][w]); b2 = fmax(b2, sm[2][w]); }
    A.bmax[blockIdx.x] = make_double4(0.0, b0, b1, b2);
  }
}

// boundary [Pb][N][3] <-> internal layout of P >= Pb bead lanes; phantom lanes (b >= Pb)
// receive a copy of bead 0 (a valid position whose results nothing reads)
template <bool BEADMAJOR>
__global__ void k_transpose_in(int N, int P, int Pb, const double* src, double* dst) {
  const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= (size_t)P * N * 3) return;
  int b, d, a;
  if (BEADMAJOR) { a = o % N; d = (o / N) % 3; b = o / (3 * (size_t)N); }
  else { b = o % P; a = (o / P) % N; d = o / ((size_t)P * N); }
  const size_t i = ((size_t)(b < Pb ? b : 0) * N + a) * 3 + d;
  dst[o] = src[i];
}

template <bool BEADMAJOR>
__global__ void k_transpose_out(int N, int P, int Pb, const double* src, double* dst,
                                double scale) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)Pb * N * 3) return;
  const int d = i % 3, a = (i / 3) % N, b = i / (3 * (size_t)N);
  const size_t o = BEADMAJOR ? ((size_t)b * 3 + d) * N + a : ((size_t)d * N + a) * P + b;
  dst[i] = scale * src[o];
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

static inline unsigned nblocks_atoms(int N, int P) { return (unsigned)((N + (NT / P) - 1) / (NT / P)); }

hipError_t launch_nm_step(qhp_ctx* c, int inner, double slow_h, bool emit) {
  NmArgs A;
  A.N = c->N; A.Q = c->Q; A.Pa = c->Pa; A.x = c->x; A.g = c->g; A.T = c->T;
  A.cc = c->mode_c; A.csw = c->mode_s_w; A.cws = c->mode_ws; A.c1 = c->mode_c1; A.c2 = c->mode_c2;
  A.mass = c->d_mass; A.sqrt_mkT = c->d_sqrt_mkT; A.charge = c->d_charge;
  A.type = c->d_type; A.pack_qt = c->pack_qt ? 1 : 0;
  A.cent = c->cent; A.cref = c->cref; A.coff = c->coff; A.cwrap = c->cwrap; A.xf = c->xf; A.ctrl = c->ctrl; A.bmax = c->bmax;
  for (int d = 0; d < 3; ++d) { A.K[d] = c->K[d]; A.KoL[d] = c->K[d] / c->p.box[d]; }
  A.order = c->p.pme_order;
  A.dt = c->p.dt; A.h = 0.5 * c->p.dt; A.seed = c->p.seed;
  const bool qtb = c->p.thermostat == QHP_ADQTB;
  A.noise = c->qtb.noise; A.vrec = c->qtb.vrec;
  A.nseg = qtb ? c->qtb.nseg : 1;
  A.qc1 = c->qtb.c1; A.qosd = c->qtb.osd;
  A.gs = c->gs; A.Cs = c->Cs; A.xs = c->xs; A.xfs = c->xfs; A.Ps = c->Ps;
  A.sP = sqrt((double)c->Pb); A.rsP = 1.0 / A.sP;
  A.sPs = sqrt((double)(c->Psb > 0 ? c->Psb : 1)); A.rsPs = 1.0 / A.sPs;
  A.step_off = inner; A.emit = emit ? 1 : 0; A.slow_h = slow_h;
  A.bins = bin_geom(c);
  const bool bm = c->p.exec == QHP_PLAIN;
  const bool f32 = c->p.precision == QHP_FP32_PAIRS && !bm;
  const unsigned nb = nblocks_atoms(c->N, c->P);
  c->n_bmax = (int)nb;
  if (c->respa) {
    if (bm || qtb) return hipErrorInvalidValue;
    QHP_SWITCH_P(c->P, if (f32) hipLaunchKernelGGL((k_nm_step<PP, false, false, true, true>), nb, NT, 0, c->stream, A);
                       else hipLaunchKernelGGL((k_nm_step<PP, false, false, false, true>), nb, NT, 0, c->stream, A));
    return hipGetLastError();
  }
  if (qtb) {
    if (c->P != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_nm_step<1, true, false, false>), nb, NT, 0, c->stream, A);
    return hipGetLastError();
  }
#define NM_CALL                                                                            \
  if (bm) hipLaunchKernelGGL((k_nm_step<PP, false, true, false>), nb, NT, 0, c->stream, A); \
  else if (f32) hipLaunchKernelGGL((k_nm_step<PP, false, false, true>), nb, NT, 0, c->stream, A); \
  else hipLaunchKernelGGL((k_nm_step<PP, false, false, false>), nb, NT, 0, c->stream, A);
  QHP_SWITCH_P(c->P, NM_CALL);
#undef NM_CALL
  return hipGetLastError();
}

hipError_t launch_beads_to_modes(qhp_ctx* c, const double* xb, const double* vb) {
  const unsigned nb = nblocks_atoms(c->N, c->P);
  const double rsP = 1.0 / sqrt((double)c->Pb);
  QHP_SWITCH_P(c->P, hipLaunchKernelGGL((k_to_modes<PP>), nb, NT, 0, c->stream, c->N, rsP, xb,
                                        vb, c->T, c->d_mass, c->Q, c->Pa));
  return hipGetLastError();
}

hipError_t launch_kick_back(qhp_ctx* c) {
  const unsigned nb = nblocks_atoms(c->N, c->P);
  const bool bm = c->p.exec == QHP_PLAIN;
  const double s = -0.5 * c->p.dt, rsP = 1.0 / sqrt((double)c->Pb);
  QHP_SWITCH_P(c->P, if (bm) hipLaunchKernelGGL((k_kick<PP, true>), nb, NT, 0, c->stream, c->N,
                                                 rsP, c->Pa, c->g, c->T, s);
               else hipLaunchKernelGGL((k_kick<PP, false>), nb, NT, 0, c->stream, c->N, rsP,
                                       c->Pa, c->g, c->T, s));
  return hipGetLastError();
}

hipError_t launch_state_out(qhp_ctx* c, double* xo, double* vo, const double* pa) {
  const unsigned nb = nblocks_atoms(c->N, c->P);
  const bool bm = c->p.exec == QHP_PLAIN;
  const double h = 0.5 * c->p.dt, rsP = 1.0 / sqrt((double)c->Pb);
  QHP_SWITCH_P(c->P, if (bm) hipLaunchKernelGGL((k_state_out<PP, true>), nb, NT, 0, c->stream,
                                                 c->N, c->Pb, rsP, c->Q, pa, c->g, c->T,
                                                 c->d_mass, h, xo, vo);
               else hipLaunchKernelGGL((k_state_out<PP, false>), nb, NT, 0, c->stream, c->N,
                                       c->Pb, rsP, c->Q, pa, c->g, c->T, c->d_mass, h, xo, vo));
  return hipGetLastError();
}

hipError_t launch_mode_energies(qhp_ctx* c, double* out2, const double* pa) {
  const unsigned nb = nblocks_atoms(c->N, c->P);
  const bool bm = c->p.exec == QHP_PLAIN;
  const double h = 0.5 * c->p.dt, rsP = 1.0 / sqrt((double)c->Pb);
  QHP_SWITCH_P(c->P, if (bm) hipLaunchKernelGGL((k_mode_energy<PP, true>), nb, NT, 0, c->stream,
                                                 c->N, rsP, c->Q, pa, c->g, c->T, c->d_mass,
                                                 c->mode_w2, h, out2);
               else hipLaunchKernelGGL((k_mode_energy<PP, false>), nb, NT, 0, c->stream, c->N,
                                       rsP, c->Q, pa, c->g, c->T, c->d_mass, c->mode_w2, h,
                                       out2));
  return hipGetLastError();
}

// ---- allocation-free mode energies ----
// File-scope scratch of the allocation-free entry point: the per-block partial sums of the
// kinetic and spring energies. Every GPU the library runs on holds its own copy until the
// process ends; its device address is looked up once per device (scratch_address) and the
// kernels receive that address, never the array's host-side name.
static __device__ __align__(256) double scratch[QHP_SCRATCH_DOUBLES];

hipError_t scratch_address(void** ptr) {
  static std::mutex mu;
  static void* addr[QHP_MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= QHP_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_mode_energies_noalloc(qhp_ctx* c, double* out2, const double* pa) {
  const unsigned nb = nblocks_atoms(c->N, c->P);
  if ((size_t)2 * nb > QHP_SCRATCH_DOUBLES) return hipErrorInvalidValue;   // checked by the caller
  double* parts = static_cast<double*>(c->scratch);
  const bool bm = c->p.exec == QHP_PLAIN;
  const double h = 0.5 * c->p.dt, rsP = 1.0 / sqrt((double)c->Pb);
  QHP_SWITCH_P(c->P, if (bm) hipLaunchKernelGGL((k_mode_energy_parts<PP, true>), nb, NT, 0,
                                                 c->stream, c->N, rsP, c->Q, pa, c->g, c->T,
                                                 c->d_mass, c->mode_w2, h, parts);
               else hipLaunchKernelGGL((k_mode_energy_parts<PP, false>), nb, NT, 0, c->stream,
                                       c->N, rsP, c->Q, pa, c->g, c->T, c->d_mass, c->mode_w2,
                                       h, parts));
  hipLaunchKernelGGL(k_sum_parts, 1, 256, 0, c->stream, parts, (int)nb, out2);
  return hipGetLastError();
}

size_t mode_energy_parts(const qhp_ctx* c) { return (size_t)2 * nblocks_atoms(c->N, c->P); }

hipError_t launch_kick_slow(qhp_ctx* c, double* dst, const double* src, double s) {
  const unsigned nb = nblocks_atoms(c->N, c->P);
  const double rsPs = 1.0 / sqrt((double)c->Psb);
  QHP_SWITCH_P(c->P, hipLaunchKernelGGL((k_kick_slow<PP>), nb, NT, 0, c->stream, c->N, c->Ps,
                                        rsPs, dst, src, c->gs, c->Cs, s));
  return hipGetLastError();
}

hipError_t launch_contract(qhp_ctx* c) {
  CentArgs A;
  A.N = c->N; A.x = c->Q; A.cent = c->cent; A.charge = c->d_charge; A.bmax = c->bmax;
  A.Pb = c->Pb; A.sPs = sqrt((double)c->Psb);
  A.xf = c->p.precision == QHP_FP32_PAIRS ? c->xfs : nullptr;
  A.bins = bin_geom(c);
  for (int d = 0; d < 3; ++d) { A.K[d] = c->K[d]; A.KoL[d] = c->K[d] / c->p.box[d]; }
  A.order = c->p.pme_order;
  const unsigned nb = nblocks_atoms(c->N, c->P);
  c->n_bmax = (int)nb;
  QHP_SWITCH_P(c->P, hipLaunchKernelGGL((k_contract<PP>), nb, NT, 0, c->stream, A, c->Ps,
                                        c->Cs, c->xs));
  return hipGetLastError();
}

hipError_t launch_centroid_of_beads(qhp_ctx* c) {
  const bool bm = c->p.exec == QHP_PLAIN;
  CentArgs A;
  A.N = c->N; A.x = c->x; A.cent = c->cent; A.charge = c->d_charge; A.bmax = c->bmax;
  A.Pb = c->Pb; A.sPs = 1.0;
  A.xf = (c->p.precision == QHP_FP32_PAIRS && !bm) ? c->xf : nullptr;
  A.bins = bin_geom(c);
  for (int d = 0; d < 3; ++d) { A.K[d] = c->K[d]; A.KoL[d] = c->K[d] / c->p.box[d]; }
  A.order = c->p.pme_order;
  const unsigned nb = (c->N + 127) / 128;
  c->n_bmax = (int)nb;
  QHP_SWITCH_P(c->P, if (bm) hipLaunchKernelGGL((k_centroid_beads<PP, true>), nb, 128, 0, c->stream, A);
               else hipLaunchKernelGGL((k_centroid_beads<PP, false>), nb, 128, 0, c->stream, A));
  return hipGetLastError();
}

hipError_t launch_transpose_in(qhp_ctx* c, const double* src, double* dst) {
  const size_t n = (size_t)c->P * c->N * 3;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (c->p.exec == QHP_PLAIN)
    hipLaunchKernelGGL(k_transpose_in<true>, nb, 256, 0, c->stream, c->N, c->P, c->Pb, src, dst);
  else
    hipLaunchKernelGGL(k_transpose_in<false>, nb, 256, 0, c->stream, c->N, c->P, c->Pb, src, dst);
  return hipGetLastError();
}

hipError_t launch_transpose_out(qhp_ctx* c, const double* src, double* dst, double scale) {
  const size_t n = (size_t)c->Pb * c->N * 3;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (c->p.exec == QHP_PLAIN)
    hipLaunchKernelGGL(k_transpose_out<true>, nb, 256, 0, c->stream, c->N, c->P, c->Pb, src, dst,
                       scale);
  else
    hipLaunchKernelGGL(k_transpose_out<false>, nb, 256, 0, c->stream, c->N, c->P, c->Pb, src,
                       dst, scale);
  return hipGetLastError();
}

namespace {
// The Gaussians the kernels draw: stream 5 -> [mode][atom][xyz] of one step,
// stream 6 -> [atom][xyz] of the adQTB white noise at counter c0.
__global__ void k_noise(uint64_t seed, uint64_t stream, uint64_t c0, int N, int P, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * P) return;
  const int a = t % N, n = t / N;
  double g[3];
  if (stream == qhp::STREAM_RPMD_O) qhp::gauss3(seed, stream, c0, (uint64_t)a, (uint64_t)n, g);
  else qhp::gauss3(seed, stream, c0, (uint64_t)a, 0ull, g);
  for (int d = 0; d < 3; ++d) out[((size_t)n * N + a) * 3 + d] = g[d];
}
}  // namespace

hipError_t launch_noise_export(qhp_ctx* c, int stream, int64_t step, double* out) {
  const int P = stream == 5 ? c->Pb : 1;
  const uint64_t c0 = stream == 5 ? (uint64_t)step : (uint64_t)(step + c->p.qtb_nseg);
  hipLaunchKernelGGL(k_noise, (c->N * P + 255) / 256, 256, 0, c->stream, c->p.seed,
                     (uint64_t)stream, c0, c->N, P, out);
  return hipGetLastError();
}
