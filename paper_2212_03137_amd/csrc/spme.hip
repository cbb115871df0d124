// Smooth particle-mesh Ewald reciprocal sum for all beads (Essmann et al., J. Chem. Phys.
// 103, 8577, 1995): order-n cardinal B-spline charge spreading, 3D FFT, multiplication
// by the influence function G(m) = C/(pi V) exp(-pi^2 m^2/alpha^2)/m^2 B(m), inverse FFT,
// and the force gather with spline derivatives. E = 1/2 sum_i q_i phi(r_i) is formed in
// the gather.
//
// Bead batching: grids are stored bead innermost, grid[k0][k1][k2][b]. Read as complex
// numbers, beads 2c and 2c+1 form the real and imaginary parts of complex slot c; since
// G is real and even, one complex transform pair convolves both real grids exactly
// (P = 1 leaves the imaginary part zero). Every FFT pass therefore reads 256-byte rows
// (16 complex beads at P = 32) and needs no R2C/C2R bookkeeping.
//
// FFT: five passes over the grid; each pass loads 4096 complex values (4096/K series of
// length K along one axis) into LDS and runs a radix-4 (+ final radix-2) Stockham FFT
// there; the z pass does forward transform, multiplication by G and inverse transform in
// one visit.
#include "qhp_internal.h"

namespace {

constexpr int NT = 256;

struct SpmeArgs {
  int N;
  int K0, K1, K2;
  int Pc2;                 // doubles per grid point (2 * complex slots)
  const double* x; double* g;
  double* grid;
  const double* charge;
  double L[3];
  double* energy;
};

template <int ORDER>
QHP_DEV void bspline(double frac, double* w, double* dw) {
  double m[ORDER];
#pragma unroll
  for (int t = 0; t < ORDER; ++t) m[t] = 0.0;
  m[0] = frac;
  m[1] = 1.0 - frac;
#pragma unroll
  for (int k = 3; k <= ORDER; ++k) {
    if (k == ORDER) {
      dw[0] = m[0];
#pragma unroll
      for (int t = 1; t < ORDER; ++t) dw[t] = m[t] - m[t - 1];
    }
    const double inv = 1.0 / (double)(k - 1);
#pragma unroll
    for (int t = k - 1; t >= 1; --t)
      m[t] = ((frac + t) * m[t] + ((double)k - frac - t) * m[t - 1]) * inv;
    m[0] = frac * m[0] * inv;
  }
#pragma unroll
  for (int t = 0; t < ORDER; ++t) w[t] = m[t];
}

template <int ORDER>
QHP_DEV void stencil(const double* xb, const double* L, const int* K, int* i0, double (*w)[ORDER],
                     double (*dw)[ORDER]) {
  for (int d = 0; d < 3; ++d) {
    double s = xb[d] / L[d];
    s = s - floor(s);
    const double u = s * (double)K[d];
    const double fl = floor(u);
    // a non-finite coordinate must not turn into an out-of-range grid index
    i0[d] = isfinite(fl) ? min(max((int)fl, 0), K[d]) : 0;
    bspline<ORDER>(u - fl, w[d], dw[d]);
  }
}

QHP_DEV int wrapk(int k, int K) { return k < 0 ? k + K : (k >= K ? k - K : k); }

template <int P, int ORDER>
__global__ __launch_bounds__(NT) void k_spread(SpmeArgs A) {
  const int tid = blockIdx.x * NT + threadIdx.x;
  const int a = tid / P, b = tid % P;
  if (a >= A.N) return;
  double xb[3];
  for (int d = 0; d < 3; ++d) xb[d] = A.x[(d * A.N + a) * P + b];
  const int K[3] = {A.K0, A.K1, A.K2};
  int i0[3];
  double w[3][ORDER], dw[3][ORDER];
  stencil<ORDER>(xb, A.L, K, i0, w, dw);
  const double q = A.charge[a];
  for (int t0 = 0; t0 < ORDER; ++t0) {
    const int k0 = wrapk(i0[0] - t0, A.K0);
    const double w0 = q * w[0][t0];
    for (int t1 = 0; t1 < ORDER; ++t1) {
      const int k1 = wrapk(i0[1] - t1, A.K1);
      const double w01 = w0 * w[1][t1];
      double* row = A.grid + ((size_t)(k0 * A.K1 + k1) * A.K2) * A.Pc2 + b;
#pragma unroll
      for (int t2 = 0; t2 < ORDER; ++t2) {
        const int k2 = wrapk(i0[2] - t2, A.K2);
        unsafeAtomicAdd(row + (size_t)k2 * A.Pc2, w01 * w[2][t2]);
      }
    }
  }
}

template <int P, int ORDER, bool ENERGY>
__global__ __launch_bounds__(NT) void k_gather(SpmeArgs A) {
  __shared__ double sred[NT];
  const int tid = blockIdx.x * NT + threadIdx.x;
  const int a = tid / P, b = tid % P;
  double e = 0;
  if (a < A.N) {
    double xb[3];
    for (int d = 0; d < 3; ++d) xb[d] = A.x[(d * A.N + a) * P + b];
    const int K[3] = {A.K0, A.K1, A.K2};
    int i0[3];
    double w[3][ORDER], dw[3][ORDER];
    stencil<ORDER>(xb, A.L, K, i0, w, dw);
    double f0 = 0, f1 = 0, f2 = 0;
    for (int t0 = 0; t0 < ORDER; ++t0) {
      const int k0 = wrapk(i0[0] - t0, A.K0);
      for (int t1 = 0; t1 < ORDER; ++t1) {
        const int k1 = wrapk(i0[1] - t1, A.K1);
        const double* row = A.grid + ((size_t)(k0 * A.K1 + k1) * A.K2) * A.Pc2 + b;
        double s = 0, sd = 0;
#pragma unroll
        for (int t2 = 0; t2 < ORDER; ++t2) {
          const int k2 = wrapk(i0[2] - t2, A.K2);
          const double ph = row[(size_t)k2 * A.Pc2];
          s += w[2][t2] * ph;
          sd += dw[2][t2] * ph;
        }
        f0 += dw[0][t0] * w[1][t1] * s;
        f1 += w[0][t0] * dw[1][t1] * s;
        f2 += w[0][t0] * w[1][t1] * sd;
        if (ENERGY) e += w[0][t0] * w[1][t1] * s;
      }
    }
    const double q = A.charge[a];
    A.g[(0 * A.N + a) * P + b] += q * f0 * (double)A.K0 / A.L[0];
    A.g[(1 * A.N + a) * P + b] += q * f1 * (double)A.K1 / A.L[1];
    A.g[(2 * A.N + a) * P + b] += q * f2 * (double)A.K2 / A.L[2];
    e *= 0.5 * q;
  }
  if (ENERGY) {
    constexpr int AT = NT / P;
    const int t = threadIdx.x;
    sred[t] = e;
    __syncthreads();
    for (int s = AT / 2; s > 0; s >>= 1) {
      if (t / P < s) sred[t] += sred[t + s * P];
      __syncthreads();
    }
    if (t < P) atomicAdd(A.energy + t * QHP_NTERMS + QHP_E_COUL_RECIP, sred[t]);
  }
}

// ------------------------------- LDS Stockham FFT -------------------------------------
QHP_DEV double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
QHP_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
QHP_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Element e of series s lives at buf[e * NS + s]; NS * K = 4096.
template <int K, int NS, bool INV, int NSTRIDE>
QHP_DEV void fft_stages(double2* buf, const double2* tw, int tid) {
  if constexpr (NSTRIDE < K) {
    constexpr int R = (K / NSTRIDE >= 4) ? 4 : 2;
    constexpr int BPT = NS * K / R / NT;
    double2 v[BPT][R];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int be = tid + i * NT, s = be % NS, j = be / NS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[(j + r * (K / R)) * NS + s];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int be = tid + i * NT, s = be % NS, j = be / NS;
      const int k = j % NSTRIDE;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double2 t = tw[r * k * (K / (NSTRIDE * R))];
        if (INV) t.y = -t.y;
        v[i][r] = cmul(v[i][r], t);
      }
      double2 y[R];
      if constexpr (R == 4) {
        const double2 t0 = cadd(v[i][0], v[i][2]), t1 = csub(v[i][0], v[i][2]);
        const double2 t2 = cadd(v[i][1], v[i][3]), t3 = csub(v[i][1], v[i][3]);
        // -i * t3 (forward) or +i * t3 (inverse)
        const double2 jt3 = INV ? make_double2(-t3.y, t3.x) : make_double2(t3.y, -t3.x);
        y[0] = cadd(t0, t2);
        y[2] = csub(t0, t2);
        y[1] = cadd(t1, jt3);
        y[3] = csub(t1, jt3);
      } else {
        y[0] = cadd(v[i][0], v[i][1]);
        y[1] = csub(v[i][0], v[i][1]);
      }
      const int idx = (j / NSTRIDE) * NSTRIDE * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(idx + r * NSTRIDE) * NS + s] = y[r];
    }
    __syncthreads();
    fft_stages<K, NS, INV, NSTRIDE * R>(buf, tw, tid);
  }
}

struct FftArgs {
  double2* grid;
  const double2* tw;       // [K] exp(-2 pi i m / K)
  const double* G;         // influence [K0][K1][K2] (fused z pass)
  long inner;              // complex elements below the axis (stride of the axis)
  int pc;                  // complex slots per grid point
  int efast;               // load order
};

// MODE 0: forward, 1: inverse, 2: forward, x G, inverse (axis 2 only)
template <int K, int MODE>
__global__ __launch_bounds__(NT) void k_fft_pass(FftArgs A) {
  constexpr int NS = 4096 / K;
  __shared__ double2 buf[4096];
  __shared__ double2 stw[K];
  const int tid = threadIdx.x;
  for (int m = tid; m < K; m += NT) stw[m] = A.tw[m];
  const long m0 = (long)blockIdx.x * NS;
  const long I = A.inner;
  for (int l = tid; l < 4096; l += NT) {
    const int e = A.efast ? l % K : l / NS;
    const int s = A.efast ? l / K : l % NS;
    const long m = m0 + s;
    buf[e * NS + s] = A.grid[(m / I) * (K * I) + (m % I) + (long)e * I];
  }
  __syncthreads();
  if (MODE == 1) {
    fft_stages<K, NS, true, 1>(buf, stw, tid);
  } else {
    fft_stages<K, NS, false, 1>(buf, stw, tid);
  }
  if (MODE == 2) {
    for (int l = tid; l < 4096; l += NT) {
      const int e = l / NS, s = l % NS;
      const long p = (m0 + s) / A.pc;
      const double gv = A.G[p * K + e];
      double2 v = buf[e * NS + s];
      v.x *= gv; v.y *= gv;
      buf[e * NS + s] = v;
    }
    __syncthreads();
    fft_stages<K, NS, true, 1>(buf, stw, tid);
  }
  for (int l = tid; l < 4096; l += NT) {
    const int e = A.efast ? l % K : l / NS;
    const int s = A.efast ? l / K : l % NS;
    const long m = m0 + s;
    A.grid[(m / I) * (K * I) + (m % I) + (long)e * I] = buf[e * NS + s];
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

#define QHP_SWITCH_ORDER(O, CALL)                      \
  switch (O) {                                         \
    case 4: { constexpr int OO = 4; CALL; } break;     \
    case 5: { constexpr int OO = 5; CALL; } break;     \
    case 6: { constexpr int OO = 6; CALL; } break;     \
    case 8: { constexpr int OO = 8; CALL; } break;     \
    default: return hipErrorInvalidValue;              \
  }

#define QHP_SWITCH_K(K, CALL)                          \
  switch (K) {                                         \
    case 8: { constexpr int KK = 8; CALL; } break;     \
    case 16: { constexpr int KK = 16; CALL; } break;   \
    case 32: { constexpr int KK = 32; CALL; } break;   \
    case 64: { constexpr int KK = 64; CALL; } break;   \
    case 128: { constexpr int KK = 128; CALL; } break; \
    case 256: { constexpr int KK = 256; CALL; } break; \
    default: return hipErrorInvalidValue;              \
  }

static hipError_t fft_pass(qhp_ctx* c, int axis, int mode, int pc) {
  const int K = c->K[axis];
  long inner = pc;
  for (int d = axis + 1; d < 3; ++d) inner *= c->K[d];
  const long total = (long)c->K[0] * c->K[1] * c->K[2] * pc;
  const long series = total / K;
  const int NS = 4096 / K;
  if (series % NS) return hipErrorInvalidValue;
  FftArgs A;
  A.grid = c->grid; A.tw = c->tw[axis]; A.G = c->influence; A.inner = inner; A.pc = pc;
  A.efast = inner < 16;
  const unsigned nb = (unsigned)(series / NS);
  if (mode == 0) { QHP_SWITCH_K(K, hipLaunchKernelGGL((k_fft_pass<KK, 0>), nb, NT, 0, c->stream, A)); }
  else if (mode == 1) { QHP_SWITCH_K(K, hipLaunchKernelGGL((k_fft_pass<KK, 1>), nb, NT, 0, c->stream, A)); }
  else { QHP_SWITCH_K(K, hipLaunchKernelGGL((k_fft_pass<KK, 2>), nb, NT, 0, c->stream, A)); }
  return hipGetLastError();
}

hipError_t launch_spme(qhp_ctx* c, bool energy, int bead) {
  const bool plain = bead >= 0;
  const int P = plain ? 1 : c->P;
  const int pc = plain ? 1 : c->Pc;
  const int N = c->N;
  SpmeArgs A;
  A.N = N; A.K0 = c->K[0]; A.K1 = c->K[1]; A.K2 = c->K[2]; A.Pc2 = 2 * pc;
  A.x = plain ? c->x + (size_t)bead * 3 * N : c->x;
  A.g = plain ? c->g + (size_t)bead * 3 * N : c->g;
  A.grid = (double*)c->grid; A.charge = c->d_charge;
  for (int d = 0; d < 3; ++d) A.L[d] = c->p.box[d];
  A.energy = c->energy + (plain ? (size_t)bead * QHP_NTERMS : 0);
  const size_t gbytes = (size_t)c->K[0] * c->K[1] * c->K[2] * pc * sizeof(double2);
  hipError_t e = launch_zero(c, c->grid, gbytes);
  if (e != hipSuccess) return e;
  const unsigned nb = (unsigned)(((size_t)N * P + NT - 1) / NT);
  hipEvent_t ev = nullptr;
  prof_begin(c, QHP_PROF_SPREAD, &ev);
  QHP_SWITCH_P(P, QHP_SWITCH_ORDER(c->p.pme_order,
               hipLaunchKernelGGL((k_spread<PP, OO>), nb, NT, 0, c->stream, A)));
  prof_end(c, QHP_PROF_SPREAD, ev);
  prof_begin(c, QHP_PROF_FFT, &ev);
  if ((e = fft_pass(c, 0, 0, pc)) != hipSuccess) return e;
  if ((e = fft_pass(c, 1, 0, pc)) != hipSuccess) return e;
  if ((e = fft_pass(c, 2, 2, pc)) != hipSuccess) return e;
  if ((e = fft_pass(c, 1, 1, pc)) != hipSuccess) return e;
  if ((e = fft_pass(c, 0, 1, pc)) != hipSuccess) return e;
  prof_end(c, QHP_PROF_FFT, ev);
  prof_begin(c, QHP_PROF_GATHER, &ev);
  QHP_SWITCH_P(P, QHP_SWITCH_ORDER(c->p.pme_order,
               if (energy) hipLaunchKernelGGL((k_gather<PP, OO, true>), nb, NT, 0, c->stream, A);
               else hipLaunchKernelGGL((k_gather<PP, OO, false>), nb, NT, 0, c->stream, A)));
  prof_end(c, QHP_PROF_GATHER, ev);
  return hipGetLastError();
}
