// Adaptive quantum thermal bath on classical beads (P = 1): segmented coloured-noise
// generation, spectra, FDT deviation and SIMPLE adaptation (Secs. "adQTB",
// "Colored Noise Generation", "Computation of the adQTB Spectra and Adaptation Procedure").
//
// Frequency grid omega_k = pi k / (N_seg dt), k = 0..N_seg. For atom type z:
//   H_k = sqrt(2 m_z gamma_z(omega_k) Theta(omega_k) / dt), Theta(0) = kT,
//   h_j = (1/2N_seg) sum_k H_k exp(2 pi i j k / 2N_seg), j = -N_seg .. N_seg-1 (H even),
//   F_t = sum_j h_j w_{t-j}: the white noise of the previous, current and next segment
//   enters segment s. It is evaluated as a circular convolution of length 4 N_seg, which
//   is exact here because the kernel support (2 N_seg) plus the window (3 N_seg) never
//   wraps onto the outputs kept (the middle N_seg).
// White noise: Philox key (seed, 6), counter (global step + N_seg, atom, 0, 0), Gaussians
// x, y, z. Spectra at the end of a segment: X_k = DFT of the segment zero-padded to
// 2 N_seg, C_XY = (dt/N_seg) X conj(Y), Delta = m gamma C_vv - Re C_vF, averaged over the
// degrees of freedom of each type; gamma <- max(gamma_min, gamma - A_gamma Delta).
#include <algorithm>

#include "qhp_internal.h"

namespace {

constexpr int NT = 256;
// the segment kernels hold one or two whole transforms in LDS (64-128 KB), so a compute
// unit runs one or two of their blocks: 1,024 threads keep 4-8 wavefronts per SIMD
constexpr int NT_SEG = 1024;
constexpr size_t QTB_LDS_MAX = 160 * 1024;   // LDS of one compute unit (gfx950)

QHP_DEV double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Single-block Stockham FFT of runtime length L (power of two) between two LDS buffers.
// tw[m] = exp(-2 pi i m / L). Returns the buffer holding the result.
QHP_DEV double2* fft_rt(double2* a, double2* b, int L, bool inv, const double2* tw) {
  for (int Ns = 1; Ns < L;) {
    const int R = (L / Ns >= 4) ? 4 : 2;
    const int nb = L / R;
    for (int j = threadIdx.x; j < nb; j += blockDim.x) {
      const int k = j % Ns;
      double2 v[4];
      for (int r = 0; r < R; ++r) {
        v[r] = a[j + r * nb];
        if (r) {
          double2 t = tw[r * k * (L / (Ns * R))];
          if (inv) t.y = -t.y;
          v[r] = cmul(v[r], t);
        }
      }
      const int idx = (j / Ns) * Ns * R + k;
      if (R == 4) {
        const double2 t0 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
        const double2 t1 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
        const double2 t2 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
        const double2 t3 = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
        const double2 jt3 = inv ? make_double2(-t3.y, t3.x) : make_double2(t3.y, -t3.x);
        b[idx] = make_double2(t0.x + t2.x, t0.y + t2.y);
        b[idx + 2 * Ns] = make_double2(t0.x - t2.x, t0.y - t2.y);
        b[idx + Ns] = make_double2(t1.x + jt3.x, t1.y + jt3.y);
        b[idx + 3 * Ns] = make_double2(t1.x - jt3.x, t1.y - jt3.y);
      } else {
        b[idx] = make_double2(v[0].x + v[1].x, v[0].y + v[1].y);
        b[idx + Ns] = make_double2(v[0].x - v[1].x, v[0].y - v[1].y);
      }
    }
    __syncthreads();
    double2* t = a; a = b; b = t;
    Ns *= R;
  }
  return a;
}

struct KerArgs {
  int nseg;
  const double* gamma;    // [T][nseg+1]
  const double* tmass;    // [T]
  double kT, hbar, dt;
  int classical;
  const double2* tw2; const double2* tw4;
  double2* hhat;          // [T][4 nseg]
};

// one block per type: H -> h (inverse DFT of length 2N) -> embed -> DFT of length 4N
__global__ __launch_bounds__(NT) void k_qtb_kernel(KerArgs A) {
  extern __shared__ double2 lds[];
  const int z = blockIdx.x, N = A.nseg, L2 = 2 * N, L4 = 4 * N;
  double2* a = lds;
  double2* b = lds + L4;
  const double m = A.tmass[z];
  const double* gz = A.gamma + (size_t)z * (N + 1);
  for (int k = threadIdx.x; k < L2; k += blockDim.x) {
    const int kk = k <= N ? k : L2 - k;
    const double om = M_PI * kk / (N * A.dt);
    double th = A.kT;
    if (!A.classical && kk > 0) {
      const double x = A.hbar * om;
      th = 0.5 * x / tanh(0.5 * x / A.kT);
    }
    a[k] = make_double2(sqrt(2.0 * m * gz[kk] * th / A.dt), 0.0);
  }
  __syncthreads();
  double2* h = fft_rt(a, b, L2, true, A.tw2);       // unnormalised inverse
  double2* o = (h == a) ? b : a;
  for (int l = threadIdx.x; l < L4; l += blockDim.x) {
    double v = 0.0;
    if (l < N) v = h[l].x;                    // j = l
    else if (l >= 3 * N) v = h[l - 2 * N].x;  // j = l - 4N, stored at 2N + j
    o[l] = make_double2(v / L2, 0.0);
  }
  __syncthreads();
  double2* other = (o == a) ? b : a;
  double2* H = fft_rt(o, other, L4, false, A.tw4);
  for (int l = threadIdx.x; l < L4; l += blockDim.x) A.hhat[(size_t)z * L4 + l] = H[l];
}

struct GenArgs {
  int N, nseg;
  uint64_t seed;
  int64_t seg;
  const int* type;
  const double2* hhat;
  const double2* tw4;
  double* noise;          // [nseg][3][N]
};

// One block per atom: the window's white noise is drawn once (each Philox counter gives
// the x, y and z Gaussians), then x + i y and z + 0 i are convolved with the type's
// kernel in turn, in the same two LDS buffers; the z samples wait in a third array.
__global__ __launch_bounds__(NT_SEG) void k_qtb_generate(GenArgs A) {
  extern __shared__ double2 lds[];
  const int a = blockIdx.x;
  const int Ns = A.nseg, L4 = 4 * Ns;
  double2* u = lds;
  double2* v = lds + L4;
  double* zs = reinterpret_cast<double*>(lds + 2 * L4);   // [3 Ns]
  const uint64_t c0 = (uint64_t)(A.seg * Ns);   // counter of window sample 0
  for (int l = threadIdx.x; l < L4; l += blockDim.x) {
    double2 w = make_double2(0.0, 0.0);
    if (l < 3 * Ns) {
      double gs[3];
      qhp::gauss3(A.seed, qhp::STREAM_QTB_WHITE, c0 + (uint64_t)l, (uint64_t)a, 0ull, gs);
      w = make_double2(gs[0], gs[1]);
      zs[l] = gs[2];
    }
    u[l] = w;
  }
  __syncthreads();
  const double2* Hz = A.hhat + (size_t)A.type[a] * L4;
  const double inv = 1.0 / L4;
  for (int slot = 0; slot < 2; ++slot) {
    if (slot == 1) {
      for (int l = threadIdx.x; l < L4; l += blockDim.x)
        u[l] = l < 3 * Ns ? make_double2(zs[l], 0.0) : make_double2(0.0, 0.0);
      __syncthreads();
    }
    double2* W = fft_rt(u, v, L4, false, A.tw4);
    for (int l = threadIdx.x; l < L4; l += blockDim.x) W[l] = cmul(W[l], Hz[l]);
    __syncthreads();
    double2* other = (W == u) ? v : u;
    double2* C = fft_rt(W, other, L4, true, A.tw4);
    for (int t = threadIdx.x; t < Ns; t += blockDim.x) {
      const double2 f = C[Ns + t];
      if (slot == 0) {
        A.noise[((size_t)t * 3 + 0) * A.N + a] = f.x * inv;
        A.noise[((size_t)t * 3 + 1) * A.N + a] = f.y * inv;
      } else {
        A.noise[((size_t)t * 3 + 2) * A.N + a] = f.x * inv;
      }
    }
    __syncthreads();                  // C is read before u is refilled
  }
}

struct SpecArgs {
  int N, nseg, ntypes, dofs_per_block;
  int z0;                 // the launch accumulates types z0 .. z0 + ntypes - 1 only
  const int* type;
  const double* mass;
  const double* gamma;
  const double* vrec; const double* noise;
  const double2* tw2;
  double dt;
  double* dsum;           // [T][nseg+1] summed Delta_FDT
  double* vvsum;          // [T][nseg+1] summed C_vv (RATIO only)
  double* vfsum;          // [T][nseg+1] summed Re C_vF (RATIO only)
  int ratio;
};

__global__ __launch_bounds__(NT_SEG) void k_qtb_spectra(SpecArgs A) {
  extern __shared__ double2 lds[];
  const int Ns = A.nseg, L2 = 2 * Ns;
  double2* u = lds;
  double2* v = lds + L2;
  const int nk = A.ntypes * (Ns + 1);
  double* acc = (double*)(lds + 2 * L2);     // [types][nseg+1] Delta; then C_vv, Re C_vF
  double* avv = acc + nk;
  double* avf = avv + nk;
  for (int k = threadIdx.x; k < (A.ratio ? 3 : 1) * nk; k += blockDim.x) acc[k] = 0.0;
  const int ndof = 3 * A.N;
  const int d0 = blockIdx.x * A.dofs_per_block;
  const double sc = A.dt / Ns;
  for (int dof = d0; dof < min(ndof, d0 + A.dofs_per_block); ++dof) {
    const int d = dof % 3, a = dof / 3;
    const int ty = A.type[a] - A.z0;
    if (ty < 0 || ty >= A.ntypes) continue;            // another launch's type (uniform)
    for (int t = threadIdx.x; t < L2; t += blockDim.x) {
      double2 z = make_double2(0.0, 0.0);
      if (t < Ns) {
        const size_t i = ((size_t)t * 3 + d) * A.N + a;
        z = make_double2(A.vrec[i], A.noise[i]);
      }
      u[t] = z;
    }
    __syncthreads();
    double2* Z = fft_rt(u, v, L2, false, A.tw2);
    const double m = A.mass[a];
    const double* gz = A.gamma + (size_t)(ty + A.z0) * (Ns + 1);
    for (int k = threadIdx.x; k <= Ns; k += blockDim.x) {
      const double2 zk = Z[k], zm = Z[(L2 - k) % L2];
      // V = (Z_k + conj Z_-k) / 2, F = (Z_k - conj Z_-k) / 2i
      const double vr = 0.5 * (zk.x + zm.x), vi = 0.5 * (zk.y - zm.y);
      const double fr = 0.5 * (zk.y + zm.y), fi = -0.5 * (zk.x - zm.x);
      const double cvv = sc * (vr * vr + vi * vi);
      const double cvf = sc * (vr * fr + vi * fi);       // Re(V conj F)
      acc[ty * (Ns + 1) + k] += m * gz[k] * cvv - cvf;
      if (A.ratio) {
        avv[ty * (Ns + 1) + k] += cvv;
        avf[ty * (Ns + 1) + k] += cvf;
      }
    }
    __syncthreads();
  }
  const size_t o = (size_t)A.z0 * (Ns + 1);
  for (int k = threadIdx.x; k < nk; k += blockDim.x) {
    if (acc[k] != 0.0) atomicAdd(A.dsum + o + k, acc[k]);
    if (A.ratio) {
      if (avv[k] != 0.0) atomicAdd(A.vvsum + o + k, avv[k]);
      if (avf[k] != 0.0) atomicAdd(A.vfsum + o + k, avf[k]);
    }
  }
}

// SIMPLE: gamma <- max(gamma_min, gamma - A Delta_bar). RATIO: the running means
// <C> <- <C> decay + C_bar (1 - decay) of C_vv and Re C_vF, then gamma <- max(gamma_min,
// Re<C_vF> / (m <C_vv>)) where <C_vv> > 0. Keep Delta_bar for export; clear the sums.
struct AdaptArgs {
  int n, nseg, ratio;
  double* gamma; double* dsum; double* dbar; double* vvsum; double* vfsum;
  double* avg_vv; double* avg_vf;
  const double* inv_count; const double* tmass;
  double rate, gmin, decay;
};

__global__ void k_qtb_adapt(AdaptArgs A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int z = i / (A.nseg + 1);
  const double ic = A.inv_count[z];
  const double d = A.dsum[i] * ic;
  A.dbar[i] = d;
  double g = A.gamma[i] - A.rate * d;
  if (A.ratio) {
    const double vv = A.avg_vv[i] * A.decay + A.vvsum[i] * ic * (1.0 - A.decay);
    const double vf = A.avg_vf[i] * A.decay + A.vfsum[i] * ic * (1.0 - A.decay);
    A.avg_vv[i] = vv;
    A.avg_vf[i] = vf;
    g = vv > 0.0 ? vf / (A.tmass[z] * vv) : A.gamma[i];
    A.vvsum[i] = 0.0;
    A.vfsum[i] = 0.0;
  }
  A.gamma[i] = fmax(A.gmin, g);
  A.dsum[i] = 0.0;
}

__global__ void k_fill(double* p, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t qtb_build_kernels(qhp_ctx* c) {
  QtbState& q = c->qtb;
  KerArgs A;
  A.nseg = q.nseg; A.gamma = q.gamma; A.tmass = q.d_tmass; A.kT = c->p.kT; A.hbar = c->p.hbar;
  A.dt = c->p.dt; A.classical = c->p.qtb_classical; A.tw2 = q.tw2; A.tw4 = q.tw4; A.hhat = q.hhat;
  const size_t lds = (size_t)8 * q.nseg * sizeof(double2);
  hipLaunchKernelGGL(k_qtb_kernel, c->p.n_types, NT, lds, c->stream, A);
  return hipGetLastError();
}

hipError_t launch_qtb_generate(qhp_ctx* c, int64_t seg) {
  QtbState& q = c->qtb;
  hipError_t e = qtb_build_kernels(c);
  if (e != hipSuccess) return e;
  GenArgs A;
  A.N = c->N; A.nseg = q.nseg; A.seed = c->p.seed; A.seg = seg; A.type = c->d_type;
  A.hhat = q.hhat; A.tw4 = q.tw4; A.noise = q.noise;
  // two transforms of 4 N_seg points and the window's z samples: 152 KB at N_seg = 1024
  const size_t lds = (size_t)8 * q.nseg * sizeof(double2) + (size_t)3 * q.nseg * sizeof(double);
  hipLaunchKernelGGL(k_qtb_generate, c->N, NT_SEG, lds, c->stream, A);
  return hipGetLastError();
}

hipError_t launch_qtb_adapt(qhp_ctx* c) {
  QtbState& q = c->qtb;
  SpecArgs A;
  A.N = c->N; A.nseg = q.nseg; A.dofs_per_block = 32;
  A.type = c->d_type; A.mass = c->d_mass; A.gamma = q.gamma; A.vrec = q.vrec; A.noise = q.noise;
  A.tw2 = q.tw2; A.dt = c->p.dt; A.dsum = q.dsum;
  A.vvsum = q.vvsum; A.vfsum = q.vfsum;
  A.ratio = c->p.qtb_adapt_scheme == QHP_QTB_RATIO;
  const int nb = (3 * c->N + A.dofs_per_block - 1) / A.dofs_per_block;
  // the per-type accumulators share the block's LDS with the two transform buffers: types
  // that do not fit together are accumulated by further launches (each skips the others)
  const size_t fft_lds = (size_t)4 * q.nseg * sizeof(double2);
  const size_t per_type = (size_t)(A.ratio ? 3 : 1) * (q.nseg + 1) * sizeof(double);
  const int fit = (int)std::max<size_t>(1, (QTB_LDS_MAX - fft_lds) / per_type);
  for (int z0 = 0; z0 < c->p.n_types; z0 += fit) {
    A.z0 = z0;
    A.ntypes = std::min(fit, c->p.n_types - z0);
    hipLaunchKernelGGL(k_qtb_spectra, nb, NT_SEG, fft_lds + A.ntypes * per_type, c->stream, A);
  }
  AdaptArgs D;
  D.n = c->p.n_types * (q.nseg + 1); D.nseg = q.nseg; D.ratio = A.ratio;
  D.gamma = q.gamma; D.dsum = q.dsum; D.dbar = q.dbar; D.vvsum = q.vvsum; D.vfsum = q.vfsum;
  D.avg_vv = q.avg_vv; D.avg_vf = q.avg_vf; D.inv_count = q.d_inv_count; D.tmass = q.d_tmass;
  D.rate = c->p.qtb_adapt_rate; D.gmin = c->p.qtb_gamma_min_frac * c->p.qtb_gamma0;
  D.decay = A.ratio ? std::exp(-q.nseg * c->p.dt / c->p.qtb_tau) : 0.0;
  hipLaunchKernelGGL(k_qtb_adapt, (D.n + 255) / 256, 256, 0, c->stream, D);
  return hipGetLastError();
}

hipError_t qtb_reset_gamma(qhp_ctx* c) {
  const int n = c->p.n_types * (c->qtb.nseg + 1);
  hipLaunchKernelGGL(k_fill, (n + 255) / 256, 256, 0, c->stream, c->qtb.gamma, n, c->p.qtb_gamma0);
  hipLaunchKernelGGL(k_fill, (n + 255) / 256, 256, 0, c->stream, c->qtb.dsum, n, 0.0);
  if (c->qtb.avg_vv) {
    for (double* p : {c->qtb.vvsum, c->qtb.vfsum, c->qtb.avg_vv, c->qtb.avg_vf})
      hipLaunchKernelGGL(k_fill, (n + 255) / 256, 256, 0, c->stream, p, n, 0.0);
  }
  return hipGetLastError();
}
