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
constexpr size_t QTB_LDS_MAX = 160 * 1024;   // LDS of one compute unit (gfx950)

QHP_DEV double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
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
  double2* h = qhp::fft_rt(a, b, L2, 1, true, A.tw2);       // unnormalised inverse
  double2* o = (h == a) ? b : a;
  for (int l = threadIdx.x; l < L4; l += blockDim.x) {
    double v = 0.0;
    if (l < N) v = h[l].x;                    // j = l
    else if (l >= 3 * N) v = h[l - 2 * N].x;  // j = l - 4N, stored at 2N + j
    o[l] = make_double2(v / L2, 0.0);
  }
  __syncthreads();
  double2* other = (o == a) ? b : a;
  double2* H = qhp::fft_rt(o, other, L4, 1, false, A.tw4);
  for (int l = threadIdx.x; l < L4; l += blockDim.x) A.hhat[(size_t)z * L4 + l] = H[l];
}

// ---- in-place transforms of one whole series per block ----
// Twiddle exp(-2 pi i m / L) from a two-level table: w(m) = hi[m >> LG] lo[m & (2^LG - 1)]
// with hi[k] = w(k 2^LG) and lo[k] = w(k), both taken from the host's table of length L.
template <int LG>
QHP_DEV double2 twid(const double2* hi, const double2* lo, int m) {
  return cmul(hi[m >> LG], lo[m & ((1 << LG) - 1)]);
}

QHP_DEV void dft4r(double2& a0, double2& a1, double2& a2, double2& a3, bool inv) {
  const double2 t0 = make_double2(a0.x + a2.x, a0.y + a2.y);
  const double2 t1 = make_double2(a0.x - a2.x, a0.y - a2.y);
  const double2 t2 = make_double2(a1.x + a3.x, a1.y + a3.y);
  const double2 t3 = make_double2(a1.x - a3.x, a1.y - a3.y);
  const double2 jt3 = inv ? make_double2(-t3.y, t3.x) : make_double2(t3.y, -t3.x);
  a0 = make_double2(t0.x + t2.x, t0.y + t2.y);
  a2 = make_double2(t0.x - t2.x, t0.y - t2.y);
  a1 = make_double2(t1.x + jt3.x, t1.y + jt3.y);
  a3 = make_double2(t1.x - jt3.x, t1.y - jt3.y);
}

// Stockham transform of length L (a power of two) in place in buf: each stage reads its
// butterflies' operands into registers, waits for the block, and writes the results in
// natural order; radix 8 while at least eight points remain per sub-transform, then 4 and
// 2. NTH threads; unnormalised; exp(+...) when INV.
template <int L, int NTH, bool INV, int LG, int NSTRIDE = 1>
QHP_DEV void fft_inplace(double2* buf, const double2* hi, const double2* lo) {
  if constexpr (NSTRIDE < L) {
    constexpr int R = (L / NSTRIDE >= 8) ? 8 : ((L / NSTRIDE >= 4) ? 4 : 2);
    constexpr int NB = L / R;                        // butterflies
    constexpr int BPT = (NB + NTH - 1) / NTH;
    const int tid = threadIdx.x;
    double2 v[BPT][R];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int j = tid + i * NTH;
      if (NB % NTH != 0 && j >= NB) break;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[j + r * NB];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int j = tid + i * NTH;
      if (NB % NTH != 0 && j >= NB) break;
      const int k = j % NSTRIDE;
      if constexpr (NSTRIDE > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double2 t = twid<LG>(hi, lo, r * k * (L / (NSTRIDE * R)));
          if (INV) t.y = -t.y;
          v[i][r] = cmul(v[i][r], t);
        }
      }
      if constexpr (R == 8) {
        dft4r(v[i][0], v[i][2], v[i][4], v[i][6], INV);
        dft4r(v[i][1], v[i][3], v[i][5], v[i][7], INV);
        const double h = 0.70710678118654752440;
        const double sg = INV ? 1.0 : -1.0;          // W8 = (1 + sg i) / sqrt(2)
        const double2 o0 = v[i][1];
        const double2 o1 = cmul(v[i][3], make_double2(h, sg * h));
        const double2 o2 = cmul(v[i][5], make_double2(0.0, sg));
        const double2 o3 = cmul(v[i][7], make_double2(-h, sg * h));
        const double2 e0 = v[i][0], e1 = v[i][2], e2 = v[i][4], e3 = v[i][6];
        v[i][0] = make_double2(e0.x + o0.x, e0.y + o0.y); v[i][4] = make_double2(e0.x - o0.x, e0.y - o0.y);
        v[i][1] = make_double2(e1.x + o1.x, e1.y + o1.y); v[i][5] = make_double2(e1.x - o1.x, e1.y - o1.y);
        v[i][2] = make_double2(e2.x + o2.x, e2.y + o2.y); v[i][6] = make_double2(e2.x - o2.x, e2.y - o2.y);
        v[i][3] = make_double2(e3.x + o3.x, e3.y + o3.y); v[i][7] = make_double2(e3.x - o3.x, e3.y - o3.y);
      } else if constexpr (R == 4) {
        dft4r(v[i][0], v[i][1], v[i][2], v[i][3], INV);
      } else {
        const double2 a = v[i][0], b = v[i][1];
        v[i][0] = make_double2(a.x + b.x, a.y + b.y);
        v[i][1] = make_double2(a.x - b.x, a.y - b.y);
      }
      const int idx = (j / NSTRIDE) * NSTRIDE * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[idx + r * NSTRIDE] = v[i][r];
    }
    __syncthreads();
    fft_inplace<L, NTH, INV, LG, NSTRIDE * R>(buf, hi, lo);
  }
}

// split of log2(L) for the two-level twiddles
template <int L>
constexpr int tw_lg() { return (__builtin_ctz(L) + 1) / 2; }

template <int L>
QHP_DEV void load_twiddles(double2* hi, double2* lo, const double2* tw) {
  constexpr int LG = tw_lg<L>();
  for (int k = threadIdx.x; k < (1 << LG); k += blockDim.x) lo[k] = tw[k];
  for (int k = threadIdx.x; k < L >> LG; k += blockDim.x) hi[k] = tw[k << LG];
}

// [t][3][N] <-> [t / 8][N][3][8] (qtb_rec) for a segment: a block takes 8 steps of 64 atoms,
// reading and writing contiguous runs on both sides through LDS. TO_TILES: per-step to
// segment layout.
template <bool TO_TILES>
__global__ __launch_bounds__(256) void k_qtb_transpose(const double* src, double* dst, int N) {
  __shared__ double sm[8][3][65];
  const int t8 = blockIdx.y, a0 = blockIdx.x * 64, tid = threadIdx.x;
  if (TO_TILES) {
    for (int k = tid; k < 8 * 3 * 64; k += 256) {          // rows of 64 atoms
      const int al = k % 64, d = (k / 64) % 3, tl = k / 192;
      if (a0 + al < N) sm[tl][d][al] = src[((size_t)(8 * t8 + tl) * 3 + d) * N + a0 + al];
    }
    __syncthreads();
    for (int k = tid; k < 64 * 24; k += 256) {             // runs of 24 per atom
      const int tl = k % 8, d = (k / 8) % 3, al = k / 24;
      if (a0 + al < N) dst[qhp::qtb_rec(8 * t8 + tl, d, a0 + al, N)] = sm[tl][d][al];
    }
  } else {
    for (int k = tid; k < 64 * 24; k += 256) {
      const int tl = k % 8, d = (k / 8) % 3, al = k / 24;
      if (a0 + al < N) sm[tl][d][al] = src[qhp::qtb_rec(8 * t8 + tl, d, a0 + al, N)];
    }
    __syncthreads();
    for (int k = tid; k < 8 * 3 * 64; k += 256) {
      const int al = k % 64, d = (k / 64) % 3, tl = k / 192;
      if (a0 + al < N) dst[((size_t)(8 * t8 + tl) * 3 + d) * N + a0 + al] = sm[tl][d][al];
    }
  }
}

struct GenArgs {
  int N, nseg;
  uint64_t seed;
  int64_t seg;
  const int* type;
  const double2* hhat;
  const double2* tw4;
  double* noise;          // qtb_rec layout
};

// One block per atom (two blocks per compute unit: 64 KB of LDS at N_seg = 1,024, and at
// most 128 VGPRs so that two 512-thread blocks fit the register file as well). The
// window's white noise is drawn once (each Philox counter gives the x, y and z Gaussians;
// z waits in registers), then x + i y and z + 0 i are convolved with the type's kernel in
// turn: forward transform of length 4 N_seg, product with the kernel's transform, inverse
// transform, the middle N_seg samples written as 64-byte runs of the segment record.
template <int L4, int NTH>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(4))) void k_qtb_generate(GenArgs A) {
  constexpr int NS = L4 / 4, LG = tw_lg<L4>(), EPT = L4 / NTH;
  __shared__ double2 buf[L4];
  __shared__ double2 hi[L4 >> LG], lo[1 << LG];
  const int a = blockIdx.x, tid = threadIdx.x;
  load_twiddles<L4>(hi, lo, A.tw4);
  const uint64_t c0 = (uint64_t)(A.seg * NS);   // counter of window sample 0
  double zr[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int l = tid + i * NTH;
    double2 w = make_double2(0.0, 0.0);
    zr[i] = 0.0;
    if (l < 3 * NS) {
      double gs[3];
      qhp::gauss3(A.seed, qhp::STREAM_QTB_WHITE, c0 + (uint64_t)l, (uint64_t)a, 0ull, gs);
      w = make_double2(gs[0], gs[1]);
      zr[i] = gs[2];
    }
    buf[l] = w;
  }
  __syncthreads();
  const double2* Hz = A.hhat + (size_t)A.type[a] * L4;
  const double inv = 1.0 / L4;
  for (int slot = 0; slot < 2; ++slot) {
    if (slot == 1) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) buf[tid + i * NTH] = make_double2(zr[i], 0.0);
      __syncthreads();
    }
    fft_inplace<L4, NTH, false, LG>(buf, hi, lo);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int l = tid + i * NTH;
      buf[l] = cmul(buf[l], Hz[l]);
    }
    __syncthreads();
    fft_inplace<L4, NTH, true, LG>(buf, hi, lo);
    for (int t = tid; t < NS; t += NTH) {
      const double2 f = buf[NS + t];
      if (slot == 0) {
        A.noise[qhp::qtb_rec(t, 0, a, A.N)] = f.x * inv;
        A.noise[qhp::qtb_rec(t, 1, a, A.N)] = f.y * inv;
      } else {
        A.noise[qhp::qtb_rec(t, 2, a, A.N)] = f.x * inv;
      }
    }
    __syncthreads();                  // buf is read before it is refilled
  }
}

// N_seg that is not a power of two (any multiple of 8 with no prime factor above 7): the
// same convolution, one atom per block, between two dynamic LDS buffers of 4 N_seg with the
// runtime mixed-radix transform. The z Gaussians are drawn again for the second series.
__global__ __launch_bounds__(NT) void k_qtb_generate_rt(GenArgs A) {
  extern __shared__ double2 lds[];
  const int NS = A.nseg, L4 = 4 * NS;
  double2* a = lds;
  double2* b = lds + L4;
  const int at = blockIdx.x, tid = threadIdx.x;
  const uint64_t c0 = (uint64_t)(A.seg * NS);   // counter of window sample 0
  const double2* Hz = A.hhat + (size_t)A.type[at] * L4;
  const double inv = 1.0 / L4;
  for (int slot = 0; slot < 2; ++slot) {
    for (int l = tid; l < L4; l += NT) {
      double2 w = make_double2(0.0, 0.0);
      if (l < 3 * NS) {
        double gs[3];
        qhp::gauss3(A.seed, qhp::STREAM_QTB_WHITE, c0 + (uint64_t)l, (uint64_t)at, 0ull, gs);
        w = slot == 0 ? make_double2(gs[0], gs[1]) : make_double2(gs[2], 0.0);
      }
      a[l] = w;
    }
    __syncthreads();
    double2* X = qhp::fft_rt(a, b, L4, 1, false, A.tw4);
    double2* Y = X == a ? b : a;
    for (int l = tid; l < L4; l += NT) X[l] = cmul(X[l], Hz[l]);
    __syncthreads();
    double2* f = qhp::fft_rt(X, Y, L4, 1, true, A.tw4);
    for (int t = tid; t < NS; t += NT) {
      const double2 v = f[NS + t];
      if (slot == 0) {
        A.noise[qhp::qtb_rec(t, 0, at, A.N)] = v.x * inv;
        A.noise[qhp::qtb_rec(t, 1, at, A.N)] = v.y * inv;
      } else {
        A.noise[qhp::qtb_rec(t, 2, at, A.N)] = v.x * inv;
      }
    }
    __syncthreads();                  // the buffers are read before they are refilled
  }
}

struct SpecArgs {
  int N, nseg, ntypes;
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

// Spectra of the finished segment: per degree of freedom the transform of v + i F over
// 2 N_seg points (the segment zero-padded), C_vv and Re C_vF from its even and odd parts,
// Delta = m gamma C_vv - Re C_vF summed per type in LDS (and C_vv, Re C_vF for RATIO),
// then added to the type sums. Each block takes the three axes of consecutive atoms.
template <int L2, int NTH>
__global__ __launch_bounds__(NTH) void k_qtb_spectra(SpecArgs A) {
  constexpr int NS = L2 / 2, LG = tw_lg<L2>(), EPT = L2 / NTH;
  __shared__ double2 buf[L2];
  __shared__ double2 hi[L2 >> LG], lo[1 << LG];
  extern __shared__ double acc[];                       // [types][NS+1] Delta; C_vv; Re C_vF
  const int tid = threadIdx.x;
  const int nk = A.ntypes * (NS + 1);
  double* avv = acc + nk;
  double* avf = avv + nk;
  load_twiddles<L2>(hi, lo, A.tw2);
  for (int k = tid; k < (A.ratio ? 3 : 1) * nk; k += NTH) acc[k] = 0.0;
  // the accumulators are cleared and read back by different threads (a block whose atoms
  // all belong to another launch's types runs no barrier in the loop below)
  __syncthreads();
  const double sc = A.dt / NS;
  const int atoms_per_block = (A.N + gridDim.x - 1) / gridDim.x;
  const int a0 = blockIdx.x * atoms_per_block, a1 = min(A.N, a0 + atoms_per_block);
  for (int a = a0; a < a1; ++a) {
    const int ty = A.type[a] - A.z0;
    if (ty < 0 || ty >= A.ntypes) continue;            // another launch's type (uniform)
    const double m = A.mass[a];
    const double* gz = A.gamma + (size_t)(ty + A.z0) * (NS + 1);
    for (int d = 0; d < 3; ++d) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int t = tid + i * NTH;
        double2 z = make_double2(0.0, 0.0);
        if (t < NS) {
          const size_t r = qhp::qtb_rec(t, d, a, A.N);
          z = make_double2(A.vrec[r], A.noise[r]);
        }
        buf[t] = z;
      }
      __syncthreads();
      fft_inplace<L2, NTH, false, LG>(buf, hi, lo);
      for (int k = tid; k <= NS; k += NTH) {
        const double2 zk = buf[k], zm = buf[(L2 - k) % L2];
        // V = (Z_k + conj Z_-k) / 2, F = (Z_k - conj Z_-k) / 2i
        const double vr = 0.5 * (zk.x + zm.x), vi = 0.5 * (zk.y - zm.y);
        const double fr = 0.5 * (zk.y + zm.y), fi = -0.5 * (zk.x - zm.x);
        const double cvv = sc * (vr * vr + vi * vi);
        const double cvf = sc * (vr * fr + vi * fi);       // Re(V conj F)
        acc[ty * (NS + 1) + k] += m * gz[k] * cvv - cvf;
        if (A.ratio) {
          avv[ty * (NS + 1) + k] += cvv;
          avf[ty * (NS + 1) + k] += cvf;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  const size_t o = (size_t)A.z0 * (NS + 1);
  for (int k = tid; k < nk; k += NTH) {
    if (acc[k] != 0.0) atomicAdd(A.dsum + o + k, acc[k]);
    if (A.ratio) {
      if (avv[k] != 0.0) atomicAdd(A.vvsum + o + k, avv[k]);
      if (avf[k] != 0.0) atomicAdd(A.vfsum + o + k, avf[k]);
    }
  }
}

// Spectra for N_seg that is not a power of two: as k_qtb_spectra, with two dynamic LDS
// buffers of 2 N_seg and the runtime mixed-radix transform; the accumulators follow them.
__global__ __launch_bounds__(NT) void k_qtb_spectra_rt(SpecArgs A) {
  extern __shared__ double2 lds[];
  const int NS = A.nseg, L2 = 2 * NS, tid = threadIdx.x;
  double2* a = lds;
  double2* b = lds + L2;
  double* acc = reinterpret_cast<double*>(lds + 2 * L2);   // [types][NS+1] Delta; C_vv; Re C_vF
  const int nk = A.ntypes * (NS + 1);
  double* avv = acc + nk;
  double* avf = avv + nk;
  for (int k = tid; k < (A.ratio ? 3 : 1) * nk; k += NT) acc[k] = 0.0;
  __syncthreads();
  const double sc = A.dt / NS;
  const int atoms_per_block = (A.N + gridDim.x - 1) / gridDim.x;
  const int a0 = blockIdx.x * atoms_per_block, a1 = min(A.N, a0 + atoms_per_block);
  for (int at = a0; at < a1; ++at) {
    const int ty = A.type[at] - A.z0;
    if (ty < 0 || ty >= A.ntypes) continue;            // another launch's type (uniform)
    const double m = A.mass[at];
    const double* gz = A.gamma + (size_t)(ty + A.z0) * (NS + 1);
    for (int d = 0; d < 3; ++d) {
      for (int t = tid; t < L2; t += NT) {
        double2 z = make_double2(0.0, 0.0);
        if (t < NS) {
          const size_t r = qhp::qtb_rec(t, d, at, A.N);
          z = make_double2(A.vrec[r], A.noise[r]);
        }
        a[t] = z;
      }
      __syncthreads();
      const double2* Z = qhp::fft_rt(a, b, L2, 1, false, A.tw2);
      for (int k = tid; k <= NS; k += NT) {
        const double2 zk = Z[k], zm = Z[(L2 - k) % L2];
        const double vr = 0.5 * (zk.x + zm.x), vi = 0.5 * (zk.y - zm.y);
        const double fr = 0.5 * (zk.y + zm.y), fi = -0.5 * (zk.x - zm.x);
        const double cvv = sc * (vr * vr + vi * vi);
        const double cvf = sc * (vr * fr + vi * fi);
        acc[ty * (NS + 1) + k] += m * gz[k] * cvv - cvf;
        if (A.ratio) {
          avv[ty * (NS + 1) + k] += cvv;
          avf[ty * (NS + 1) + k] += cvf;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  const size_t o = (size_t)A.z0 * (NS + 1);
  for (int k = tid; k < nk; k += NT) {
    if (acc[k] != 0.0) atomicAdd(A.dsum + o + k, acc[k]);
    if (A.ratio) {
      if (avv[k] != 0.0) atomicAdd(A.vvsum + o + k, avv[k]);
      if (avf[k] != 0.0) atomicAdd(A.vfsum + o + k, avf[k]);
    }
  }
}

// Per type z, by its scheme: SIMPLE: gamma <- max(gamma_min, gamma - A Delta_bar). RATIO:
// the running means <C> <- <C> decay_z + C_bar (1 - decay_z) of C_vv and Re C_vF,
// decay_z = exp(-N_seg dt / tau_z), then gamma <- max(gamma_min, Re<C_vF> / (m <C_vv>))
// where <C_vv> > 0. Keep Delta_bar for export; clear the sums.
struct AdaptArgs {
  int n, nseg, any_ratio;
  double* gamma; double* dsum; double* dbar; double* vvsum; double* vfsum;
  double* avg_vv; double* avg_vf;
  const double* inv_count; const double* tmass;
  double rate, gmin;
  int ratio_of[QHP_MAX_TYPES];
  double decay[QHP_MAX_TYPES];
};

__global__ void k_qtb_adapt(AdaptArgs A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int z = i / (A.nseg + 1);
  const double ic = A.inv_count[z];
  const double d = A.dsum[i] * ic;
  A.dbar[i] = d;
  double g = A.gamma[i] - A.rate * d;
  if (A.any_ratio) {
    if (A.ratio_of[z]) {
      const double dz = A.decay[z];
      const double vv = A.avg_vv[i] * dz + A.vvsum[i] * ic * (1.0 - dz);
      const double vf = A.avg_vf[i] * dz + A.vfsum[i] * ic * (1.0 - dz);
      A.avg_vv[i] = vv;
      A.avg_vf[i] = vf;
      g = vv > 0.0 ? vf / (A.tmass[z] * vv) : A.gamma[i];
    }
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

#define QHP_SWITCH_NSEG(NS, CALL)                      \
  switch (NS) {                                         \
    case 16: { constexpr int SS = 16; CALL; } break;    \
    case 32: { constexpr int SS = 32; CALL; } break;    \
    case 64: { constexpr int SS = 64; CALL; } break;    \
    case 128: { constexpr int SS = 128; CALL; } break;  \
    case 256: { constexpr int SS = 256; CALL; } break;  \
    case 512: { constexpr int SS = 512; CALL; } break;  \
    case 1024: { constexpr int SS = 1024; CALL; } break; \
    default: return hipErrorInvalidValue;               \
  }

// threads of the segment kernels: one radix-8 butterfly per thread for the longest
// transform, at least a wavefront
template <int L>
constexpr int seg_threads() { return L / 8 < 64 ? 64 : (L / 8 > 512 ? 512 : L / 8); }

hipError_t launch_qtb_generate(qhp_ctx* c, int64_t seg) {
  QtbState& q = c->qtb;
  hipError_t e = qtb_build_kernels(c);
  if (e != hipSuccess) return e;
  GenArgs A;
  A.N = c->N; A.nseg = q.nseg; A.seed = c->p.seed; A.seg = seg; A.type = c->d_type;
  A.hhat = q.hhat; A.tw4 = q.tw4; A.noise = q.noise_t;
  if (q.nseg & (q.nseg - 1)) {
    hipLaunchKernelGGL(k_qtb_generate_rt, c->N, NT, (size_t)8 * q.nseg * sizeof(double2),
                       c->stream, A);
  } else {
    QHP_SWITCH_NSEG(q.nseg, hipLaunchKernelGGL((k_qtb_generate<4 * SS, seg_threads<4 * SS>()>),
                                               c->N, seg_threads<4 * SS>(), 0, c->stream, A));
  }
  // the per-step copy (the segment kernels keep theirs for the spectra)
  const dim3 tg((c->N + 63) / 64, q.nseg / 8);
  hipLaunchKernelGGL(k_qtb_transpose<false>, tg, 256, 0, c->stream, q.noise_t, q.noise, c->N);
  return hipGetLastError();
}

hipError_t launch_qtb_adapt(qhp_ctx* c) {
  QtbState& q = c->qtb;
  SpecArgs A;
  A.N = c->N; A.nseg = q.nseg;
  A.type = c->d_type; A.mass = c->d_mass; A.gamma = q.gamma; A.vrec = q.vrec_t; A.noise = q.noise_t;
  {
    const dim3 tg((c->N + 63) / 64, q.nseg / 8);
    hipLaunchKernelGGL(k_qtb_transpose<true>, tg, 256, 0, c->stream, q.vrec, q.vrec_t, c->N);
  }
  A.tw2 = q.tw2; A.dt = c->p.dt; A.dsum = q.dsum;
  A.vvsum = q.vvsum; A.vfsum = q.vfsum;
  A.ratio = q.any_ratio;
  // a few atoms per block, several blocks per compute unit; the per-type accumulators are
  // dynamic LDS next to the transform: types that do not fit together are accumulated by
  // further launches (each skips the others' atoms)
  const int nb = std::max(1, std::min(c->N, 4096));
  const bool rt = (q.nseg & (q.nseg - 1)) != 0;        // not a power of two
  const size_t fft_lds = rt ? (size_t)4 * q.nseg * sizeof(double2)
                            : (size_t)(2 * q.nseg + 64) * sizeof(double2);
  const size_t per_type = (size_t)(A.ratio ? 3 : 1) * (q.nseg + 1) * sizeof(double);
  const int fit = (int)std::max<size_t>(1, (QTB_LDS_MAX / 2 - fft_lds) / per_type);
  for (int z0 = 0; z0 < c->p.n_types; z0 += fit) {
    A.z0 = z0;
    A.ntypes = std::min(fit, c->p.n_types - z0);
    if (rt) {
      hipLaunchKernelGGL(k_qtb_spectra_rt, nb, NT, fft_lds + A.ntypes * per_type, c->stream, A);
    } else {
      QHP_SWITCH_NSEG(q.nseg, hipLaunchKernelGGL((k_qtb_spectra<2 * SS, seg_threads<2 * SS>()>), nb,
                                                 seg_threads<2 * SS>(), A.ntypes * per_type,
                                                 c->stream, A));
    }
  }
  AdaptArgs D;
  D.n = c->p.n_types * (q.nseg + 1); D.nseg = q.nseg; D.any_ratio = A.ratio;
  D.gamma = q.gamma; D.dsum = q.dsum; D.dbar = q.dbar; D.vvsum = q.vvsum; D.vfsum = q.vfsum;
  D.avg_vv = q.avg_vv; D.avg_vf = q.avg_vf; D.inv_count = q.d_inv_count; D.tmass = q.d_tmass;
  D.rate = c->p.qtb_adapt_rate; D.gmin = c->p.qtb_gamma_min_frac * c->p.qtb_gamma0;
  for (int z = 0; z < QHP_MAX_TYPES; ++z) {
    D.ratio_of[z] = z < c->p.n_types ? q.ratio_of[z] : 0;
    D.decay[z] = D.ratio_of[z] ? std::exp(-q.nseg * c->p.dt / q.tau_of[z]) : 0.0;
  }
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
