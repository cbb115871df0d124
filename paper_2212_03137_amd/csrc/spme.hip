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
// FFT: five passes over the grid; a block of each pass transforms 2048 complex values
// (2048/K series of length K along one axis) by Stockham stages of radix 8 (then 4, 2).
// The first stage reads its operands from the grid and the last writes the grid, so
// for K = 64 (two radix-8 stages) the data cross LDS once; the z pass does the forward
// transform, the multiplication by G (folded into the forward's last stage) and the
// inverse transform in one visit.
#include <algorithm>

#include "qhp_internal.h"

namespace {

constexpr int NT = 256;

struct SpmeArgs {
  int N;
  int nblocks;             // logical blocks of the gather
  const int* order;        // atoms in tile order (spatially compact blocks)
  int K0, K1, K2;
  int Pc2;                 // doubles per grid point (2 * complex slots)
  const double* x; double* g;
  double* grid;
  const double* charge;
  double L[3];
  double* energy;
  double* dq;              // parameter gradients: d E_recip / d q = interpolated potential
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

// Values, first and second derivatives of the order-n B-spline weights (the second
// derivative is M_{n-2}(u) - 2 M_{n-2}(u-1) + M_{n-2}(u-2)).
template <int ORDER>
QHP_DEV void bspline2(double frac, double* w, double* dw, double* ddw) {
  double m[ORDER];
#pragma unroll
  for (int t = 0; t < ORDER; ++t) m[t] = 0.0;
  m[0] = frac;
  m[1] = 1.0 - frac;
  auto second = [&]() {
#pragma unroll
    for (int t = 0; t < ORDER; ++t)
      ddw[t] = m[t] - (t >= 1 ? 2.0 * m[t - 1] : 0.0) + (t >= 2 ? m[t - 2] : 0.0);
  };
  if (ORDER == 3) second();
#pragma unroll
  for (int k = 3; k <= ORDER; ++k) {
    if (k == ORDER - 1) second();
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

// physical block -> logical block so that XCD k (blocks k, k+8, ...) gets a contiguous range
QHP_DEV int xcd_block(int bid, int nphys) { return (bid & 7) * (nphys >> 3) + (bid >> 3); }

// PG: also add the interpolated potential sum_k theta(k) phi(k) of every bead, summed over
// the beads, to dq of the atom (the charge derivative of the reciprocal energy).
template <int P, int ORDER, bool ENERGY, bool PG = false>
__global__ __launch_bounds__(NT) void k_gather(SpmeArgs A) {
  __shared__ double sred[NT];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int tid = lb * NT + threadIdx.x;
  const int k = tid / P, b = tid % P;
  const int a = (lb < A.nblocks && k < A.N) ? A.order[k] : A.N;
  double e = 0;
  if (a < A.N) {
    double xb[3];
    for (int d = 0; d < 3; ++d) xb[d] = A.x[(d * A.N + a) * P + b];
    const int K[3] = {A.K0, A.K1, A.K2};
    int i0[3];
    double w[3][ORDER], dw[3][ORDER];
    stencil<ORDER>(xb, A.L, K, i0, w, dw);
    double f0 = 0, f1 = 0, f2 = 0;
    int o2[ORDER];                    // offsets of the z stencil points within a grid row
#pragma unroll
    for (int t2 = 0; t2 < ORDER; ++t2) o2[t2] = wrapk(i0[2] - t2, A.K2) * A.Pc2;
    const double* gb = A.grid + b;
#pragma unroll 1
    for (int t0 = 0; t0 < ORDER; ++t0) {
      const int k0 = wrapk(i0[0] - t0, A.K0);
      // issue the ORDER x ORDER loads of this x plane together, then reduce
      double ph[ORDER][ORDER];
#pragma unroll
      for (int t1 = 0; t1 < ORDER; ++t1) {
        const double* row = gb + (size_t)((k0 * A.K1 + wrapk(i0[1] - t1, A.K1)) * A.K2) * A.Pc2;
#pragma unroll
        for (int t2 = 0; t2 < ORDER; ++t2) ph[t1][t2] = row[o2[t2]];
      }
      __builtin_amdgcn_sched_barrier(0);   // keep the loads in flight together
#pragma unroll
      for (int t1 = 0; t1 < ORDER; ++t1) {
        double s = 0, sd = 0;
#pragma unroll
        for (int t2 = 0; t2 < ORDER; ++t2) {
          s += w[2][t2] * ph[t1][t2];
          sd += dw[2][t2] * ph[t1][t2];
        }
        f0 += dw[0][t0] * w[1][t1] * s;
        f1 += w[0][t0] * dw[1][t1] * s;
        f2 += w[0][t0] * w[1][t1] * sd;
        if (ENERGY || PG) e += w[0][t0] * w[1][t1] * s;
      }
    }
    const double q = A.charge[a];
    A.g[(0 * A.N + a) * P + b] += q * f0 * (double)A.K0 / A.L[0];
    A.g[(1 * A.N + a) * P + b] += q * f1 * (double)A.K1 / A.L[1];
    A.g[(2 * A.N + a) * P + b] += q * f2 * (double)A.K2 / A.L[2];
    if (PG) {
      double phi = e;                  // the P lanes of an atom are consecutive
      for (int o = 1; o < P; o <<= 1) phi += __shfl_xor(phi, o);
      if (b == 0) A.dq[a] += phi;
    }
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

// One bead (P = 1): a group of 8 lanes per atom, lane t0 < ORDER taking the x plane t0 of
// the stencil (ORDER^2 loads instead of ORDER^3 per lane), the group summed by shuffles:
// eight times the wavefronts of one lane per atom, enough to hide the latency of the
// scattered grid loads.
template <int ORDER, bool ENERGY, bool PG = false>
__global__ __launch_bounds__(NT) void k_gather_one(SpmeArgs A) {
  static_assert(ORDER <= 8, "one x plane per lane of a group of eight");
  __shared__ double sred[NT / 64];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int tid = lb * NT + threadIdx.x;
  const int k = tid >> 3, t0 = tid & 7;
  const int a = (lb < A.nblocks && k < A.N) ? A.order[k] : A.N;
  double f0 = 0, f1 = 0, f2 = 0, e = 0;
  if (a < A.N && t0 < ORDER) {
    double xb[3];
    for (int d = 0; d < 3; ++d) xb[d] = A.x[d * A.N + a];
    const int K[3] = {A.K0, A.K1, A.K2};
    int i0[3];
    double w[3][ORDER], dw[3][ORDER];
    stencil<ORDER>(xb, A.L, K, i0, w, dw);
    int o2[ORDER];
#pragma unroll
    for (int t2 = 0; t2 < ORDER; ++t2) o2[t2] = wrapk(i0[2] - t2, A.K2) * A.Pc2;
    const int k0 = wrapk(i0[0] - t0, A.K0);
    double ph[ORDER][ORDER];
#pragma unroll
    for (int t1 = 0; t1 < ORDER; ++t1) {
      const double* row = A.grid + (size_t)((k0 * A.K1 + wrapk(i0[1] - t1, A.K1)) * A.K2) * A.Pc2;
#pragma unroll
      for (int t2 = 0; t2 < ORDER; ++t2) ph[t1][t2] = row[o2[t2]];
    }
    // this lane's plane: the weights of x point t0 (selected without indexing by t0)
    double wx = 0, dwx = 0;
#pragma unroll
    for (int t = 0; t < ORDER; ++t)
      if (t == t0) { wx = w[0][t]; dwx = dw[0][t]; }
#pragma unroll
    for (int t1 = 0; t1 < ORDER; ++t1) {
      double sm = 0, sd = 0;
#pragma unroll
      for (int t2 = 0; t2 < ORDER; ++t2) {
        sm += w[2][t2] * ph[t1][t2];
        sd += dw[2][t2] * ph[t1][t2];
      }
      f0 += dwx * w[1][t1] * sm;
      f1 += wx * dw[1][t1] * sm;
      f2 += wx * w[1][t1] * sd;
      if (ENERGY || PG) e += wx * w[1][t1] * sm;
    }
  }
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    f0 += __shfl_xor(f0, o); f1 += __shfl_xor(f1, o); f2 += __shfl_xor(f2, o);
    if (ENERGY || PG) e += __shfl_xor(e, o);
  }
  double eq = 0.0;
  if (a < A.N && t0 == 0) {
    const double q = A.charge[a];
    A.g[0 * A.N + a] += q * f0 * (double)A.K0 / A.L[0];
    A.g[1 * A.N + a] += q * f1 * (double)A.K1 / A.L[1];
    A.g[2 * A.N + a] += q * f2 * (double)A.K2 / A.L[2];
    if (PG) A.dq[a] += e;
    eq = 0.5 * q * e;
  }
  if (ENERGY) {
#pragma unroll
    for (int o = 8; o < 64; o <<= 1) eq += __shfl_xor(eq, o);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = eq;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int w = 0; w < NT / 64; ++w) sum += sred[w];
      atomicAdd(A.energy + QHP_E_COUL_RECIP, sum);
    }
  }
}

// Hessian-vector product of the reciprocal energy: with phi the potential grid of x and
// dphi the potential of the tangent density sum_b q_b grad W_b . u_b,
//   (H u)_a = q_a [ sum_k (grad grad W_a(k)) u_a phi(k) + sum_k grad W_a(k) dphi(k) ].
// With A.dq set, also add d(u . grad E_recip)/dq_a = sum_k grad W_a(k) . u_a phi(k) +
// sum_k W_a(k) dphi(k), summed over the beads.
template <int P, int ORDER>
__global__ __launch_bounds__(NT) void k_gather_hvp(SpmeArgs A, const double* dgrid,
                                                   const double* u, double* hu) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int tid = lb * NT + threadIdx.x;
  const int k = tid / P, b = tid % P;
  const int a = (lb < A.nblocks && k < A.N) ? A.order[k] : A.N;
  if (a >= A.N) return;
  const int K[3] = {A.K0, A.K1, A.K2};
  int i0[3];
  double w[3][ORDER], dw[3][ORDER], ddw[3][ORDER], KoL[3];
  for (int d = 0; d < 3; ++d) {
    KoL[d] = (double)K[d] / A.L[d];
    double sfr = A.x[(d * A.N + a) * P + b] / A.L[d];
    sfr = sfr - floor(sfr);
    const double uu = sfr * (double)K[d];
    const double fl = floor(uu);
    i0[d] = isfinite(fl) ? min(max((int)fl, 0), K[d]) : 0;
    bspline2<ORDER>(uu - fl, w[d], dw[d], ddw[d]);
  }
  double h00 = 0, h11 = 0, h22 = 0, h01 = 0, h02 = 0, h12 = 0, g0 = 0, g1 = 0, g2 = 0;
  double f0 = 0, f1 = 0, f2 = 0, wd = 0;
  for (int t0 = 0; t0 < ORDER; ++t0) {
    const int k0 = wrapk(i0[0] - t0, A.K0);
#pragma unroll
    for (int t1 = 0; t1 < ORDER; ++t1) {
      const int k1 = wrapk(i0[1] - t1, A.K1);
      const size_t ro = ((size_t)(k0 * A.K1 + k1) * A.K2) * A.Pc2 + b;
      double sv = 0, sd = 0, sdd = 0, tv = 0, td = 0;
#pragma unroll
      for (int t2 = 0; t2 < ORDER; ++t2) {
        const size_t o = ro + (size_t)wrapk(i0[2] - t2, A.K2) * A.Pc2;
        const double ph = A.grid[o], dph = dgrid[o];
        sv += w[2][t2] * ph;
        sd += dw[2][t2] * ph;
        sdd += ddw[2][t2] * ph;
        tv += w[2][t2] * dph;
        td += dw[2][t2] * dph;
      }
      h00 += ddw[0][t0] * w[1][t1] * sv;
      h11 += w[0][t0] * ddw[1][t1] * sv;
      h22 += w[0][t0] * w[1][t1] * sdd;
      h01 += dw[0][t0] * dw[1][t1] * sv;
      h02 += dw[0][t0] * w[1][t1] * sd;
      h12 += w[0][t0] * dw[1][t1] * sd;
      g0 += dw[0][t0] * w[1][t1] * tv;
      g1 += w[0][t0] * dw[1][t1] * tv;
      g2 += w[0][t0] * w[1][t1] * td;
      f0 += dw[0][t0] * w[1][t1] * sv;
      f1 += w[0][t0] * dw[1][t1] * sv;
      f2 += w[0][t0] * w[1][t1] * sd;
      wd += w[0][t0] * w[1][t1] * tv;
    }
  }
  const double q = A.charge[a];
  const double u0 = u[(0 * A.N + a) * P + b] * KoL[0], u1 = u[(1 * A.N + a) * P + b] * KoL[1],
               u2 = u[(2 * A.N + a) * P + b] * KoL[2];
  hu[(0 * A.N + a) * P + b] += q * KoL[0] * (h00 * u0 + h01 * u1 + h02 * u2 + g0);
  hu[(1 * A.N + a) * P + b] += q * KoL[1] * (h01 * u0 + h11 * u1 + h12 * u2 + g1);
  hu[(2 * A.N + a) * P + b] += q * KoL[2] * (h02 * u0 + h12 * u1 + h22 * u2 + g2);
  if (A.dq) {                          // the P lanes of an atom are consecutive
    double m = u0 * f0 + u1 * f1 + u2 * f2 + wd;
    for (int o = 1; o < P; o <<= 1) m += __shfl_xor(m, o);
    if (b == 0) A.dq[a] += m;
  }
}

// ------------------------------- owner-computes spreading ------------------------------
// The grid is cut into TB^3-point tiles. Atoms are binned every step by the tile of their
// centroid's stencil base; one block per (tile, group of GB beads) accumulates in LDS the
// contributions of the atoms binned in the tile and its 26 neighbours and writes the tile
// once. This is exact as long as no bead's base index differs from its centroid's by more
// than TB points above or TB - n + 1 below, which the binning kernel checks (error flag).
constexpr int TB = QHP_TB;

struct TileArgs {
  int N, P, K0, K1, K2, nt0, nt1, nt2, order;
  const double* x;            // [3][N][P]
  const double4* cent;        // centroids (batched) or null (P = 1: the bead itself)
  double L[3], KoL[3];
  int* tile_of; int* tile_count; int* tile_fill; int* tile_start; int* tile_atoms;
  int ntiles;
};

using qhp::base_of;
using qhp::grid_coord;

// bin every atom by the tile of its centroid's grid base (P = 1: of the bead itself)
__global__ __launch_bounds__(256) void k_tile_bin(TileArgs A) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A.N) return;
  const int K[3] = {A.K0, A.K1, A.K2};
  int bc[3];
  for (int d = 0; d < 3; ++d) {
    const double cd = A.cent ? (&A.cent[a].x)[d] : A.x[(size_t)d * A.N + a];
    const int b = base_of(cd, A.KoL[d], K[d]);
    bc[d] = b >= K[d] ? b - K[d] : b;
  }
  const int t = (bc[0] / TB * A.nt1 + bc[1] / TB) * A.nt2 + bc[2] / TB;
  A.tile_of[a] = t;
  atomicAdd(&A.tile_count[t], 1);
}

__global__ __launch_bounds__(256) void k_tile_scan(TileArgs A) {
  __shared__ int part[256];
  const int t = threadIdx.x;
  const int per = (A.ntiles + 255) / 256;
  const int b0 = min(A.ntiles, t * per), b1 = min(A.ntiles, b0 + per);
  int s = 0;
  for (int k = b0; k < b1; ++k) s += A.tile_count[k];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int k = 0; k < 256; ++k) { const int v = part[k]; part[k] = acc; acc += v; }
    A.tile_start[A.ntiles] = acc;
  }
  __syncthreads();
  int acc = part[t];
  for (int k = b0; k < b1; ++k) {
    A.tile_start[k] = acc;
    acc += A.tile_count[k];
    A.tile_fill[k] = 0;
    A.tile_count[k] = 0;        // consumed; ready for the next binning
  }
}

__global__ void k_tile_scatter(TileArgs A) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A.N) return;
  const int t = A.tile_of[a];
  const int slot = atomicAdd(&A.tile_fill[t], 1);
  A.tile_atoms[A.tile_start[t] + slot] = a;
}

struct TSpreadArgs {
  int N, P, K0, K1, K2, nt1, nt2, Pc2;
  const double* x; double* grid; const double* charge;
  const double4* cent;        // centroids (null for P = 1: the bead itself)
  double L[3], KoL[3];        // box and K / L per axis
  const NlCtrl* ctrl;         // spread_m: largest bead-centroid base offset this step
  const int* tile_start; const int* tile_atoms;   // tiles' atom ranges, atoms by tile
  const double* u;            // tangent spreading: direction [3][N][P]
};

// in-tile range of the stencil points base - t, t = 0..ORDER-1, along one axis:
// lo = (base - ORDER + 1 - t0) mod K is the tile-relative position of the lowest point
// v mod K in [0, K) (a mask when K is a power of two)
QHP_DEV int wrap_mod(int v, int K) { return (K & (K - 1)) ? ((v % K) + K) % K : (v & (K - 1)); }

template <int ORDER>
QHP_DEV int tile_lo(int base, int t0, int K) {
  return wrap_mod(base - (ORDER - 1) - t0, K);
}

// TAN: spread the derivative of the charge density along the direction u instead,
// sum_a q_a grad W_a(k) . u_a (the tangent grid of a Hessian-vector product).
// Z: the block's tile spans Z consecutive tiles along z (TB x TB x Z TB points; atoms
// binned per TB^3 tile, so the neighbourhood is 3 x 3 columns of Z + 2 tiles). A taller
// tile splits fewer stencil rows between blocks.
template <int ORDER, int GB, bool TAN = false, int Z = 1>
__global__ __launch_bounds__(NT) void k_spread_tiles(TSpreadArgs A) {
  constexpr int CAP = 1024;                // compacted atoms per round
  constexpr int TZ = TB * Z;
  constexpr int NR = 18;                   // neighbour ranges: 9 columns x 2 z pieces
  __shared__ double acc[TB * TB * TZ * GB];
  __shared__ int cand[CAP];
  __shared__ int ncand;
  __shared__ int tofs[NR + 1], tbeg[NR];
  const int tile = blockIdx.x, grp = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
  for (int k = tid; k < TB * TB * TZ * GB; k += NT) acc[k] = 0.0;
  const int nz = A.nt2 / Z;
  const int T2 = (tile % nz) * Z, T1 = (tile / nz) % A.nt1, T0 = tile / (nz * A.nt1);
  const int K[3] = {A.K0, A.K1, A.K2};
  const int t0[3] = {T0 * TB, T1 * TB, T2 * TB};
  const int ext[3] = {TB, TB, TZ};
  const int P = A.P;
  const int m = A.cent ? A.ctrl->spread_m : 0;
  // the atoms of the distinct neighbouring columns' tiles T2 - 1 .. T2 + Z (wrapped:
  // at most two contiguous pieces per column), concatenated
  if (tid < NR) {
    const int col = tid >> 1, part = tid & 1, dx = col / 3 - 1, dy = col % 3 - 1;
    const int nt0 = A.K0 / TB, nt1 = A.nt1, nt2 = A.nt2;
    const bool okx = nt0 >= 3 || (nt0 == 2 && dx != 1) || (nt0 == 1 && dx == 0);
    const bool oky = nt1 >= 3 || (nt1 == 2 && dy != 1) || (nt1 == 1 && dy == 0);
    int zlo = 0, zhi = 0;
    if (Z + 2 >= nt2) {
      if (part == 0) zhi = nt2;
    } else {
      const int z0 = (T2 - 1 + nt2) % nt2, n = Z + 2;
      if (z0 + n <= nt2) {
        if (part == 0) { zlo = z0; zhi = z0 + n; }
      } else if (part == 0) {
        zlo = z0; zhi = nt2;
      } else {
        zhi = z0 + n - nt2;
      }
    }
    int beg = 0, len = 0;
    if (okx && oky && zhi > zlo) {
      const int cx = (T0 + dx + nt0) % nt0, cy = (T1 + dy + nt1) % nt1;
      const int base = (cx * nt1 + cy) * nt2;
      beg = A.tile_start[base + zlo];
      len = A.tile_start[base + zhi] - beg;
    }
    tbeg[tid] = beg;
    tofs[tid + 1] = len;
  }
  __syncthreads();
  if (tid == 0) {
    tofs[0] = 0;
    for (int k = 1; k <= NR; ++k) tofs[k] += tofs[k - 1];
  }
  __syncthreads();
  const int total = tofs[NR];
  int pos = 0;
  for (;;) {
    // 1) collect atoms whose centroid stencil, widened by m points, reaches the tile
    if (tid == 0) ncand = 0;
    __syncthreads();
    while (pos < total && ncand <= CAP - NT) {
      const int p = pos + tid;
      bool hit = false;
      int a = -1;
      if (p < total) {
        int lo = 0, hi = NR;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (tofs[mid] <= p) lo = mid; else hi = mid;
        }
        a = A.tile_atoms[tbeg[lo] + (p - tofs[lo])];
        hit = true;
        if (A.cent) {
          const double4 c = A.cent[a];
          const double cc[3] = {c.x, c.y, c.z};
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int bc = base_of(cc[d], A.KoL[d], K[d]);
            const int l0 = tile_lo<ORDER>(bc - m, t0[d], K[d]);
            if (!(l0 < ext[d] || l0 > K[d] - (ORDER + 2 * m) || K[d] <= ext[d])) hit = false;
          }
        }
      }
      const unsigned long long bal = __ballot(hit);
      int off = 0;
      if (lane == 0 && bal) off = atomicAdd(&ncand, __popcll(bal));
      off = __shfl(off, 0);
      if (hit) cand[off + __popcll(bal & ((1ull << lane) - 1ull))] = a;
      pos += NT;
      __syncthreads();
    }
    const bool more = pos < total;
    const int nc = ncand;
    // 2) every compacted atom at every bead of the group: spline weights, in-tile points
    for (int it = tid; it < nc * GB; it += NT) {
      const int a = cand[it / GB], b = grp * GB + it % GB, bl = it % GB;
      double fr[3];
      int lo[3];
      bool hit = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double u = grid_coord(A.x[((size_t)d * A.N + a) * P + b], A.KoL[d], K[d]);
        const double fl = floor(u);
        const int base = isfinite(fl) ? min(max((int)fl, 0), K[d]) : 0;
        fr[d] = u - fl;
        lo[d] = tile_lo<ORDER>(base, t0[d], K[d]);
        if (!(lo[d] < ext[d] || lo[d] > K[d] - ORDER || K[d] <= ext[d])) hit = false;
      }
      if (!hit) continue;
      double w[3][ORDER], dw[3][ORDER];
      int rel[2][ORDER], oz[ORDER];
      double wz[ORDER], mz[ORDER];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        bspline<ORDER>(fr[d], w[d], dw[d]);
#pragma unroll
        for (int t = 0; t < ORDER; ++t) {
          // stencil point base - t sits at tile-relative position lo + ORDER - 1 - t (mod K)
          const int r0 = lo[d] + ORDER - 1 - t;            // in [0, K + ORDER - 2]
          const int r = r0 >= K[d] ? r0 - K[d] : r0;
          if (d < 2) {
            rel[d][t] = r < TB ? r : -1;
          } else {
            // along z a point outside the tile is skipped (lanes whose point lies outside
            // issue no LDS atomic); the tangent spreading adds zero to the row's first point
            oz[t] = r < TZ ? r * GB : 0;
            wz[t] = r < TZ ? w[2][t] : 0.0;
            mz[t] = r < TZ ? 1.0 : 0.0;
          }
        }
      }
      const double qa = A.charge[a];
      if (TAN) {
        // grad W . u = u0 K0/L0 W0' W1 W2 + u1 K1/L1 W0 W1' W2 + u2 K2/L2 W0 W1 W2'
        double t[3][ORDER];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double ud = A.u[((size_t)d * A.N + a) * P + b] * A.KoL[d];
#pragma unroll
          for (int q = 0; q < ORDER; ++q) t[d][q] = ud * dw[d][q];
        }
        double tz[ORDER];
#pragma unroll
        for (int q = 0; q < ORDER; ++q) tz[q] = mz[q] * t[2][q];
#pragma unroll
        for (int ta = 0; ta < ORDER; ++ta) {
          if (rel[0][ta] < 0) continue;
#pragma unroll
          for (int tb = 0; tb < ORDER; ++tb) {
            if (rel[1][tb] < 0) continue;
            const double c1 = qa * (t[0][ta] * w[1][tb] + w[0][ta] * t[1][tb]);
            const double c2 = qa * w[0][ta] * w[1][tb];
            double* row = acc + (rel[0][ta] * TB + rel[1][tb]) * TZ * GB + bl;
#pragma unroll
            for (int tc = 0; tc < ORDER; ++tc) atomicAdd(row + oz[tc], c1 * wz[tc] + c2 * tz[tc]);
          }
        }
        continue;
      }
#pragma unroll
      for (int ta = 0; ta < ORDER; ++ta) {
        if (rel[0][ta] < 0) continue;
        const double wa = qa * w[0][ta];
#pragma unroll
        for (int tb = 0; tb < ORDER; ++tb) {
          if (rel[1][tb] < 0) continue;
          const double wab = wa * w[1][tb];
          double* row = acc + (rel[0][ta] * TB + rel[1][tb]) * TZ * GB + bl;
#pragma unroll
          for (int tc = 0; tc < ORDER; ++tc)
            if (mz[tc] != 0.0) atomicAdd(row + oz[tc], wab * wz[tc]);   // in-tile points only
        }
      }
    }
    __syncthreads();
    if (!more) break;
  }
  for (int k = tid; k < TB * TB * TZ * GB; k += NT) {
    const int bb = k % GB, pt = k / GB;
    const int r2 = pt % TZ, r1 = (pt / TZ) % TB, r0 = pt / (TZ * TB);
    const size_t g = ((size_t)((t0[0] + r0) * A.K1 + (t0[1] + r1)) * A.K2 + (t0[2] + r2)) * A.Pc2;
    A.grid[g + grp * GB + bb] = acc[k];
    if (P == 1) A.grid[g + 1] = 0.0;
  }
}

// ------------------------------- LDS Stockham FFT -------------------------------------
QHP_DEV double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
QHP_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
QHP_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// radix-4 DFT in registers (forward: exp(-2 pi i / 4) = -i)
template <bool INV>
QHP_DEV void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
  const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const double2 t2 = cadd(a1, a3), t3 = csub(a1, a3);
  const double2 jt3 = INV ? make_double2(-t3.y, t3.x) : make_double2(t3.y, -t3.x);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, jt3);
  a3 = csub(t1, jt3);
}

struct FftArgs {
  double2* grid;
  const double2* tw;       // [K] exp(-2 pi i m / K)
  const double* G;         // influence [K0][K1][K2] (fused z pass)
  int lgI;                 // log2 of the complex elements below the axis (its stride)
  int lgpc;                // log2 of the complex slots per grid point
  int efast;               // the axis is (nearly) contiguous: stage through LDS instead
};

// Where one FFT pass reads and writes: series m, element e of the pass's axis sits at
// (m / I) * K * I + (m % I) + e * I in the grid, I a power of two.
template <int K>
struct GridIO {
  double2* grid;
  long m0;                 // first series of the block
  int lgI;
  QHP_DEV long at(int s, int e) const {
    constexpr int LGK = __builtin_ctz(K);
    const long m = m0 + s;
    return ((m >> lgI) << (lgI + LGK)) + (m & ((1l << lgI) - 1)) + ((long)e << lgI);
  }
};

// Stockham stages of radix 8 while at least 8 points remain per sub-transform, then 4,
// then 2, on NS series of length K held at buf[e * NS + s] (NS * K = FFT_E). With LOADG the
// first stage takes its operands from the grid (no LDS copy-in; its twiddles are all 1),
// with STOREG the last stage writes the grid; SCALE multiplies the last stage's outputs by
// the influence function (forward half of the fused z pass).
template <int K, int NS, bool INV, int NSTRIDE, bool LOADG, bool STOREG, bool SCALE,
          int NTH = NT>
QHP_DEV void fft_stages(double2* buf, const double2* tw, int tid, const GridIO<K>& io,
                        const double* G, int lgpc) {
  if constexpr (NSTRIDE < K) {
    constexpr int R = (K / NSTRIDE >= 8) ? 8 : ((K / NSTRIDE >= 4) ? 4 : 2);
    constexpr int BPT = NS * K / R / NTH;
    static_assert(BPT * R * NTH == NS * K, "stage tasks must split evenly over the threads");
    constexpr bool FIRST = NSTRIDE == 1, LAST = NSTRIDE * R == K;
    double2 v[BPT][R];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int be = tid + i * NTH, s = be % NS, j = be / NS;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = j + r * (K / R);
        v[i][r] = (FIRST && LOADG) ? io.grid[io.at(s, e)] : buf[e * NS + s];
      }
    }
    if (!(FIRST && LOADG)) __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int be = tid + i * NTH, s = be % NS, j = be / NS;
      const int k = j % NSTRIDE;
      if constexpr (!FIRST) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double2 t = tw[r * k * (K / (NSTRIDE * R))];
          if (INV) t.y = -t.y;
          v[i][r] = cmul(v[i][r], t);
        }
      }
      if constexpr (R == 8) {
        // two radix-4 transforms of the even and odd inputs, joined by W8^q
        dft4<INV>(v[i][0], v[i][2], v[i][4], v[i][6]);
        dft4<INV>(v[i][1], v[i][3], v[i][5], v[i][7]);
        const double h = 0.70710678118654752440;
        const double sg = INV ? 1.0 : -1.0;       // W8 = (1 + sg i) / sqrt(2)
        const double2 o0 = v[i][1];
        const double2 o1 = cmul(v[i][3], make_double2(h, sg * h));
        const double2 o2 = cmul(v[i][5], make_double2(0.0, sg));
        const double2 o3 = cmul(v[i][7], make_double2(-h, sg * h));
        const double2 e0 = v[i][0], e1 = v[i][2], e2 = v[i][4], e3 = v[i][6];
        v[i][0] = cadd(e0, o0); v[i][4] = csub(e0, o0);
        v[i][1] = cadd(e1, o1); v[i][5] = csub(e1, o1);
        v[i][2] = cadd(e2, o2); v[i][6] = csub(e2, o2);
        v[i][3] = cadd(e3, o3); v[i][7] = csub(e3, o3);
      } else if constexpr (R == 4) {
        dft4<INV>(v[i][0], v[i][1], v[i][2], v[i][3]);
      } else {
        const double2 a = v[i][0], b2 = v[i][1];
        v[i][0] = cadd(a, b2);
        v[i][1] = csub(a, b2);
      }
      const int idx = (j / NSTRIDE) * NSTRIDE * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = idx + r * NSTRIDE;
        if constexpr (LAST && SCALE) {
          const double gv = G[((io.m0 + s) >> lgpc) * K + e];
          v[i][r].x *= gv; v[i][r].y *= gv;
        }
        if constexpr (LAST && STOREG) io.grid[io.at(s, e)] = v[i][r];
        else buf[e * NS + s] = v[i][r];
      }
    }
    if constexpr (!(LAST && STOREG)) __syncthreads();
    fft_stages<K, NS, INV, NSTRIDE * R, LOADG, STOREG, SCALE, NTH>(buf, tw, tid, io, G, lgpc);
  }
}

// MODE 0: forward, 1: inverse, 2: forward, x G, inverse (axis 2 only). With the series
// as the fast index (every axis but a nearly contiguous innermost one) the first and last
// stages read and write the grid directly; otherwise the block stages through LDS.
constexpr int FFT_E = QHP_FFT_E;           // complex values per block (LDS 32 KB)

template <int K, int MODE>
__global__ __launch_bounds__(NT) void k_fft_pass(FftArgs A) {
  constexpr int NS = FFT_E / K;
  constexpr int LGK = __builtin_ctz(K);
  __shared__ double2 buf[FFT_E];
  __shared__ double2 stw[K];
  const int tid = threadIdx.x;
  for (int m = tid; m < K; m += NT) stw[m] = A.tw[m];
  GridIO<K> io{A.grid, (long)blockIdx.x * NS, A.lgI};
  if (!A.efast) {
    __syncthreads();                                 // twiddles
    if (MODE == 0) fft_stages<K, NS, false, 1, true, true, false>(buf, stw, tid, io, A.G, A.lgpc);
    if (MODE == 1) fft_stages<K, NS, true, 1, true, true, false>(buf, stw, tid, io, A.G, A.lgpc);
    if (MODE == 2) {
      fft_stages<K, NS, false, 1, true, false, true>(buf, stw, tid, io, A.G, A.lgpc);
      fft_stages<K, NS, true, 1, false, true, false>(buf, stw, tid, io, A.G, A.lgpc);
    }
    return;
  }
  for (int l = tid; l < FFT_E; l += NT) {
    const int e = l & (K - 1), s = l >> LGK;
    buf[e * NS + s] = A.grid[io.at(s, e)];
  }
  __syncthreads();
  if (MODE == 1) {
    fft_stages<K, NS, true, 1, false, false, false>(buf, stw, tid, io, A.G, A.lgpc);
  } else {
    fft_stages<K, NS, false, 1, false, false, MODE == 2>(buf, stw, tid, io, A.G, A.lgpc);
  }
  if (MODE == 2) fft_stages<K, NS, true, 1, false, false, false>(buf, stw, tid, io, A.G, A.lgpc);
  for (int l = tid; l < FFT_E; l += NT) {
    const int e = l & (K - 1), s = l >> LGK;
    A.grid[io.at(s, e)] = buf[e * NS + s];
  }
}

// --------------------- spreading fused with the forward x transform ---------------------
// One block owns whole x lines: all K0 points along x of a yr x zr rectangle of (y, z)
// lines for gc consecutive complex slots (2 gc beads), 8,192 complex values in LDS. It
// accumulates the spline-weighted charges of every atom whose stencil reaches the
// rectangle (FP64 LDS atomics; each grid value is owned by exactly one block), transforms
// the lines along x in LDS and writes them: the forward x pass of the convolution happens
// without a round trip of the grid through memory, and the plane kernels and inverse
// passes that follow are unchanged. The rectangle's shape and the slots per block trade
// the spline work repeated for atoms near the rectangle's edges against the length of the
// contiguous pieces written (launch shapes picked by the autotuner). The candidate atoms
// are found from the tile bins (one thread per tile range, then a scan) and sorted by the
// offset of their centroid's stencil base from the rectangle, so that the lanes of a
// wavefront visit the same stencil rows.
constexpr int SX_E = 8192;                  // complex values of one block
constexpr int SX_NT = 1024;

struct SpreadXArgs {
  int N, P, K0, K1, K2, Pc, nt0, nt1, nt2;
  int yr, zr, gc;             // rectangle of (y, z) lines and complex slots per block
  int ny, nz;                 // rectangles along y and z
  const double* x;            // [3][N][P]
  double2* grid;              // [K0][K1][K2][Pc], written x-transformed
  const double* charge;
  const double4* cent;
  double L[3], KoL[3];
  const NlCtrl* ctrl;         // spread_m: largest bead-centroid base offset this step
  const int* tile_start; const int* tile_atoms;
  const double2* tw;          // [K0] twiddles of the x axis
  int remap;                  // blocks are a multiple of 8: XCD-contiguous block order
  int pairs;                  // write slot-pair planes [K0][Pc/2][K1][K2][2] instead
};

template <int ORDER, int K>
__global__ __launch_bounds__(SX_NT) void k_spread_x(SpreadXArgs A) {
  constexpr int CAP = 2048;                 // compacted atoms per round
  constexpr int MAXR = 160;                 // candidate tile ranges (checked by the launcher)
  constexpr int NBIN = SX_NT;               // candidate classes of the sort
  __shared__ double2 buf[SX_E];
  __shared__ double2 stw[K];
  __shared__ int cand[CAP];
  __shared__ int ckey[CAP];                 // class of each candidate, then the sorted atoms
  __shared__ int hist[NBIN];
  __shared__ int ncand;
  __shared__ int tofs[MAXR + 1], tbeg[MAXR];
  __shared__ int nranges;
  __shared__ int wsum[(MAXR + 63) / 64];
  __shared__ int wtot[SX_NT / 64];
  double* acc = reinterpret_cast<double*>(buf);        // [x][yl][zl][2 gc]
  const int tid = threadIdx.x, lane = tid & 63;
  const int lb = A.remap ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int yr = A.yr, zr = A.zr, gc = A.gc, gb = 2 * gc;
  const int rect = lb % (A.ny * A.nz), grp = lb / (A.ny * A.nz);
  const int y0 = (rect / A.nz) * yr, z0 = (rect % A.nz) * zr, c0 = grp * gc;
  const int NSr = yr * zr * gc;             // series of the block (= SX_E / K)
  for (int k = tid; k < SX_E; k += SX_NT) buf[k] = make_double2(0.0, 0.0);
  for (int k = tid; k < K; k += SX_NT) stw[k] = A.tw[k];
  const int m = min(A.ctrl->spread_m, QHP_TB);  // larger offsets are flagged by the binning
  // a stencil with base b covers b - ORDER + 1 .. b: it reaches [lo, lo + n) when b lies in
  // [lo, lo + n + ORDER - 2]; centroid bases widened by m points either way
  const int ylo = y0 - m, yn = yr + ORDER - 1 + 2 * m;
  const int zlo = z0 - m, zn = zr + ORDER - 1 + 2 * m;
  {
    // ranges of binned atoms: every x tile; the y tiles of [ylo, ylo + yn) (all if that
    // spans the axis); for each, the z tiles of [zlo, zlo + zn) as one or two runs. One
    // thread per range reads its bounds, an exclusive scan of the lengths places them
    // (empty ranges are kept: the search below never lands on one).
    const int ys = ylo & (A.K1 - 1), zs = zlo & (A.K2 - 1);
    const int ty0 = yn >= A.K1 ? 0 : ys / QHP_TB;
    const int tyn = yn >= A.K1 ? A.nt1 : min(A.nt1, (ys + yn - 1) / QHP_TB - ty0 + 1);
    int zp0[2] = {0, 0}, zp1[2] = {A.nt2, A.nt2}, nzp = 1;
    if (zn < A.K2) {
      const int za = zs / QHP_TB, zb = (zs + zn - 1) / QHP_TB;   // zb may pass the last tile
      if (zb < A.nt2) { zp0[0] = za; zp1[0] = zb + 1; }
      else { zp0[0] = za; zp1[0] = A.nt2; zp1[1] = min(za, zb - A.nt2 + 1); nzp = 2; }
    }
    // at most MAXR ranges (the launcher's bound on x tiles x y tiles x 2)
    const int nr = min(A.nt0 * tyn * nzp, MAXR);
    int len = 0, beg = 0;
    if (tid < nr) {
      const int pz = tid % nzp, q = (tid / nzp) % tyn, tx = tid / (nzp * tyn);
      const int base = (tx * A.nt1 + (ty0 + q) % A.nt1) * A.nt2;
      beg = A.tile_start[base + zp0[pz]];
      len = A.tile_start[base + zp1[pz]] - beg;
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    if (lane == 63 && (tid >> 6) < (MAXR + 63) / 64) wsum[tid >> 6] = incl;
    __syncthreads();
    if (tid < nr) {
      int off = incl - len;
      for (int w = 0; w < (tid >> 6); ++w) off += wsum[w];
      tbeg[tid] = beg;
      tofs[tid] = off;
      if (tid == nr - 1) { tofs[nr] = off + len; nranges = nr; }
    }
  }
  __syncthreads();
  const int nr = nranges, total = tofs[nr];
  const int Kd[3] = {A.K0, A.K1, A.K2};
  const int nb = min(gb, A.P - 2 * c0);     // beads of the block (P = 1: one)
  // candidate classes: the centroid base's offsets (dy, dz) from (ylo, zlo), merged into
  // NBIN ordered classes when there are more
  const int nzk = min(zn, A.K2), nkey = max(min(yn, A.K1) * nzk, NBIN);
  const int lgb = __builtin_ctz((unsigned)gb);
  int pos = 0;
  for (;;) {
    // 1) atoms whose centroid base lies in the widened y and z ranges
    if (tid == 0) ncand = 0;
    __syncthreads();
    while (pos < total && ncand <= CAP - SX_NT) {
      const int p = pos + tid;
      bool hit = false;
      int a = -1, key = 0;
      if (p < total) {
        int lo = 0, hi = nr;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (tofs[mid] <= p) lo = mid; else hi = mid;
        }
        a = A.tile_atoms[tbeg[lo] + (p - tofs[lo])];
        const double4 c = A.cent[a];
        const int by = base_of(c.y, A.KoL[1], A.K1), bz = base_of(c.z, A.KoL[2], A.K2);
        const int dy = (by - ylo) & (A.K1 - 1), dz = (bz - zlo) & (A.K2 - 1);   // K powers of two
        hit = (yn >= A.K1 || dy < yn) && (zn >= A.K2 || dz < zn);
        key = (int)((long)(dy * nzk + dz) * NBIN / nkey);
      }
      const unsigned long long bal = __ballot(hit);
      int off = 0;
      if (lane == 0 && bal) off = atomicAdd(&ncand, __popcll(bal));
      off = __shfl(off, 0);
      if (hit) {
        const int k = off + __popcll(bal & ((1ull << lane) - 1ull));
        cand[k] = a;
        ckey[k] = key;
      }
      pos += SX_NT;
      __syncthreads();
    }
    const bool more = pos < total;
    const int nc = ncand;
    // counting sort of the candidates by the (y, z) offset of their centroid base from the
    // rectangle: the lanes of a wavefront then mostly share which stencil rows fall on the
    // block's lines, and the row loop below runs uniformly over those rows only
    for (int k = tid; k < NBIN; k += SX_NT) hist[k] = 0;
    __syncthreads();
    for (int k = tid; k < nc; k += SX_NT) atomicAdd(&hist[ckey[k]], 1);
    __syncthreads();
    {
      const int h = hist[tid];              // NBIN = SX_NT: one class per thread
      int incl = h;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
      }
      if (lane == 63) wtot[tid >> 6] = incl;
      __syncthreads();
      int off = incl - h;
      for (int w = 0; w < (tid >> 6); ++w) off += wtot[w];
      hist[tid] = off;
    }
    constexpr int PER = CAP / SX_NT;
    int ka[PER], kk[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int k = tid + r * SX_NT;
      ka[r] = k < nc ? cand[k] : -1;
      kk[r] = k < nc ? ckey[k] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r)
      if (ka[r] >= 0) ckey[atomicAdd(&hist[kk[r]], 1)] = ka[r];
    __syncthreads();
    // 2) every compacted atom at every bead of the block: spline weights, the points of
    //    its stencil on the block's lines
    for (int it = tid; it < nc * gb; it += SX_NT) {
      const int bl = it & (gb - 1), b = 2 * c0 + bl;       // gb: a power of two
      if (bl >= nb) continue;
      const int a = ckey[it >> lgb];
      int base[3];
      double fr[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double u = grid_coord(A.x[((size_t)d * A.N + a) * A.P + b], A.KoL[d], Kd[d]);
        const double fl = floor(u);
        base[d] = isfinite(fl) ? min(max((int)fl, 0), Kd[d]) : 0;
        fr[d] = u - fl;
      }
      // the stencil rows on the rectangle (nothing to do for most beads of edge atoms)
      int ry[ORDER], rz[ORDER];
      bool any_y = false, any_z = false;
#pragma unroll
      for (int t = 0; t < ORDER; ++t) {
        ry[t] = (base[1] - t - y0) & (A.K1 - 1);
        rz[t] = (base[2] - t - z0) & (A.K2 - 1);
        any_y = any_y || ry[t] < yr;
        any_z = any_z || rz[t] < zr;
      }
      if (!(any_y && any_z)) continue;
      double w[3][ORDER], dw[3][ORDER];
#pragma unroll
      for (int d = 0; d < 3; ++d) bspline<ORDER>(fr[d], w[d], dw[d]);
      const double qa = A.charge[a];
      int xk[ORDER];
#pragma unroll
      for (int t = 0; t < ORDER; ++t) xk[t] = ((base[0] - t) & (A.K0 - 1)) * (NSr * 2);
#pragma unroll
      for (int ty = 0; ty < ORDER; ++ty) {
        if (ry[ty] >= yr) continue;
        const double wy = qa * w[1][ty];
#pragma unroll
        for (int tz = 0; tz < ORDER; ++tz) {
          if (rz[tz] >= zr) continue;
          const double wyz = wy * w[2][tz];
          double* row = acc + (ry[ty] * zr + rz[tz]) * gb + bl;
#pragma unroll
          for (int tx = 0; tx < ORDER; ++tx) atomicAdd(row + xk[tx], wyz * w[0][tx]);
        }
      }
    }
    __syncthreads();
    if (!more) break;
  }
  // 3) forward transform of every line along x in LDS, then the lines to the grid
  GridIO<K> io{A.grid, 0, 0};
  if (NSr == SX_E / K)
    fft_stages<K, SX_E / K, false, 1, false, false, false, SX_NT>(buf, stw, tid, io, nullptr, 0);
  const int KK = A.K1 * A.K2;
  if (A.pairs) {
    // slot-pair planes: consecutive threads take the two slots of a point, then z
    const int Gg = A.Pc >> 1;
    for (int k = tid; k < SX_E; k += SX_NT) {
      const int s2 = k & 1, zl = (k >> 1) % zr, r = (k >> 1) / zr;
      const int yl = r % yr, gl = (r / yr) % (gc >> 1), e = r / (yr * (gc >> 1));
      const int c = c0 + 2 * gl + s2;
      const size_t pl = (size_t)e * Gg + (c >> 1);
      A.grid[(pl * KK + (size_t)(y0 + yl) * A.K2 + (z0 + zl)) * 2 + s2] =
          buf[e * NSr + (yl * zr + zl) * gc + 2 * gl + s2];
    }
    return;
  }
  for (int k = tid; k < SX_E; k += SX_NT) {
    const int e = k / NSr, sr = k % NSr;
    const int cl = sr % gc, zl = (sr / gc) % zr, yl = sr / (gc * zr);
    A.grid[((size_t)e * KK + (size_t)(y0 + yl) * A.K2 + (z0 + zl)) * A.Pc + c0 + cl] = buf[k];
  }
}

// Inverse x transform from slot-pair planes [K0][Pc/2][K1][K2][2] to the point-major grid
// [K0][K1][K2][Pc] the gather reads: one block holds a run of (y, z) lines for every slot
// and all x (8,192 complex values); it reads 256-byte runs of each pair plane and writes
// whole point rows. The layout change rides on the pass that reads and writes the grid
// anyway.
template <int K>
__global__ __launch_bounds__(SX_NT) void k_fft_x_pairs(const double2* src, double2* dst,
                                                       const double2* tw, int KK, int Pc,
                                                       int lgI, int remap) {
  constexpr int NS = SX_E / K;
  __shared__ double2 buf[SX_E];
  __shared__ double2 stw[K];
  const int tid = threadIdx.x;
  const int lb = remap ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int lines = NS / Pc, first = lb * lines, Gg = Pc >> 1;
  for (int k = tid; k < K; k += SX_NT) stw[k] = tw[k];
  for (int k = tid; k < SX_E; k += SX_NT) {
    const int s2 = k & 1, l = (k >> 1) % lines, r = (k >> 1) / lines;
    const int g = r % Gg, e = r / Gg;
    buf[e * NS + l * Pc + 2 * g + s2] = src[(((size_t)e * Gg + g) * KK + first + l) * 2 + s2];
  }
  __syncthreads();
  GridIO<K> io{dst, (long)first * Pc, lgI};
  fft_stages<K, NS, true, 1, false, true, false, SX_NT>(buf, stw, tid, io, nullptr, 0);
}

// ------------------------- fused y-z convolution of one x plane ------------------------
// After the forward x pass, everything the reciprocal sum does along y and z for a fixed
// x frequency k0 is local to that plane: forward transforms along z and y, the product
// with G(k0, k1, k2), inverse transforms along y and z. One block holds the K x K plane of
// NB complex slots in LDS and does all of it, so the grid crosses HBM twice for the four
// transforms instead of six times.

// 8-point DFT in registers, natural order in and out (forward: exp(-2 pi i / 8)).
template <bool INV>
QHP_DEV void dft8(double2* v) {
  dft4<INV>(v[0], v[2], v[4], v[6]);
  dft4<INV>(v[1], v[3], v[5], v[7]);
  const double h = 0.70710678118654752440;
  const double sg = INV ? 1.0 : -1.0;
  const double2 o0 = v[1];
  const double2 o1 = cmul(v[3], make_double2(h, sg * h));
  const double2 o2 = cmul(v[5], make_double2(0.0, sg));
  const double2 o3 = cmul(v[7], make_double2(-h, sg * h));
  const double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// K-point transforms (K = 8 B, B = 4 or 8) of NSER series held in LDS, series q's element
// e at buf[off(q) + e * es]. Cooley-Tukey with x[B n1 + n2]: DFT_8 over n1 for every n2,
// twiddle W_K^(n2 k1), written back in place (element B k1 + n2); then DFT_B over n2 for
// every k1, giving X[k1 + 8 k2]. NT_ threads; the second step's tasks stay in registers
// across the barrier that separates its reads from its writes.
template <int K, int NSER, int NT_, bool INV, class Off>
QHP_DEV void lds_fft(double2* buf, const double2* tw, Off off, int es) {
  constexpr int B = K / 8;
  static_assert(B == 4 || B == 8, "K must be 32 or 64");
  constexpr int TA = NSER * B, TB = NSER * 8;
  constexpr int IA = (TA + NT_ - 1) / NT_, IB = (TB + NT_ - 1) / NT_;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const int t = tid + i * NT_, n2 = t % B, q = t / B;
    if (TA % NT_ != 0 && t >= TA) break;
    double2* p = buf + off(q) + n2 * es;
    double2 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = p[r * B * es];
    dft8<INV>(v);
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) {
      double2 w = tw[n2 * k1];
      if (INV) w.y = -w.y;
      v[k1] = cmul(v[k1], w);
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) p[r * B * es] = v[r];
  }
  __syncthreads();
  double2 v[IB][B];
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    const int t = tid + i * NT_, k1 = t % 8, q = t / 8;
    if (TB % NT_ != 0 && t >= TB) break;
    const double2* p = buf + off(q) + (B * k1) * es;
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) v[i][n2] = p[n2 * es];
    if constexpr (B == 8) {
      dft8<INV>(v[i]);
    } else {
      dft4<INV>(v[i][0], v[i][1], v[i][2], v[i][3]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    const int t = tid + i * NT_, k1 = t % 8, q = t / 8;
    if (TB % NT_ != 0 && t >= TB) break;
    double2* p = buf + off(q) + k1 * es;
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) p[(8 * k2) * es] = v[i][k2];
  }
  __syncthreads();
}

struct FftYZArgs {
  double2* grid;           // [planes][K][K][pc]
  const double2* tw;       // [K] exp(-2 pi i m / K) (y and z share it: K1 = K2)
  const double* G;         // [K0][K][K]
  int pc;                  // complex slots per grid point
  int gdiv;                // grid planes per x frequency (1; slot-pair planes: Pc / 2)
};

constexpr int YZ_NT = 1024;

// threads of the generic plane kernel: one per second-step task, at most 1,024
template <int K, int NB>
constexpr int yz_threads() { return K * NB * 8 < YZ_NT ? K * NB * 8 : YZ_NT; }

template <int K, int NB>
__global__ __launch_bounds__((yz_threads<K, NB>())) void k_fft_yz(FftYZArgs A) {
  constexpr int NTH = yz_threads<K, NB>();
  constexpr int ROW = K * NB + NB;        // one k1 row of LDS, padded against bank conflicts
  __shared__ double2 buf[K * ROW];
  __shared__ double2 stw[K];
  const int tid = threadIdx.x;
  const int groups = A.pc / NB;
  const int lb = xcd_block(blockIdx.x, gridDim.x);   // the slot groups of a plane: one XCD
  const int k0 = lb / groups, s0 = (lb % groups) * NB;
  for (int m = tid; m < K; m += NTH) stw[m] = A.tw[m];
  const size_t plane = (size_t)k0 * K * K, gplane = (size_t)(k0 / A.gdiv) * K * K;
  constexpr int PER = K * K * NB / NTH;            // values per thread (a power of two)
  static_assert(PER * NTH == K * K * NB, "plane size");
  {
    double2 r[PER];                                  // all loads in flight, then to LDS
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int l = tid + i * NTH, s = l % NB, pt = l / NB;
      r[i] = A.grid[(plane + pt) * A.pc + s0 + s];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int l = tid + i * NTH, s = l % NB, k2 = (l / NB) % K, k1 = l / (NB * K);
      buf[k1 * ROW + k2 * NB + s] = r[i];
    }
  }
  __syncthreads();
  // series along z: q = (k1, s); along y: q = (k2, s)
  auto offz = [](int q) { return (q / NB) * ROW + q % NB; };
  auto offy = [](int q) { return (q / NB) * NB + q % NB; };
  lds_fft<K, K * NB, NTH, false>(buf, stw, offz, NB);
  lds_fft<K, K * NB, NTH, false>(buf, stw, offy, ROW);
  for (int l = tid; l < K * K * NB; l += NTH) {
    const int s = l % NB, k2 = (l / NB) % K, k1 = l / (NB * K);
    const double g = A.G[gplane + (size_t)k1 * K + k2];
    double2& v = buf[k1 * ROW + k2 * NB + s];
    v.x *= g; v.y *= g;
  }
  __syncthreads();
  lds_fft<K, K * NB, NTH, true>(buf, stw, offy, ROW);
  lds_fft<K, K * NB, NTH, true>(buf, stw, offz, NB);
  double2 r[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int l = tid + i * NTH, s = l % NB, k2 = (l / NB) % K, k1 = l / (NB * K);
    r[i] = buf[k1 * ROW + k2 * NB + s];
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int l = tid + i * NTH, s = l % NB, pt = l / NB;
    A.grid[(plane + pt) * A.pc + s0 + s] = r[i];
  }
}

// K = 64, one or two slots: the same transforms with one (series, index) task per thread and
// each 8 x 8 step kept in registers where the data layout allows: the forward z step
// reads the grid directly, the forward y step's second half, the product with G and the
// inverse y step's first half run on the same registers (the eight outputs X[k1 + 8 k2]
// of one thread are exactly the eight inputs x[8 n1 + n2], n2 = k1, of the inverse
// step), and the last inverse z step writes the grid directly.
template <int NB>
__global__ __launch_bounds__(512 * NB) __attribute__((amdgpu_waves_per_eu(4))) void k_fft_yz64(FftYZArgs A) {
  constexpr int K = 64, ROW = K * NB + 2;   // padded rows: conflict-free for NB = 1 and 2
  __shared__ double2 buf[K * ROW];
  __shared__ double2 stw[K];
  const int tid = threadIdx.x, j = tid & 7, q = tid >> 3, s = q % NB, r = q / NB;
  const int groups = A.pc / NB;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int k0 = lb / groups, s0 = (lb % groups) * NB;
  if (tid < K) stw[tid] = A.tw[tid];
  const size_t plane = (size_t)k0 * K * K, gplane = (size_t)(k0 / A.gdiv) * K * K;
  // Point (k1, k2) of slot s sits at LDS row sw(k1), column sw(k2), sw(e) permuting the
  // low three bits of e by its high three (e ^ (e >> 3) within each group of eight):
  // every access below reads or writes elements 8a + b with one of a, b running over the
  // eight lanes of a series, and the permutation spreads those over distinct banks.
  auto sw = [](int e) { return (e & 56) | ((e ^ (e >> 3)) & 7); };
  // z series of this thread: row k1 = r, slot s; y series: column k2 = r, slot s
  double2* zs = buf + sw(r) * ROW + s;      // element e at zs[sw(e) * NB]
  double2* ys = buf + sw(r) * NB + s;       // element e at ys[sw(e) * ROW]
  double2 v[8];
  // 1. forward z, first half, from the grid: x[8 n1 + j]
  {
    const double2* g = A.grid + (plane + (size_t)r * K + j) * A.pc + s0 + s;
#pragma unroll
    for (int n1 = 0; n1 < 8; ++n1) v[n1] = g[(size_t)(8 * n1) * A.pc];
  }
  __syncthreads();                          // twiddles
  // every twiddle step of this thread uses W^(j k), k = 1..7: kept in registers
  double2 wj[8];
#pragma unroll
  for (int k = 1; k < 8; ++k) wj[k] = stw[j * k];
  auto tw8 = [&](double2* v, int, bool inv) {
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      double2 w = wj[k];
      if (inv) w.y = -w.y;
      v[k] = cmul(v[k], w);
    }
  };
  dft8<false>(v);
  tw8(v, j, false);
#pragma unroll
  for (int k = 0; k < 8; ++k) zs[sw(8 * k + j) * NB] = v[k];
  __syncthreads();
  // 2. forward z, second half: elements 8 j + n2 -> X[j + 8 k2]
#pragma unroll
  for (int n2 = 0; n2 < 8; ++n2) v[n2] = zs[sw(8 * j + n2) * NB];
  dft8<false>(v);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) zs[sw(j + 8 * k) * NB] = v[k];
  __syncthreads();
  // 3. forward y, first half, in place
#pragma unroll
  for (int n1 = 0; n1 < 8; ++n1) v[n1] = ys[sw(8 * n1 + j) * ROW];
  dft8<false>(v);
  tw8(v, j, false);
#pragma unroll
  for (int k = 0; k < 8; ++k) ys[sw(8 * k + j) * ROW] = v[k];
  __syncthreads();
  // 4. forward y second half, x G, inverse y first half (n2 = j)
#pragma unroll
  for (int n2 = 0; n2 < 8; ++n2) v[n2] = ys[sw(8 * j + n2) * ROW];
  dft8<false>(v);
#pragma unroll
  for (int k = 0; k < 8; ++k) {             // v[k] = X[k1 = j + 8 k] at column k2 = r
    const double gv = A.G[gplane + (size_t)(j + 8 * k) * K + r];
    v[k].x *= gv; v[k].y *= gv;
  }
  dft8<true>(v);
  tw8(v, j, true);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) ys[sw(8 * k + j) * ROW] = v[k];
  __syncthreads();
  // 5. inverse y, second half
#pragma unroll
  for (int n2 = 0; n2 < 8; ++n2) v[n2] = ys[sw(8 * j + n2) * ROW];
  dft8<true>(v);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) ys[sw(j + 8 * k) * ROW] = v[k];
  __syncthreads();
  // 6. inverse z, first half, in place
#pragma unroll
  for (int n1 = 0; n1 < 8; ++n1) v[n1] = zs[sw(8 * n1 + j) * NB];
  dft8<true>(v);
  tw8(v, j, true);
#pragma unroll
  for (int k = 0; k < 8; ++k) zs[sw(8 * k + j) * NB] = v[k];
  __syncthreads();
  // 7. inverse z, second half, to the grid: X[j + 8 k2]
#pragma unroll
  for (int n2 = 0; n2 < 8; ++n2) v[n2] = zs[sw(8 * j + n2) * NB];
  dft8<true>(v);
  double2* g = A.grid + (plane + (size_t)r * K + j) * A.pc + s0 + s;
#pragma unroll
  for (int k = 0; k < 8; ++k) g[(size_t)(8 * k) * A.pc] = v[k];
}


// ---------- grids whose edges are not powers of two (prime factors 2, 3, 5, 7) ----------
// The same grid layout ([k0][k1][k2] points, the complex slots of a point contiguous) and
// the tiled spreading and gather kernels (which wrap their offsets for any edge); each
// axis transformed a few lines at a time in LDS by runtime mixed-radix stages, the last
// axis forward, times G and inverse in one visit.
// nl lines along an axis per block: the pc complex slots of their K points to LDS as
// nl pc series, transformed, and back. Line l covers the points
// (l / inner) K inner + (l mod inner) + e inner (point stride `inner`, the slots of a point
// contiguous). With inner > 1 the block's lines are nl neighbouring points of one plane
// (nl divides inner), so the slots of the nl lines at one e are contiguous; with
// inner = 1 each line is contiguous. Consecutive threads take consecutive addresses.
// PC (slots) and nl (lines, 2^lgnl) are powers of two: shifts and masks; the one division
// left, by K, is a double-precision multiply by 1/K (exact for these small integers)
template <int PC>
QHP_DEV void line_point(int i, int K, double invK, int lgnl, long inner, long l0, long base0,
                        int& j, int& e, int& sl, long& pt) {
  constexpr int LGPC = __builtin_ctz(PC);
  sl = i & (PC - 1);
  const int r = i >> LGPC;
  if (inner > 1) {
    j = r & ((1 << lgnl) - 1); e = r >> lgnl;
    pt = base0 + j + (long)e * inner;
  } else {
    j = (int)(((double)r + 0.5) * invK); e = r - j * K;
    pt = l0 * K + r;
  }
}

// mode 0: forward, 1: inverse, 2: forward, times G, inverse (one visit of the last axis)
template <int PC>
__global__ __launch_bounds__(NT) void k_fft_line_gen(double2* grid, const double2* tw,
                                                     const double* G, int K, long inner,
                                                     int lgnl, int mode) {
  extern __shared__ double2 lbuf[];
  constexpr int pc = PC;
  const int nl = 1 << lgnl;
  const double invK = 1.0 / K;
  const int ns = nl * pc, n = K * ns;
  double2* a = lbuf;
  double2* b = lbuf + (size_t)n;
  double2* stw = lbuf + 2 * (size_t)n;     // the axis' twiddles
  for (int k = threadIdx.x; k < K; k += NT) stw[k] = tw[k];
  const long l0 = (long)blockIdx.x * nl;
  const long base0 = (l0 / inner) * K * inner + (l0 % inner);
  for (int i = threadIdx.x; i < n; i += NT) {
    int j, e, sl;
    long pt;
    line_point<PC>(i, K, invK, lgnl, inner, l0, base0, j, e, sl, pt);
    a[(size_t)(j * pc + sl) * K + e] = grid[pt * pc + sl];
  }
  __syncthreads();
  double2* r = qhp::fft_rt(a, b, K, ns, mode == 1, stw);
  if (mode == 2) {
    for (int i = threadIdx.x; i < n; i += NT) {
      int j, e, sl;
      long pt;
      line_point<PC>(i, K, invK, lgnl, inner, l0, base0, j, e, sl, pt);
      double2& v = r[(size_t)(j * pc + sl) * K + e];
      const double g = G[pt];
      v.x *= g;
      v.y *= g;
    }
    __syncthreads();
    r = qhp::fft_rt(r, r == a ? b : a, K, ns, true, stw);
  }
  for (int i = threadIdx.x; i < n; i += NT) {
    int j, e, sl;
    long pt;
    line_point<PC>(i, K, invK, lgnl, inner, l0, base0, j, e, sl, pt);
    grid[pt * pc + sl] = r[(size_t)(j * pc + sl) * K + e];
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

static hipError_t fft_pass(qhp_ctx* c, int axis, int mode, int pc, double2* grid) {
  const int K = c->K[axis];
  long inner = pc;
  for (int d = axis + 1; d < 3; ++d) inner *= c->K[d];
  const long total = (long)c->K[0] * c->K[1] * c->K[2] * pc;
  const long series = total / K;
  const int NS = FFT_E / K;
  if (series % NS) return hipErrorInvalidValue;
  FftArgs A;
  A.grid = grid; A.tw = c->tw[axis]; A.G = c->influence;
  A.lgI = __builtin_ctzl((unsigned long)inner); A.lgpc = __builtin_ctz((unsigned)pc);
  A.efast = inner < 16;
  const unsigned nb = (unsigned)(series / NS);
  if (mode == 0) { QHP_SWITCH_K(K, hipLaunchKernelGGL((k_fft_pass<KK, 0>), nb, NT, 0, c->stream, A)); }
  else if (mode == 1) { QHP_SWITCH_K(K, hipLaunchKernelGGL((k_fft_pass<KK, 1>), nb, NT, 0, c->stream, A)); }
  else { QHP_SWITCH_K(K, hipLaunchKernelGGL((k_fft_pass<KK, 2>), nb, NT, 0, c->stream, A)); }
  return hipGetLastError();
}

// The reciprocal-space convolution of a spread grid: forward 3D transform, product with
// G, inverse transform (unnormalised: G carries the factors). Square y-z planes of 32 or
// 64 points take the fused plane kernel between the two x passes (unless the autotuner
// found the one-axis passes faster: fft_nb < 0); other grids take five one-axis passes
// (the z pass fusing G).
// Grid edges that are not powers of two: five passes of a few lines per block (the last
// axis forward, times G and inverse in one visit).
static hipError_t convolve_lines(qhp_ctx* c, int pc, double2* grid) {
  const size_t npts = (size_t)c->K[0] * c->K[1] * c->K[2];
  auto pass = [&](int axis, int mode) {
    long inner = 1;
    for (int d = axis + 1; d < 3; ++d) inner *= c->K[d];
    const int K = c->K[axis];
    const long lines = (long)(npts / K);
    // lines per block: a power of two dividing the plane's points (or the line count),
    // at most 1,024 complex values per LDS buffer (2,048: 181 against 153 us for the
    // 112^3 transforms of the one-bead 21,952-water box, 512: 176 us)
    const long div = inner > 1 ? inner : lines;
    int lgnl = 0;
    while ((long)2 * (2 << lgnl) * K * pc <= 2048 && div % (2 << lgnl) == 0) ++lgnl;
    const unsigned blocks = (unsigned)(lines >> lgnl);
    const size_t lds = ((size_t)2 * (1 << lgnl) * K * pc + K) * sizeof(double2);
#define LINE_CALL(PCV)                                                                        \
    hipLaunchKernelGGL((k_fft_line_gen<PCV>), blocks, NT, lds, c->stream, grid, c->tw[axis], \
                       c->influence, K, inner, lgnl, mode)
    switch (pc) {
      case 1: LINE_CALL(1); break;
      case 2: LINE_CALL(2); break;
      case 4: LINE_CALL(4); break;
      case 8: LINE_CALL(8); break;
      case 16: LINE_CALL(16); break;
      default: LINE_CALL(32); break;
    }
#undef LINE_CALL
  };
  pass(0, 0);
  pass(1, 0);
  pass(2, 2);                        // forward z, the product with G, inverse z
  pass(1, 1);
  pass(0, 1);
  return hipGetLastError();
}

static hipError_t convolve(qhp_ctx* c, int pc, double2* grid, bool x_done = false) {
  if (c->spme_generic) return convolve_lines(c, pc, grid);
  const int K = c->K[1];
  int nb = 0;                                      // slots per plane block (0: five passes)
  if (K == c->K[2] && (K == 64 || K == 32)) {
    const int cap = K == 64 ? 2 : 8;               // 8,192 complex values in LDS
    if (c->fft_nb > 0) {
      nb = c->fft_nb < cap ? c->fft_nb : cap;
    } else if (c->fft_nb == 0) {                   // default: 64^2 planes two slots; 32^2
      nb = K == 64 ? 2 : 1;                        // planes as many as keep 256 blocks
      if (K == 32)
        while (nb < cap && (long)c->K[0] * (pc / (2 * nb)) >= 256) nb *= 2;
    }
    if (nb > pc) nb = pc;
  }
  hipError_t e;
  if (!x_done && (e = fft_pass(c, 0, 0, pc, grid)) != hipSuccess) return e;
  if (nb) {
    FftYZArgs A;
    A.grid = grid; A.tw = c->tw[1]; A.G = c->influence; A.pc = pc; A.gdiv = 1;
    const unsigned blocks = (unsigned)(c->K[0] * (pc / nb));
#define YZ_CALL(KK, NBV)                                                                    \
    hipLaunchKernelGGL((k_fft_yz<KK, NBV>), blocks, (yz_threads<KK, NBV>()), 0, c->stream, A)
    if (K == 64) {
      if (nb == 1) hipLaunchKernelGGL(k_fft_yz64<1>, blocks, 512, 0, c->stream, A);
      else hipLaunchKernelGGL(k_fft_yz64<2>, blocks, 1024, 0, c->stream, A);
    } else {
      if (nb == 1) YZ_CALL(32, 1);
      else if (nb == 2) YZ_CALL(32, 2);
      else if (nb == 4) YZ_CALL(32, 4);
      else YZ_CALL(32, 8);
    }
#undef YZ_CALL
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    if ((e = fft_pass(c, 1, 0, pc, grid)) != hipSuccess) return e;
    if ((e = fft_pass(c, 2, 2, pc, grid)) != hipSuccess) return e;
    if ((e = fft_pass(c, 1, 1, pc, grid)) != hipSuccess) return e;
  }
  return fft_pass(c, 0, 1, pc, grid);
}

// Block shape of the fused spreading and forward x transform: gc complex slots (2 gc beads,
// from the spreading beads per block of qhp_set_launch / the autotuner; default 4 slots)
// and a yr x zr rectangle of (y, z) lines with yr zr gc K0 = 8,192, zr = 8 z tiles of the
// launch shape (default one tile of 8 points) where that fits. Not applicable (false) when
// the grid or the slots do not fill such blocks, or when the binned atoms a block scans
// could exceed its list of tile ranges (centroid-bead base offsets up to one tile, which
// the normal-mode kernel enforces).
static bool spread_x_shape(const qhp_ctx* c, int P, int pc, SpreadXArgs& X) {
  const int K0 = c->K[0], K1 = c->K[1], K2 = c->K[2];
  if (c->spread_gb < 0) return false;                  // the tiled spreading was asked for
  // one slot (a single bead): the tiled spreading with the separate x pass measured faster
  if (pc < 2 || K0 < 16 || K0 > 128) return false;
  int gc = c->spread_gb > 0 ? std::max(1, c->spread_gb / 2) : 4;
  gc = std::min(gc, pc);
  if ((long)K0 * gc > SX_E) return false;
  const long lines = SX_E / ((long)K0 * gc);
  if (lines > (long)K1 * K2) return false;
  int zr = std::min<long>(lines, std::min(K2, QHP_TB * (c->spread_z > 0 ? c->spread_z : 1)));
  long yr = lines / zr;
  if (yr > K1) { yr = K1; zr = (int)(lines / K1); }
  if (zr > K2 || yr * zr != lines) return false;
  const int yn = (int)yr + c->p.pme_order - 1 + 2 * QHP_TB;
  const int nt1 = K1 / QHP_TB, tyn = std::min(nt1, (yn + QHP_TB - 2) / QHP_TB + 1);
  if ((K0 / QHP_TB) * tyn * 2 > 160) return false;
  X.gc = gc; X.yr = (int)yr; X.zr = zr; X.ny = K1 / (int)yr; X.nz = K2 / zr;
  (void)P;
  return true;
}

hipError_t launch_spme(qhp_ctx* c, bool energy, int bead, const BeadSet* bs, int part) {
  const bool plain = bead >= 0;
  const BeadSet B = bs ? *bs : full_beads(c);
  const int P = plain ? 1 : B.P;
  const int pc = plain ? 1 : B.Pc;
  const int N = c->N;
  SpmeArgs A;
  A.N = N; A.K0 = c->K[0]; A.K1 = c->K[1]; A.K2 = c->K[2]; A.Pc2 = 2 * pc;
  A.order = c->tile_atoms;
  A.x = plain ? c->x + (size_t)bead * 3 * N : B.x;
  A.g = plain ? c->g + (size_t)bead * 3 * N : B.g;
  A.grid = (double*)c->grid; A.charge = c->d_charge;
  for (int d = 0; d < 3; ++d) A.L[d] = c->p.box[d];
  A.energy = plain ? c->energy + (size_t)bead * QHP_NTERMS : B.energy;
  A.dq = c->pg_dq;
  const bool pg = !plain && B.pgrad;
  const unsigned nb = (unsigned)(((size_t)N * P + NT - 1) / NT);
  hipEvent_t ev = nullptr;
  if ((part & SPME_FRONT) && c->spme_generic) {
    // grid edges that are not powers of two: the plain path
    prof_begin(c, QHP_PROF_SPREAD, &ev);
    if (plain) {     // one bead of the plain mode: bin its atoms here (as below)
      TileArgs T;
      T.N = N; T.P = 1; T.K0 = c->K[0]; T.K1 = c->K[1]; T.K2 = c->K[2];
      T.nt0 = c->K[0] / TB; T.nt1 = c->K[1] / TB; T.nt2 = c->K[2] / TB; T.order = c->p.pme_order;
      T.x = A.x; T.cent = nullptr;
      for (int d = 0; d < 3; ++d) { T.L[d] = c->p.box[d]; T.KoL[d] = c->K[d] / c->p.box[d]; }
      T.tile_of = c->tile_of; T.tile_count = c->tile_count; T.tile_fill = c->tile_fill;
      T.tile_start = c->tile_start; T.tile_atoms = c->tile_atoms; T.ntiles = c->ntiles;
      hipLaunchKernelGGL(k_tile_bin, (N + 255) / 256, 256, 0, c->stream, T);
      hipLaunchKernelGGL(k_tile_scan, 1, 256, 0, c->stream, T);
      hipLaunchKernelGGL(k_tile_scatter, (N + 255) / 256, 256, 0, c->stream, T);
    }
    {
      // the tiled spreading (atoms binned by the list stage; every grid point written once):
      // gb beads per block, z tiles along z dividing the tile count
      TSpreadArgs S;
      S.N = N; S.P = P; S.K0 = c->K[0]; S.K1 = c->K[1]; S.K2 = c->K[2];
      S.nt1 = c->K[1] / TB; S.nt2 = c->K[2] / TB; S.Pc2 = 2 * pc;
      S.x = A.x; S.grid = A.grid; S.charge = c->d_charge;
      S.cent = plain ? nullptr : c->cent; S.ctrl = c->ctrl;
      for (int d = 0; d < 3; ++d) { S.L[d] = c->p.box[d]; S.KoL[d] = c->K[d] / c->p.box[d]; }
      S.tile_start = c->tile_start; S.tile_atoms = c->tile_atoms;
      int gb = c->spread_gb > 0 ? c->spread_gb : 8;
      if (gb > P) gb = P;
      int z = c->spread_z > 0 ? c->spread_z : 1;
      while (z > 1 && (S.nt2 % z || z * gb > 16)) z >>= 1;
      const dim3 sgrid(c->ntiles / z, P / gb);
#define SPREAD_GEN(GBV, ZV)                                                                  \
      QHP_SWITCH_ORDER(c->p.pme_order, hipLaunchKernelGGL((k_spread_tiles<OO, GBV, false, ZV>),  \
                                                          sgrid, NT, 0, c->stream, S))
      switch (gb * 16 + z) {
        case 16 + 1: SPREAD_GEN(1, 1); break;
        case 16 + 2: SPREAD_GEN(1, 2); break;
        case 16 + 4: SPREAD_GEN(1, 4); break;
        case 16 + 8: SPREAD_GEN(1, 8); break;
        case 32 + 1: SPREAD_GEN(2, 1); break;
        case 32 + 2: SPREAD_GEN(2, 2); break;
        case 32 + 4: SPREAD_GEN(2, 4); break;
        case 32 + 8: SPREAD_GEN(2, 8); break;
        case 64 + 1: SPREAD_GEN(4, 1); break;
        case 64 + 2: SPREAD_GEN(4, 2); break;
        case 64 + 4: SPREAD_GEN(4, 4); break;
        case 128 + 1: SPREAD_GEN(8, 1); break;
        case 128 + 2: SPREAD_GEN(8, 2); break;
        case 256 + 1: SPREAD_GEN(16, 1); break;
        default: return hipErrorInvalidValue;
      }
#undef SPREAD_GEN
    }
    prof_end(c, QHP_PROF_SPREAD, ev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    prof_begin(c, QHP_PROF_FFT, &ev);
    if ((e = convolve(c, pc, c->grid)) != hipSuccess) return e;
    prof_end(c, QHP_PROF_FFT, ev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else if (part & SPME_FRONT) {
    prof_begin(c, QHP_PROF_SPREAD, &ev);
    {
      TileArgs T;
      T.N = N; T.P = P; T.K0 = c->K[0]; T.K1 = c->K[1]; T.K2 = c->K[2];
      T.nt0 = c->K[0] / TB; T.nt1 = c->K[1] / TB; T.nt2 = c->K[2] / TB; T.order = c->p.pme_order;
      T.x = A.x; T.cent = plain ? nullptr : c->cent;
      for (int d = 0; d < 3; ++d) { T.L[d] = c->p.box[d]; T.KoL[d] = c->K[d] / c->p.box[d]; }
      T.tile_of = c->tile_of; T.tile_count = c->tile_count; T.tile_fill = c->tile_fill;
      T.tile_start = c->tile_start; T.tile_atoms = c->tile_atoms; T.ntiles = c->ntiles;
      if (plain) {   // batched: the prep kernel of the neighbour-list stage has binned the atoms
        hipLaunchKernelGGL(k_tile_bin, (N + 255) / 256, 256, 0, c->stream, T);
        hipLaunchKernelGGL(k_tile_scan, 1, 256, 0, c->stream, T);
        hipLaunchKernelGGL(k_tile_scatter, (N + 255) / 256, 256, 0, c->stream, T);
      }
      SpreadXArgs X;
      if (!plain && spread_x_shape(c, P, pc, X)) {
        X.N = N; X.P = P; X.K0 = c->K[0]; X.K1 = c->K[1]; X.K2 = c->K[2]; X.Pc = pc;
        X.nt0 = T.nt0; X.nt1 = T.nt1; X.nt2 = T.nt2;
        X.x = A.x; X.charge = c->d_charge; X.cent = c->cent; X.ctrl = c->ctrl;
        for (int d = 0; d < 3; ++d) { X.L[d] = c->p.box[d]; X.KoL[d] = c->K[d] / c->p.box[d]; }
        X.tile_start = c->tile_start; X.tile_atoms = c->tile_atoms; X.tw = c->tw[0];
        // slot-pair planes for the y-z plane kernel when it applies
        const int K = c->K[1];
        const bool pairs = c->grid_l1 && pc >= 2 && X.gc % 2 == 0 && K == c->K[2] &&
                           (K == 64 || K == 32) && c->fft_nb >= 0 && SX_E % (c->K[0] * pc) == 0 &&
                           (long)SX_E / (c->K[0] * pc) <= (long)K * K;
        X.pairs = pairs;
        X.grid = pairs ? c->grid_l1 : c->grid;
        const unsigned blocks = (unsigned)(X.ny * X.nz * (pc / X.gc));
        X.remap = blocks % 8 == 0;
#define SPREADX_CALL(KK)                                                                      \
        QHP_SWITCH_ORDER(c->p.pme_order, hipLaunchKernelGGL((k_spread_x<OO, KK>), blocks, SX_NT, 0, \
                                                            c->stream, X))
        switch (c->K[0]) {
          case 16: SPREADX_CALL(16); break;
          case 32: SPREADX_CALL(32); break;
          case 64: SPREADX_CALL(64); break;
          case 128: SPREADX_CALL(128); break;
          default: return hipErrorInvalidValue;
        }
#undef SPREADX_CALL
        prof_end(c, QHP_PROF_SPREAD, ev);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        prof_begin(c, QHP_PROF_FFT, &ev);
        if (pairs) {
          // y-z planes of slot pairs (contiguous 2-slot planes), then the inverse x pass
          // that also returns the grid to the point-major layout
          const int nbs = c->fft_nb == 1 ? 1 : 2;
          FftYZArgs Y;
          Y.grid = c->grid_l1; Y.tw = c->tw[1]; Y.G = c->influence; Y.pc = 2; Y.gdiv = pc / 2;
          const unsigned yblocks = (unsigned)(c->K[0] * (pc / 2) * (2 / nbs));
          if (K == 64) {
            if (nbs == 1) hipLaunchKernelGGL(k_fft_yz64<1>, yblocks, 512, 0, c->stream, Y);
            else hipLaunchKernelGGL(k_fft_yz64<2>, yblocks, 1024, 0, c->stream, Y);
          } else {
            if (nbs == 1) hipLaunchKernelGGL((k_fft_yz<32, 1>), yblocks, (yz_threads<32, 1>()), 0, c->stream, Y);
            else hipLaunchKernelGGL((k_fft_yz<32, 2>), yblocks, (yz_threads<32, 2>()), 0, c->stream, Y);
          }
          const int KK = c->K[1] * c->K[2], lines = SX_E / (c->K[0] * pc);
          const unsigned xblocks = (unsigned)(KK / lines);
          const int lgI = __builtin_ctzl((unsigned long)KK * pc), remap = xblocks % 8 == 0;
          switch (c->K[0]) {
            case 16: hipLaunchKernelGGL(k_fft_x_pairs<16>, xblocks, SX_NT, 0, c->stream, c->grid_l1, c->grid, c->tw[0], KK, pc, lgI, remap); break;
            case 32: hipLaunchKernelGGL(k_fft_x_pairs<32>, xblocks, SX_NT, 0, c->stream, c->grid_l1, c->grid, c->tw[0], KK, pc, lgI, remap); break;
            case 64: hipLaunchKernelGGL(k_fft_x_pairs<64>, xblocks, SX_NT, 0, c->stream, c->grid_l1, c->grid, c->tw[0], KK, pc, lgI, remap); break;
            case 128: hipLaunchKernelGGL(k_fft_x_pairs<128>, xblocks, SX_NT, 0, c->stream, c->grid_l1, c->grid, c->tw[0], KK, pc, lgI, remap); break;
            default: return hipErrorInvalidValue;
          }
          if ((e = hipGetLastError()) != hipSuccess) return e;
        } else if ((e = convolve(c, pc, c->grid, true)) != hipSuccess) {
          return e;
        }
        prof_end(c, QHP_PROF_FFT, ev);
        goto gather;
      }
      TSpreadArgs S;
      S.N = N; S.P = P; S.K0 = c->K[0]; S.K1 = c->K[1]; S.K2 = c->K[2];
      S.nt1 = T.nt1; S.nt2 = T.nt2; S.Pc2 = 2 * pc;
      S.x = A.x; S.grid = A.grid; S.charge = c->d_charge;
      S.cent = plain ? nullptr : c->cent;
      S.ctrl = c->ctrl;
      for (int d = 0; d < 3; ++d) { S.L[d] = c->p.box[d]; S.KoL[d] = c->K[d] / c->p.box[d]; }
      S.tile_start = c->tile_start; S.tile_atoms = c->tile_atoms;
      // block shape: gb beads, z tiles along z (at most 16 x 8^3 points of LDS)
      int gb = c->spread_gb > 0 ? c->spread_gb : 8;
      if (gb > P) gb = P;
      int z = c->spread_z > 0 ? c->spread_z : 1;
      if (z > S.nt2) z = S.nt2;
      while (z * gb > 16) z >>= 1;
      const dim3 grid(c->ntiles / z, P / gb);
#define SPREAD_CALL(GBV, ZV)                                                                 \
      QHP_SWITCH_ORDER(c->p.pme_order, hipLaunchKernelGGL((k_spread_tiles<OO, GBV, false, ZV>),  \
                                                          grid, NT, 0, c->stream, S))
      switch (gb * 16 + z) {
        case 16 + 1: SPREAD_CALL(1, 1); break;
        case 16 + 2: SPREAD_CALL(1, 2); break;
        case 16 + 4: SPREAD_CALL(1, 4); break;
        case 16 + 8: SPREAD_CALL(1, 8); break;
        case 32 + 1: SPREAD_CALL(2, 1); break;
        case 32 + 2: SPREAD_CALL(2, 2); break;
        case 32 + 4: SPREAD_CALL(2, 4); break;
        case 32 + 8: SPREAD_CALL(2, 8); break;
        case 64 + 1: SPREAD_CALL(4, 1); break;
        case 64 + 2: SPREAD_CALL(4, 2); break;
        case 64 + 4: SPREAD_CALL(4, 4); break;
        case 128 + 1: SPREAD_CALL(8, 1); break;
        case 128 + 2: SPREAD_CALL(8, 2); break;
        case 256 + 1: SPREAD_CALL(16, 1); break;
        default: return hipErrorInvalidValue;
      }
#undef SPREAD_CALL
    }
    prof_end(c, QHP_PROF_SPREAD, ev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    prof_begin(c, QHP_PROF_FFT, &ev);
    if ((e = convolve(c, pc, c->grid)) != hipSuccess) return e;
    prof_end(c, QHP_PROF_FFT, ev);
  }
gather:
  if (!(part & SPME_GATHER)) return hipGetLastError();
  prof_begin(c, QHP_PROF_GATHER, &ev);
  if (P == 1) {
    const unsigned nbo = (unsigned)(((size_t)N * 8 + NT - 1) / NT);
    A.nblocks = (int)nbo;
    const unsigned nbo8 = (nbo + 7) / 8 * 8;
    QHP_SWITCH_ORDER(c->p.pme_order,
                     if (pg) hipLaunchKernelGGL((k_gather_one<OO, false, true>), nbo8, NT, 0, c->stream, A);
                     else if (energy) hipLaunchKernelGGL((k_gather_one<OO, true>), nbo8, NT, 0, c->stream, A);
                     else hipLaunchKernelGGL((k_gather_one<OO, false>), nbo8, NT, 0, c->stream, A));
    prof_end(c, QHP_PROF_GATHER, ev);
    return hipGetLastError();
  }
  A.nblocks = (int)nb;
  const unsigned nb8 = (nb + 7) / 8 * 8;
  QHP_SWITCH_P(P, QHP_SWITCH_ORDER(c->p.pme_order,
               if (pg) hipLaunchKernelGGL((k_gather<PP, OO, false, true>), nb8, NT, 0, c->stream, A);
               else if (energy) hipLaunchKernelGGL((k_gather<PP, OO, true>), nb8, NT, 0, c->stream, A);
               else hipLaunchKernelGGL((k_gather<PP, OO, false>), nb8, NT, 0, c->stream, A)));
  prof_end(c, QHP_PROF_GATHER, ev);
  return hipGetLastError();
}

hipError_t launch_spme_hvp(qhp_ctx* c, const double* u, double* hu, bool mix) {
  const int P = c->P, pc = c->Pc, N = c->N;
  if (!c->grid2) {
    const size_t n = (size_t)c->K[0] * c->K[1] * c->K[2] * pc;
    hipError_t e = hipMalloc((void**)&c->grid2, n * sizeof(double2));
    if (e != hipSuccess) { c->grid2 = nullptr; return e; }
  }
  TSpreadArgs S;
  S.N = N; S.P = P; S.K0 = c->K[0]; S.K1 = c->K[1]; S.K2 = c->K[2];
  S.nt1 = c->K[1] / TB; S.nt2 = c->K[2] / TB; S.Pc2 = 2 * pc;
  S.x = c->x; S.grid = (double*)c->grid2; S.charge = c->d_charge;
  S.cent = c->cent; S.ctrl = c->ctrl; S.u = u;
  for (int d = 0; d < 3; ++d) { S.L[d] = c->p.box[d]; S.KoL[d] = c->K[d] / c->p.box[d]; }
  S.tile_start = c->tile_start; S.tile_atoms = c->tile_atoms;
  const int gbeads = P < 8 ? P : 8;
  const dim3 grid(c->ntiles, P / gbeads);
#define SPREAD_CALL(GBV)                                                                     \
  QHP_SWITCH_ORDER(c->p.pme_order,                                                           \
                   hipLaunchKernelGGL((k_spread_tiles<OO, GBV, true>), grid, NT, 0, c->stream, S))
  switch (gbeads) {
    case 1: SPREAD_CALL(1); break;
    case 2: SPREAD_CALL(2); break;
    case 4: SPREAD_CALL(4); break;
    default: SPREAD_CALL(8); break;
  }
#undef SPREAD_CALL
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = convolve(c, pc, c->grid2)) != hipSuccess) return e;
  SpmeArgs A;
  A.N = N; A.K0 = c->K[0]; A.K1 = c->K[1]; A.K2 = c->K[2]; A.Pc2 = 2 * pc;
  A.order = c->tile_atoms; A.x = c->x; A.g = nullptr; A.grid = (double*)c->grid;
  A.charge = c->d_charge;
  for (int d = 0; d < 3; ++d) A.L[d] = c->p.box[d];
  A.energy = nullptr; A.dq = mix ? c->pg_dq : nullptr;
  const unsigned nb = (unsigned)(((size_t)N * P + NT - 1) / NT);
  A.nblocks = (int)nb;
  const unsigned nb8 = (nb + 7) / 8 * 8;
  QHP_SWITCH_P(P, QHP_SWITCH_ORDER(c->p.pme_order,
               hipLaunchKernelGGL((k_gather_hvp<PP, OO>), nb8, NT, 0, c->stream, A,
                                  (const double*)c->grid2, u, hu)));
  return hipGetLastError();
}
