// Centroid neighbour list (Sec. "Massively Parallel Implementation": neighbour lists are
// computed on ring-polymer centroids; if two centroids are neighbours, all their beads
// are). One list serves every bead of every step until the skin is used up.
//
// Build: cells of edge >= r_list on the centroids (wrapped fractional coordinate x n_c,
// floored, clamped to n_c - 1), a deterministic fill of each cell in atom order, then for
// every atom a scan of the distinct neighbouring cells. A pair (i, j) of different
// molecules is kept when the minimum-image centroid distance squared is < r_list^2,
// evaluated as dx - L rint(dx / L) per axis and dx*dx + dy*dy, then + dz*dz, without
// contraction, so the list is reproducible bit for bit.
//
// Entry k of atom i is nbr[k * N + i] = j | (sx+1) << 26 | (sy+1) << 28 | (sz+1) << 30
// with s the image shift between the two centroids in the frame wrapped at build time
// (each centroid minus L floor(c / L)); the pair kernel reuses it on the wrapped
// centroids, which stay continuous until the next build.
//
// Rebuild rule, checked on the device every step: rebuild when
// 2 (max centroid displacement since the build + max bead-centroid distance) > skin.
#include "qhp_internal.h"

namespace {

struct NlArgs {
  int N, cap, ncell, nc0, nc1, nc2;
  double L0, L1, L2, rl2, skin;
  const double4* cent; double4* cref; double4* coff; double4* cwrap;
  int* cell_of; int* cell_count; int* cell_start; int* cell_atoms;
  const int* stencil; int* nbr; int* nnbr;
  NlCtrl* ctrl;
  const double2* bmax;
  int n_bmax;
};

__global__ __launch_bounds__(256) void k_nl_check(NlArgs A, int force) {
  __shared__ double s0[256], s1[256];
  __shared__ int go;
  double a0 = 0.0, a1 = 0.0;
  if (!force)
    for (int k = threadIdx.x; k < A.n_bmax; k += blockDim.x) {
      const double2 v = A.bmax[k];
      a0 = fmax(a0, v.x);
      a1 = fmax(a1, v.y);
    }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + st]);
      s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    NlCtrl* c = A.ctrl;
    const double dc = sqrt(s0[0]), db = sqrt(s1[0]);
    const int b = force || c->force_build || !(2.0 * (dc + db) <= A.skin);
    c->do_build = b;
    c->force_build = 0;
    if (b) { c->n_builds += 1; c->max_count = 0; }
    go = b;
  }
  __syncthreads();
  if (go)
    for (int k = threadIdx.x; k < A.ncell; k += blockDim.x) A.cell_count[k] = 0;
}

#pragma clang fp contract(off)
QHP_DEV int cell_coord(double x, double L, int n) {
  double f = x / L;
  f = f - floor(f);
  if (!isfinite(f)) return 0;
  int i = (int)(f * (double)n);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__global__ void k_nl_assign(NlArgs A) {
  if (!A.ctrl->do_build) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A.N) return;
  const double4 c = A.cent[a];
  const int id = (cell_coord(c.x, A.L0, A.nc0) * A.nc1 + cell_coord(c.y, A.L1, A.nc1)) * A.nc2 +
                 cell_coord(c.z, A.L2, A.nc2);
  A.cell_of[a] = id;
  A.cref[a] = c;
  const double4 o = make_double4(A.L0 * floor(c.x / A.L0), A.L1 * floor(c.y / A.L1),
                                 A.L2 * floor(c.z / A.L2), 0.0);
  A.coff[a] = o;
  A.cwrap[a] = make_double4(c.x - o.x, c.y - o.y, c.z - o.z, 0.0);
  atomicAdd(&A.cell_count[id], 1);
}

__global__ void k_nl_scan(NlArgs A) {
  if (!A.ctrl->do_build) return;
  if (threadIdx.x == 0) {
    int s = 0;
    for (int k = 0; k < A.ncell; ++k) { A.cell_start[k] = s; s += A.cell_count[k]; }
    A.cell_start[A.ncell] = s;
  }
}

// one block per cell: gather that cell's atoms in increasing atom order
__global__ __launch_bounds__(256) void k_nl_fill(NlArgs A) {
  if (!A.ctrl->do_build) return;
  __shared__ int wsum[4];
  __shared__ int base;
  const int cell = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) base = A.cell_start[cell];
  __syncthreads();
  for (int a0 = 0; a0 < A.N; a0 += 256) {
    const int a = a0 + tid;
    const bool in = a < A.N && A.cell_of[a] == cell;
    const unsigned long long m = __ballot(in);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int k = 0; k < w; ++k) off += wsum[k];
    if (in) A.cell_atoms[off + before] = a;
    __syncthreads();
    if (tid == 0) base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
}

__global__ __launch_bounds__(128) void k_nl_build(NlArgs A) {
  if (!A.ctrl->do_build) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.N) return;
  const double4 ci = A.cent[i];
  const double4 wi = make_double4(ci.x - A.L0 * floor(ci.x / A.L0), ci.y - A.L1 * floor(ci.y / A.L1),
                                  ci.z - A.L2 * floor(ci.z / A.L2), 0.0);
  const int mi = i / 3;
  const int* st = A.stencil + A.cell_of[i] * 27;
  int cnt = 0;
  for (int s = 0; s < 27; ++s) {
    const int cell = st[s];
    if (cell < 0) break;
    const int e = A.cell_start[cell + 1];
    for (int k = A.cell_start[cell]; k < e; ++k) {
      const int j = A.cell_atoms[k];
      if (j / 3 == mi) continue;
      const double4 cj = A.cent[j];
      double dx = cj.x - ci.x, dy = cj.y - ci.y, dz = cj.z - ci.z;
      dx = dx - A.L0 * rint(dx / A.L0);
      dy = dy - A.L1 * rint(dy / A.L1);
      dz = dz - A.L2 * rint(dz / A.L2);
      double d2 = dx * dx + dy * dy;
      d2 = d2 + dz * dz;
      if (d2 < A.rl2) {
        if (cnt < A.cap) {
          // image shift in the frame wrapped at this build: both wrapped centroids lie in
          // [0, L), so the shift is -1, 0 or +1 per axis
          const double wx = cj.x - A.L0 * floor(cj.x / A.L0) - wi.x;
          const double wy = cj.y - A.L1 * floor(cj.y / A.L1) - wi.y;
          const double wz = cj.z - A.L2 * floor(cj.z / A.L2) - wi.z;
          const int sx = -(int)rint(wx / A.L0), sy = -(int)rint(wy / A.L1), sz = -(int)rint(wz / A.L2);
          const unsigned code = (unsigned)j | ((unsigned)(sx + 1) << 26) |
                                ((unsigned)(sy + 1) << 28) | ((unsigned)(sz + 1) << 30);
          A.nbr[(size_t)cnt * A.N + i] = (int)code;
        }
        ++cnt;
      }
    }
  }
  A.nnbr[i] = cnt < A.cap ? cnt : A.cap;
  if (cnt > A.cap) A.ctrl->overflow = 1;
  atomicMax(&A.ctrl->max_count, cnt);
}
#pragma clang fp contract(fast)

}  // namespace

hipError_t launch_nlist(qhp_ctx* c, bool from_step) {
  NlArgs A;
  A.N = c->N; A.cap = c->cap; A.ncell = c->ncell;
  A.nc0 = c->nc[0]; A.nc1 = c->nc[1]; A.nc2 = c->nc[2];
  A.L0 = c->p.box[0]; A.L1 = c->p.box[1]; A.L2 = c->p.box[2];
  A.rl2 = c->rlist * c->rlist; A.skin = c->p.skin;
  A.cent = c->cent; A.cref = c->cref; A.coff = c->coff; A.cwrap = c->cwrap; A.cell_of = c->cell_of; A.cell_count = c->cell_count;
  A.cell_start = c->cell_start; A.cell_atoms = c->cell_atoms; A.stencil = c->stencil;
  A.nbr = c->nbr; A.nnbr = c->nnbr; A.ctrl = c->ctrl; A.bmax = c->bmax; A.n_bmax = c->n_bmax;
  hipLaunchKernelGGL(k_nl_check, 1, 256, 0, c->stream, A, from_step ? 0 : 1);
  hipLaunchKernelGGL(k_nl_assign, (c->N + 255) / 256, 256, 0, c->stream, A);
  hipLaunchKernelGGL(k_nl_scan, 1, 64, 0, c->stream, A);
  hipLaunchKernelGGL(k_nl_fill, c->ncell, 256, 0, c->stream, A);
  hipLaunchKernelGGL(k_nl_build, (c->N + 127) / 128, 128, 0, c->stream, A);
  return hipGetLastError();
}
