// Centroid neighbour list (Sec. "Massively Parallel Implementation": neighbour lists are
// computed on ring-polymer centroids; if two centroids are neighbours, all their beads
// are). One list serves every bead of every step until the skin is used up.
//
// Build: cells of edge >= r_list / 2 on the centroids (wrapped fractional coordinate x n_c,
// floored, clamped to n_c - 1); one block per
// cell stages the atoms of its (up to) 5 x 5 x 5 distinct neighbouring cells in LDS and
// every wavefront scans them for one atom i of the cell. A pair (i, j) of different
// molecules is kept when the minimum-image centroid distance squared is < r_list^2,
// evaluated as d - L rint(d * (1/L)) per axis and (dx*dx + dy*dy) + dz*dz without
// contraction, so the set of pairs is reproducible bit for bit (the order of a row is not).
//
// Row i of the list (nbr[i * cap + k]) holds j | (sx+1) << 26 | (sy+1) << 28 | (sz+1) << 30,
// with s the image shift between the two centroids in the frame wrapped at build time
// (each centroid minus L floor(c / L)); the pair kernel reuses it on the wrapped
// centroids, which stay continuous until the next build.
//
// Rebuild rule, checked on the device every step: rebuild unless
// 2 (max centroid displacement since the build + max bead-centroid distance) <= skin.
#include "qhp_internal.h"

namespace {

constexpr int MAXM = 2560;        // neighbourhood atoms staged per chunk
constexpr int MAXC = 512;         // atoms of one cell handled by one block

struct NlArgs {
  int N, cap, ncell, nc0, nc1, nc2, nst;
  int nadv;                   // steps a propagation advances (inner steps of one outer step)
  double L0, L1, L2, iL0, iL1, iL2, rl2, skin;
  const double4* cent; double4* cref; double4* coff; double4* cwrap;
  int* cell_of; int* cell_count; int* cell_fill; int* cell_start; int* cell_atoms;
  const int* stencil; int* nbr; int* nnbr;
  NlCtrl* ctrl;
  const double4* bmax;
  int n_bmax;
  const double* charge; const int* type; int pack_qt;   // packed records: see qhp_internal.h
};

__global__ __launch_bounds__(256) void k_nl_check(NlArgs A, int force) {
  __shared__ double sm[4][256];
  __shared__ int go;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < A.n_bmax; k += blockDim.x) {
    const double4 v = A.bmax[k];
    a[0] = fmax(a[0], v.x); a[1] = fmax(a[1], v.y); a[2] = fmax(a[2], v.z); a[3] = fmax(a[3], v.w);
  }
  for (int q = 0; q < 4; ++q) sm[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int q = 0; q < 4; ++q) sm[q][threadIdx.x] = fmax(sm[q][threadIdx.x], sm[q][threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    NlCtrl* c = A.ctrl;
    const double dc = sqrt(sm[0][0]), db = sqrt(sm[1][0]);
    const int b = force || c->force_build || !(2.0 * (dc + db) <= A.skin);
    c->do_build = b;
    c->force_build = 0;
    if (!force) c->step += A.nadv;  // a propagation step's forces: the step is done
    c->spread_m = (int)sm[2][0];
    c->max_db = db;
    if (sm[3][0] != 0.0) c->spread_margin = 1;
    if (b) { c->n_builds += 1; c->max_count = 0; }
    go = b;
  }
  __syncthreads();
  if (go)
    for (int k = threadIdx.x; k < A.ncell; k += blockDim.x) { A.cell_count[k] = 0; A.cell_fill[k] = 0; }
}

#pragma clang fp contract(off)
using qhp::cell_coord;

QHP_DEV double wrapped(double x, double L, double iL) { return x - L * floor(x * iL); }

__global__ void k_nl_assign(NlArgs A) {
  if (!A.ctrl->do_build) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A.N) return;
  const double4 c = A.cent[a];
  const int id = (cell_coord(c.x, A.iL0, A.nc0) * A.nc1 + cell_coord(c.y, A.iL1, A.nc1)) * A.nc2 +
                 cell_coord(c.z, A.iL2, A.nc2);
  A.cell_of[a] = id;
  A.cref[a] = c;
  const double4 w = make_double4(wrapped(c.x, A.L0, A.iL0), wrapped(c.y, A.L1, A.iL1),
                                 wrapped(c.z, A.L2, A.iL2), c.w);
  A.cwrap[a] = A.pack_qt ? make_double4(w.x, w.y, w.z, qhp::pack_record(A.charge[a], A.type[a], c.w)) : w;
  A.coff[a] = make_double4(c.x - w.x, c.y - w.y, c.z - w.z, 0.0);
  atomicAdd(&A.cell_count[id], 1);
}

// exclusive scan of the cell counts (one block)
__global__ __launch_bounds__(256) void k_nl_scan(NlArgs A) {
  if (!A.ctrl->do_build) return;
  __shared__ int part[256];
  const int t = threadIdx.x;
  const int per = (A.ncell + 255) / 256;
  const int b0 = min(A.ncell, t * per), b1 = min(A.ncell, b0 + per);
  int s = 0;
  for (int k = b0; k < b1; ++k) s += A.cell_count[k];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int k = 0; k < 256; ++k) { const int v = part[k]; part[k] = acc; acc += v; }
    A.cell_start[A.ncell] = acc;
  }
  __syncthreads();
  int acc = part[t];
  for (int k = b0; k < b1; ++k) { A.cell_start[k] = acc; acc += A.cell_count[k]; }
}

__global__ void k_nl_scatter(NlArgs A) {
  if (!A.ctrl->do_build) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A.N) return;
  const int id = A.cell_of[a];
  const int slot = atomicAdd(&A.cell_fill[id], 1);
  A.cell_atoms[A.cell_start[id] + slot] = a;
}

// Batched path, two kernels per step. k_prep_count: every block reduces a share of the
// per-block maxima written by the normal-mode (or centroid) kernel and counts its atoms
// into their SPME tiles and centroid cells (the kernels that write the centroids also write
// each centroid's tile and cell); the last block to finish decides the rebuild, turns the
// counts into offsets and clears them for the next step. k_prep_scatter then places every
// atom in its tile and, on a rebuild, in its cell. The order within a tile or a cell is
// not significant (the exported list is canonical; spreading sums in LDS).
struct PrepArgs {
  NlArgs nl;
  int ntiles;
  int* tile_of; int* tile_count; int* tile_fill; int* tile_start; int* tile_atoms;
};
constexpr int PREP_NT = 512;              // threads of a prep block
constexpr int PREP_ATOMS = 1024;          // atoms of a prep block

// Exclusive prefix sum over the block of one value per thread (wavefront shuffles, then
// the wavefront totals); *total receives the sum of all values.
QHP_DEV int block_exclusive_scan(int v, int* swave, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) swave[w] = x;
  __syncthreads();
  if (w == 0) {
    int t = lane < nw ? swave[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(t, o);
      if (lane >= o) t += y;
    }
    if (lane < nw) swave[lane] = t;       // inclusive over wavefronts
  }
  __syncthreads();
  const int before = w > 0 ? swave[w - 1] : 0;
  *total = swave[nw - 1];
  __syncthreads();                        // swave is reused by the next scan
  return before + x - v;
}

// Bin counting and scattering by a whole wavefront whose lanes hold consecutive atoms
// (bin t, or -1 for no atom): neighbouring atoms mostly share a bin, so each run of equal
// bins takes one atomic, issued by its first lane, instead of one per lane to the same
// address. Every lane of the wavefront must take part.
struct WaveRuns {
  unsigned long long starts;   // lanes where a run begins
  int lane, head, len;         // this lane's run: first lane and length (at the first lane)
};
QHP_DEV WaveRuns wave_runs(int t) {
  WaveRuns w;
  w.lane = threadIdx.x & 63;
  const int prev = __shfl_up(t, 1);
  w.starts = __ballot(w.lane == 0 || prev != t);
  const unsigned long long upto = w.lane == 63 ? ~0ull : ((2ull << w.lane) - 1ull);
  w.head = 63 - __clzll(w.starts & upto);
  const unsigned long long after = w.lane == 63 ? 0ull : (w.starts >> (w.lane + 1));
  w.len = (after ? w.lane + 1 + __ffsll((long long)after) - 1 : 64) - w.lane;
  return w;
}
QHP_DEV void wave_count(int* cnt, int t) {
  const WaveRuns w = wave_runs(t);
  if (t >= 0 && w.head == w.lane) atomicAdd(&cnt[t], w.len);
}
QHP_DEV void wave_scatter(int* fill, int* out, int t, int atom) {
  const WaveRuns w = wave_runs(t);
  int b = 0;
  if (t >= 0 && w.head == w.lane) b = atomicAdd(&fill[t], w.len);
  b = __shfl(b, w.head);
  if (t >= 0) out[b + (w.lane - w.head)] = atom;
}

QHP_DEV double wave_fmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// non-negative doubles order like their bit patterns read as unsigned integers
QHP_DEV unsigned long long max_bits(double v) { return (unsigned long long)__double_as_longlong(v); }

__global__ __launch_bounds__(PREP_NT) void k_prep_count(PrepArgs B, int force) {
  NlArgs& A = B.nl;
  __shared__ double sm[4][PREP_NT / 64];
  __shared__ int swave[PREP_NT / 64];
  __shared__ int last, go;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nblk = gridDim.x;
  // ---- 1. this block's share of the per-block maxima ----
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = blockIdx.x * PREP_NT + tid; k < A.n_bmax; k += nblk * PREP_NT) {
    const double4 v = A.bmax[k];
    a[0] = fmax(a[0], v.x); a[1] = fmax(a[1], v.y); a[2] = fmax(a[2], v.z); a[3] = fmax(a[3], v.w);
  }
  for (int q = 0; q < 4; ++q) a[q] = wave_fmax(a[q]);
  if (lane == 0)
    for (int q = 0; q < 4; ++q) sm[q][wv] = a[q];
  // ---- 2. tile and cell counts of the block's atoms (consecutive atoms in consecutive
  //         lanes: one atomic per run of equal bins) ----
  for (int r = 0; r < PREP_ATOMS / PREP_NT; ++r) {
    const int i = blockIdx.x * PREP_ATOMS + r * PREP_NT + tid;
    wave_count(B.tile_count, i < A.N ? B.tile_of[i] : -1);
    wave_count(A.cell_count, i < A.N ? A.cell_of[i] : -1);
  }
  // every wavefront's atomics are complete at the barrier; one device-scope release fence
  // of the block then orders them before its arrival is counted (a fence in every thread
  // costs a device-wide write-back per wavefront on a chip of eight L2 caches)
  __syncthreads();
  if (tid == 0) {
    for (int q = 0; q < 4; ++q) {
      double m = sm[q][0];
      for (int w = 1; w < PREP_NT / 64; ++w) m = fmax(m, sm[q][w]);
      atomicMax(&A.ctrl->prep_max[q], max_bits(m));
    }
    __threadfence();
    last = atomicAdd(&A.ctrl->prep_done, 1) == nblk - 1;
    if (last) __threadfence();                      // acquire: the other blocks' counts
  }
  __syncthreads();
  if (!last) return;
  // ---- 3. the last block: rebuild decision and step bookkeeping ----
  __shared__ double smax[4];
  if (tid < 4) smax[tid] = __longlong_as_double((long long)atomicExch(&A.ctrl->prep_max[tid], 0ull));
  __syncthreads();
  if (tid == 0) {
    NlCtrl* c = A.ctrl;
    const double m[4] = {smax[0], smax[1], smax[2], smax[3]};
    const double dc = sqrt(m[0]), db = sqrt(m[1]);
    const int b = force || c->force_build || !(2.0 * (dc + db) <= A.skin);
    c->do_build = b;
    c->force_build = 0;
    if (!force) c->step += A.nadv;  // a propagation step's forces: the step is done
    c->spread_m = (int)m[2];
    c->max_db = db;
    if (m[3] != 0.0) c->spread_margin = 1;
    if (b) { c->n_builds += 1; c->max_count = 0; }
    c->prep_done = 0;
    go = b;
  }
  __syncthreads();
  // ---- 4. offsets (start and the scatter's fill pointer) from the counts, which are
  //         cleared for the next step; cell offsets only on a rebuild ----
  // (the fence above made the other blocks' counts visible to plain loads: they were
  // added at device scope, and the acquire invalidated this compute unit's caches)
  auto scan = [&](int* cnt, int* start_g, int* fill, int n, bool write) {
    if (!write) {                                   // counts only to be cleared
      for (int k = tid; k < n; k += PREP_NT) cnt[k] = 0;
      return;
    }
    const int pc = (n + PREP_NT - 1) / PREP_NT;
    const int b0 = min(n, tid * pc), b1 = min(n, b0 + pc);
    int s = 0;
    for (int k0 = b0; k0 < b1; k0 += 8) {           // eight loads in flight at a time
      int v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = k0 + u < b1 ? cnt[k0 + u] : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    int total;
    int acc = block_exclusive_scan(s, swave, &total);
    for (int k0 = b0; k0 < b1; k0 += 8) {
      int v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = k0 + u < b1 ? cnt[k0 + u] : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (k0 + u >= b1) break;
        if (write) { start_g[k0 + u] = acc; fill[k0 + u] = acc; }
        acc += v[u];
        cnt[k0 + u] = 0;
      }
    }
    if (write && tid == 0) start_g[n] = total;
  };
  scan(B.tile_count, B.tile_start, B.tile_fill, B.ntiles, true);
  scan(A.cell_count, A.cell_start, A.cell_fill, A.ncell, go);
}

__global__ __launch_bounds__(PREP_NT) void k_prep_scatter(PrepArgs B) {
  NlArgs& A = B.nl;
  const bool go = A.ctrl->do_build;
  for (int r = 0; r < PREP_ATOMS / PREP_NT; ++r) {
    const int i = blockIdx.x * PREP_ATOMS + r * PREP_NT + threadIdx.x;
    wave_scatter(B.tile_fill, B.tile_atoms, i < A.N ? B.tile_of[i] : -1, i);
    if (go) wave_scatter(A.cell_fill, A.cell_atoms, i < A.N ? A.cell_of[i] : -1, i);
  }
}

// One block per cell, NL_THREADS / 64 wavefronts sharing the cell's atoms. Also records
// the build frame of the cell's atoms: reference centroid, centroid wrapped into the box
// (w: bead spread) and the offset between the two.
constexpr int NL_THREADS = 1024;
QHP_DEV void nl_build_cell(const NlArgs& A, const int cell) {
  __shared__ double sx[MAXM], sy[MAXM], sz[MAXM];
  __shared__ int sj[MAXM];
  __shared__ int sofs[126];
  __shared__ int scnt[MAXC];
  __shared__ int sbeg[126];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int* st = A.stencil + (size_t)cell * A.nst;
  // sizes and first entries of the neighbouring cells, loaded in parallel, then a prefix sum
  if (tid < A.nst) {
    const int c = st[tid];
    sbeg[tid] = c >= 0 ? A.cell_start[c] : 0;
    sofs[tid + 1] = c >= 0 ? A.cell_start[c + 1] - A.cell_start[c] : 0;
  }
  __syncthreads();
  if (tid < 64) {              // inclusive prefix sum of sofs[1..nst], two entries per lane
    const int k0 = 1 + 2 * tid, k1 = k0 + 1;
    const int a0 = k0 <= A.nst ? sofs[k0] : 0, a1 = k1 <= A.nst ? sofs[k1] : 0;
    int t = a0 + a1;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(t, o);
      if (lane >= o) t += u;
    }
    const int ex = t - a0 - a1;
    if (k0 <= A.nst) sofs[k0] = ex + a0;
    if (k1 <= A.nst) sofs[k1] = ex + a0 + a1;
    if (tid == 0) sofs[0] = 0;
  }
  const int c0 = A.cell_start[cell], nin = A.cell_start[cell + 1] - c0;
  if (nin > MAXC) {                       // cannot happen at liquid densities
    if (tid == 0) A.ctrl->overflow = 1;
    return;
  }
  for (int k = tid; k < nin; k += blockDim.x) scnt[k] = 0;
  __syncthreads();
  const int M = sofs[A.nst];
  for (int base = 0; base < M; base += MAXM) {
    const int len = min(MAXM, M - base);
    for (int p = tid; p < len; p += blockDim.x) {
      // neighbouring cell k holding concatenated position base + p (binary search)
      const int gp = base + p;
      int lo = 0, hi = A.nst;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sofs[mid] <= gp) lo = mid; else hi = mid;
      }
      const int j = A.cell_atoms[sbeg[lo] + (gp - sofs[lo])];
      const double4 cj = A.cent[j];
      sx[p] = cj.x; sy[p] = cj.y; sz[p] = cj.z; sj[p] = j;
    }
    __syncthreads();
    for (int ii = wv; ii < nin; ii += NL_THREADS / 64) {
      const int i = A.cell_atoms[c0 + ii];
      const double4 ci = A.cent[i];
      const double wx = wrapped(ci.x, A.L0, A.iL0), wy = wrapped(ci.y, A.L1, A.iL1),
                   wz = wrapped(ci.z, A.L2, A.iL2);
      const int mi = i / 3;
      int cnt = scnt[ii];
      for (int p0 = 0; p0 < len; p0 += 64) {
        const int p = p0 + lane;
        bool keep = false;
        unsigned code = 0;
        if (p < len) {
          const int j = sj[p];
          double dx = sx[p] - ci.x, dy = sy[p] - ci.y, dz = sz[p] - ci.z;
          dx = dx - A.L0 * rint(dx * A.iL0);
          dy = dy - A.L1 * rint(dy * A.iL1);
          dz = dz - A.L2 * rint(dz * A.iL2);
          double d2 = dx * dx + dy * dy;
          d2 = d2 + dz * dz;
          keep = (j / 3 != mi) && (d2 < A.rl2);
          if (keep) {
            // image shift of the two centroids in the frame wrapped at this list build
            const int sxi = -(int)rint((wrapped(sx[p], A.L0, A.iL0) - wx) * A.iL0);
            const int syi = -(int)rint((wrapped(sy[p], A.L1, A.iL1) - wy) * A.iL1);
            const int szi = -(int)rint((wrapped(sz[p], A.L2, A.iL2) - wz) * A.iL2);
            code = (unsigned)j | ((unsigned)(sxi + 1) << 26) | ((unsigned)(syi + 1) << 28) |
                   ((unsigned)(szi + 1) << 30);
          }
        }
        const unsigned long long m = __ballot(keep);
        if (keep) {
          const int slot = cnt + __popcll(m & ((1ull << lane) - 1ull));
          if (slot < A.cap) A.nbr[(size_t)i * A.cap + slot] = (int)code;
        }
        cnt += __popcll(m);
      }
      if (lane == 0) scnt[ii] = cnt;
    }
    __syncthreads();
  }
  int most = 0;                 // the block's largest count: one global atomic per block
  for (int ii = tid; ii < nin; ii += blockDim.x) {
    const int i = A.cell_atoms[c0 + ii];
    const int cnt = scnt[ii];
    A.nnbr[i] = cnt < A.cap ? cnt : A.cap;
    if (cnt > A.cap) A.ctrl->overflow = 1;
    most = max(most, cnt);
    const double4 c = A.cent[i];
    A.cref[i] = c;
    const double4 w = make_double4(wrapped(c.x, A.L0, A.iL0), wrapped(c.y, A.L1, A.iL1),
                                   wrapped(c.z, A.L2, A.iL2), c.w);
    A.cwrap[i] = A.pack_qt ? make_double4(w.x, w.y, w.z, qhp::pack_record(A.charge[i], A.type[i], c.w)) : w;
    A.coff[i] = make_double4(c.x - w.x, c.y - w.y, c.z - w.z, 0.0);
  }
  for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
  if (lane == 0 && most > 0) atomicMax(&A.ctrl->max_count, most);
}

// A fixed grid of blocks takes the cells in turn, so a step without a rebuild costs the
// start and exit of a few hundred blocks rather than of one block per cell.
constexpr int NL_BLOCKS = 512;   // two blocks of 74 KB of LDS per compute unit
__global__ __launch_bounds__(NL_THREADS) void k_nl_build(NlArgs A) {
  if (!A.ctrl->do_build) return;
  for (int cell = blockIdx.x; cell < A.ncell; cell += gridDim.x) {
    nl_build_cell(A, cell);
    __syncthreads();                 // the block's LDS is reused by the next cell
  }
}
#pragma clang fp contract(fast)

}  // namespace

static NlArgs nl_args(qhp_ctx* c) {
  NlArgs A;
  A.N = c->N; A.cap = c->cap; A.ncell = c->ncell; A.nst = c->nst;
  A.nc0 = c->nc[0]; A.nc1 = c->nc[1]; A.nc2 = c->nc[2];
  A.L0 = c->p.box[0]; A.L1 = c->p.box[1]; A.L2 = c->p.box[2];
  A.iL0 = 1.0 / A.L0; A.iL1 = 1.0 / A.L1; A.iL2 = 1.0 / A.L2;
  A.rl2 = c->rlist * c->rlist; A.skin = c->p.skin;
  A.cent = c->cent; A.cref = c->cref; A.coff = c->coff; A.cwrap = c->cwrap;
  A.cell_of = c->cell_of; A.cell_count = c->cell_count; A.cell_fill = c->cell_fill;
  A.cell_start = c->cell_start; A.cell_atoms = c->cell_atoms; A.stencil = c->stencil;
  A.nbr = c->nbr; A.nnbr = c->nnbr; A.ctrl = c->ctrl; A.bmax = c->bmax; A.n_bmax = c->n_bmax;
  A.nadv = c->nalt;
  A.charge = c->d_charge; A.type = c->d_type; A.pack_qt = c->pack_qt ? 1 : 0;
  return A;
}

qhp::BinGeom bin_geom(const qhp_ctx* c) {
  qhp::BinGeom G;
  G.tile_of = c->tile_of; G.cell_of = c->cell_of;
  for (int d = 0; d < 3; ++d) {
    G.K[d] = c->K[d]; G.KoL[d] = c->K[d] / c->p.box[d];
    G.nc[d] = c->nc[d]; G.iL[d] = 1.0 / c->p.box[d];
  }
  G.nt1 = c->K[1] / QHP_TB; G.nt2 = c->K[2] / QHP_TB;
  return G;
}

// Batched path: the prep kernels (decision, SPME tiles, cells of a rebuild), then the
// build. Plain path: the decision and cells by separate kernels (tiles are binned per bead).
hipError_t launch_nlist(qhp_ctx* c, bool from_step) {
  NlArgs A = nl_args(c);
  if (c->p.exec != QHP_PLAIN) {
    PrepArgs B;
    B.nl = A;
    B.ntiles = c->ntiles;
    B.tile_of = c->tile_of; B.tile_count = c->tile_count; B.tile_fill = c->tile_fill;
    B.tile_start = c->tile_start; B.tile_atoms = c->tile_atoms;
    const unsigned nb = (unsigned)((c->N + PREP_ATOMS - 1) / PREP_ATOMS);
    hipLaunchKernelGGL(k_prep_count, nb, PREP_NT, 0, c->stream, B, from_step ? 0 : 1);
    hipLaunchKernelGGL(k_prep_scatter, nb, PREP_NT, 0, c->stream, B);
    hipLaunchKernelGGL(k_nl_build, std::min(c->ncell, NL_BLOCKS), NL_THREADS, 0, c->stream, A);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_nl_check, 1, 256, 0, c->stream, A, from_step ? 0 : 1);
  hipLaunchKernelGGL(k_nl_assign, (c->N + 255) / 256, 256, 0, c->stream, A);
  hipLaunchKernelGGL(k_nl_scan, 1, 256, 0, c->stream, A);
  hipLaunchKernelGGL(k_nl_scatter, (c->N + 255) / 256, 256, 0, c->stream, A);
  hipLaunchKernelGGL(k_nl_build, std::min(c->ncell, NL_BLOCKS), NL_THREADS, 0, c->stream, A);
  return hipGetLastError();
}
