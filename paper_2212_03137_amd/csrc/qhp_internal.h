// Internal declarations of the MI355X ring-polymer MD library: device state, launch
// helpers and the device-side counter-based Gaussian generator.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qhp.h"

#define QHP_MAX_TYPES 8
#define QHP_MAX_DEVICES 64
#define QHP_SCRATCH_DOUBLES 131072   // 1 MiB file-scope scratch of the allocation-free call
#define QHP_PAIR_TAB 1024           // intervals of the FP32 pair kernel's tables

// ---------------------------------------------------------------------------------------
// Device layout (all FP64 unless noted; "bead innermost"):
//   Q, Pa, x, g        [3][N][P]   mode amplitudes, momenta, bead positions, grad V
//   cent, cref         [N] double4 centroid now / at the last neighbour-list build
//   cwrap              [N] double4 centroid in the frame wrapped at the last build
//   nbr                [N][cap]    int32 neighbour k of atom i at nbr[i*cap + k] (full list)
//   grid               [K0][K1][K2][Pc] double2, bead b in component b%2 of complex b/2
// In plain mode x and g are bead-major [P][3][N] and each bead is evaluated alone.
// ---------------------------------------------------------------------------------------

struct NlCtrl {               // device-side control block (neighbour list, step counter)
  long long step;             // MD step of the next normal-mode kernel
  int do_build;               // this step rebuilds
  int force_build;            // host request
  int overflow;               // a neighbour count exceeded the capacity
  int nonfinite;              // a non-finite coordinate or momentum was seen
  int max_count;              // largest neighbour count of the last build
  int n_builds;               // builds so far
  int spread_margin;          // a bead left the SPME tile margin of its centroid
  int spread_m;               // largest bead-centroid grid-base offset this step
  double max_db;              // largest bead-centroid distance this step
  unsigned long long prep_max[4];  // per-step maxima being reduced (zero between steps)
  int prep_done;              // prep blocks finished this step (zero between steps)
};

// The beads a force launch works on: the full ring polymer, or its contraction (V_s under
// ring-polymer contraction), or a scratch gradient target (stateless evaluation).
struct BeadSet {
  int P;                      // bead lanes (a power of two; phantom beads beyond the real ones)
  int Pc;                     // complex SPME grid slots, max(1, P / 2)
  const double* x;            // [3][N][P]
  double* g;                  // [3][N][P] grad V (initialised by launch_bonded)
  const float4* xf;           // [N][P] FP32 bead - centroid offsets and charge
  double* energy;             // [P][QHP_NTERMS]
  int terms;                  // QHP_TERMS_* for launch_bonded
  int pgrad = 0;              // also accumulate the parameter gradients (FP64 kernels)
  const double* hvp_u = nullptr;  // Hessian-vector product along u [3][N][P]: g receives H u
};
#define QHP_TERMS_BONDED 1    // O-H bonds and H-O-H angles (V_f)
#define QHP_TERMS_EXCL   2    // intramolecular Ewald exclusion correction (part of V_s)
#define QHP_TERMS_ALL    3

struct QtbState {
  int nseg;
  double* gamma = nullptr;    // [n_types][nseg+1]
  double2* hhat = nullptr;    // [n_types][4 nseg]  DFT of the embedded kernel h
  double2* hker = nullptr;    // [n_types][2 nseg]  scratch: H then h
  double* noise = nullptr;    // [nseg][3][N] coloured force of the current segment (per step)
  double* vrec = nullptr;     // [nseg][3][N] recorded O-midpoint velocities (per step)
  double* noise_t = nullptr;  // the same two records in the segment kernels' layout
  double* vrec_t = nullptr;   //   (qtb_rec: eight consecutive steps contiguous)
  double* dsum = nullptr;     // [n_types][nseg+1] summed Delta_FDT of the running segment
  double* dbar = nullptr;     // [n_types][nseg+1] type-averaged Delta_FDT of the last segment
  double* vvsum = nullptr;    // [n_types][nseg+1] RATIO: summed C_vv of the running segment
  double* vfsum = nullptr;    // [n_types][nseg+1] RATIO: summed Re C_vF
  double* avg_vv = nullptr;   // [n_types][nseg+1] RATIO: running means (null for SIMPLE)
  double* avg_vf = nullptr;
  double* d_tmass = nullptr;  // [n_types]
  double* d_inv_count = nullptr; // [n_types] 1 / (3 * atoms of the type)
  double2* tw2 = nullptr;     // twiddles of length 2 nseg
  double2* tw4 = nullptr;     // twiddles of length 4 nseg
  int type_count[QHP_MAX_TYPES];
  double type_mass[QHP_MAX_TYPES];
  double c1, osd;             // O step: p <- c1 p + osd F
  int ratio_of[QHP_MAX_TYPES] = {};   // adaptation of each type: 1 = RATIO, 0 = SIMPLE
  double tau_of[QHP_MAX_TYPES] = {};  // RATIO running-mean time of each type
  bool any_ratio = false;             // the RATIO accumulators exist
};

struct qhp_ctx {
  qhp_params p;
  int N, P, NW, Pc;           // atoms, bead lanes (a power of two), waters, complex grid batch
  int Pb;                     // beads of the ring polymer (<= P; the rest are phantoms)
  hipStream_t stream;
  bool own_stream = false;    // created here because the caller passed none
  // second stream of the bead-batched force evaluation (default priority): the SPME
  // spread and transforms run on it, concurrent with the bonded and real-space kernels
  // on `stream`, forked from and joined back to `stream` by the two events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraphExec_t step_exec = nullptr;   // one captured (outer) MD step (no energies)
  bool use_graph = true;
  bool serial_forces = false; // set while a group captures the member's step: no side branch
  bool spme_generic = false;  // an SPME grid edge is not a power of two: the plain SPME path
  std::string err;
  bool have_state = false;
  int64_t step = 0;

  // host copies of per-atom data (charge: as used, i.e. solute charges times lambda_elec)
  std::vector<int32_t> type;
  std::vector<double> mass, charge, sigma, eps;

  // alchemical coupling (type_soft given): solute types, couplings, unscaled charges
  bool alch = false;
  std::vector<int32_t> soft;
  std::vector<double> q_given;
  double lam_e = 1.0, lam_v = 1.0;
  double* d_charge_alt = nullptr;   // charges at other couplings (qhp_eval_lambda)
  std::vector<double> charge_alt;
  int64_t graph_epoch = 0;          // bumped whenever captured kernel arguments go stale
  int pair_wpb = 0;                 // FP32 pair kernel: atoms per block (0 = 4; 2, 4, 8)
  int spread_gb = 0;                // SPME spreading: beads per block (0 = min(P, 8))
  int spread_z = 0;                 // SPME spreading: 8^3 tiles per block along z (0 = 1)
  int fft_nb = 0;                   // y-z plane kernel: slots per block (0 = default,
                                    // < 0 = one-axis passes instead)

  // normal modes
  double* T = nullptr;        // [P][P] T[bead][mode]
  double* mode_c = nullptr;   // [P] cos(w h)
  double* mode_s_w = nullptr; // [P] sin(w h)/w   (h for the centroid)
  double* mode_ws = nullptr;  // [P] w sin(w h)
  double* mode_c1 = nullptr;  // [P] exp(-gamma_n dt)
  double* mode_c2 = nullptr;  // [P] sqrt(1 - c1^2)
  double* mode_w2 = nullptr;  // [P] w^2 (spring energy)
  std::vector<double> h_omega;

  // per-atom device arrays
  int* d_type = nullptr;
  double* d_mass = nullptr;
  double* d_charge = nullptr;
  double* d_sqrt_mkT = nullptr;
  double* d_sigma = nullptr;
  double* d_eps = nullptr;
  double tether_k = 0.0;      // test-only harmonic tether (0 = off)
  double* d_anchor = nullptr; // its anchors [3][N]

  // state
  double *Q = nullptr, *Pa = nullptr, *x = nullptr, *g = nullptr;
  double4* cent = nullptr;
  double4* cref = nullptr;
  double4* coff = nullptr;    // [N] L * floor(c / L) per axis at the last build
  double4* cwrap = nullptr;   // [N] centroid - coff (continuous between builds)
  float4* xf = nullptr;       // FP32-pair mode: per bead (x - c) and charge, [N][P]

  // neighbour list
  NlCtrl* ctrl = nullptr;
  double4* bmax = nullptr;    // per block: (max |dc|^2, max |db|^2, max base offset, bad)
  int n_bmax = 0;             // entries written by the last normal-mode launch
  int* cell_of = nullptr;     // [N]
  int* cell_count = nullptr;  // [ncell]
  int* cell_fill = nullptr;   // [ncell]
  int* cell_start = nullptr;  // [ncell + 1]
  int* cell_atoms = nullptr;  // [N]
  int* stencil = nullptr;     // [ncell][nst] distinct neighbour cells, -1 padded
  int* nbr = nullptr;         // [N][cap]
  int* nnbr = nullptr;        // [N]
  int cap = 0, nc[3] = {1, 1, 1}, ncell = 1, nst = 125;
  double rlist = 0;

  // SPME
  int K[3];
  double2* grid = nullptr;    // [K0][K1][K2][Pc] (plain: [K0][K1][K2])
  double2* grid2 = nullptr;   // tangent grid of Hessian-vector products (allocated on use)
  double2* grid_l1 = nullptr; // the transforms' slot-pair planes [K0][Pc/2][K1][K2][2]
  double* influence = nullptr;// [K0][K1][K2]
  int ntiles = 0;             // 8^3-point spreading tiles
  int* tile_of = nullptr;     // [N]
  int* tile_count = nullptr;  // [ntiles]
  int* tile_fill = nullptr;   // [ntiles]
  int* tile_start = nullptr;  // [ntiles + 1]
  int* tile_atoms = nullptr;  // [N]
  double2* tw[3] = {nullptr, nullptr, nullptr};

  // energies
  double* energy = nullptr;   // [P][QHP_NTERMS]
  double self_energy = 0;

  // scratch for boundary transposes
  double* io_a = nullptr;     // [P][N][3]
  double* io_b = nullptr;

  // multiple time stepping and ring-polymer contraction
  bool respa = false;         // rpc_beads < P or respa_nalt > 1
  bool pack_qt = false;       // centroid records carry charge, type and spread (no contraction)
  int Ps = 0, nalt = 1;       // contracted bead lanes (a power of two), inner steps per outer step
  int Psb = 0;                // contracted beads (<= Ps; the rest are phantoms)
  double* xs = nullptr;       // [3][N][Ps] contracted beads
  double* gs = nullptr;       // [3][N][Ps] grad V_s there
  float4* xfs = nullptr;      // [N][Ps]
  double* Cs = nullptr;       // [Ps][Ps] contraction matrix C[j][n]
  double* pa_tmp = nullptr;   // [3][N][P] scratch momenta
  double* g_eval = nullptr;   // [3][N][P] gradient target of qhp_eval

  float4* pair_tab = nullptr; // FP32 pairs: [2][QHP_PAIR_TAB] cubic pieces of the screened
                              // Coulomb force and energy kernels over r^2 in [0, rc^2]
  float pair_tab_scale = 0.f; // intervals per A^2 (maps rc^2 just below QHP_PAIR_TAB)
  int pair_tab_kmin = 0;      // first interval the tables serve (closer pairs: the formula)
  // parameter gradients of the summed bead energies
  double* pg_dq = nullptr;    // [N] d/d charge
  double* pg_lj = nullptr;    // [2][QHP_MAX_TYPES] d/d epsilon, d/d sigma per type
  double* hvp_out = nullptr;  // [3][N][P] Hessian-vector product (allocated on use)

  QtbState qtb;

  // state at the start of the current qhp_step call (repeated after a list-row overflow)
  double* snap = nullptr;
  NlCtrl* snap_ctrl = nullptr;
  int list_grown = 0;         // times the neighbour rows were enlarged
  void* scratch = nullptr;    // device address of the file-scope scratch on this context's GPU

  // profiling
  int prof_which = 0;
  double prof_ms = 0;
  int64_t prof_launches = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
};

// SPME spreading tiles: TB^3 grid points; a bead's grid base may differ from its centroid's
// by at most TB points above and TB - order + 1 below (checked every step).
constexpr int QHP_TB = 8;
// complex values one FFT block transforms (series of length K times FFT_E / K series)
constexpr int QHP_FFT_E = 2048;

// ---------------------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------------------
int qhp_fail(qhp_ctx* c, int code, const std::string& msg);
#define QHP_HIP(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return qhp_fail((ctx), QHP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// profiling brackets around the launches of one kernel class
void prof_begin(qhp_ctx* c, int which, hipEvent_t* ev);
void prof_end(qhp_ctx* c, int which, hipEvent_t ev);

// ---------------------------------------------------------------------------------------
// launchers implemented in the kernel files (all enqueue on c->stream, return hipError_t)
// ---------------------------------------------------------------------------------------
hipError_t launch_beads_to_modes(qhp_ctx* c, const double* xb, const double* vb);
// inner: index of the inner step in its outer step; slow_h: factor of the slow kick in this
// inner step (0 or n dt); emit: write the bead set of the slow forces (centroids, list
// and tile bookkeeping inputs); without RESPA (0, 0, true).
hipError_t launch_nm_step(qhp_ctx* c, int inner, double slow_h, bool emit);
// dst = src + s * f_s on the modes n < Ps (f_s from gs); the other modes are copied
hipError_t launch_kick_slow(qhp_ctx* c, double* dst, const double* src, double s);
// pa: the stored momenta to report from (c->Pa, or Pa plus the pending slow kick)
hipError_t launch_state_out(qhp_ctx* c, double* xb, double* vb, const double* pa);
hipError_t launch_kick_back(qhp_ctx* c);
hipError_t launch_mode_energies(qhp_ctx* c, double* out2, const double* pa);
// the allocation-free variant: partial sums in the file-scope scratch (c->scratch), the
// two totals written to device memory out2; mode_energy_parts gives the scratch doubles
hipError_t launch_mode_energies_noalloc(qhp_ctx* c, double* out2, const double* pa);
size_t mode_energy_parts(const qhp_ctx* c);
// device address of the file-scope scratch on the current device (looked up once per device)
hipError_t scratch_address(void** ptr);
// contracted beads, their FP32 offsets, centroids and block maxima from the modes Q
hipError_t launch_contract(qhp_ctx* c);
hipError_t launch_transpose_in(qhp_ctx* c, const double* src, double* dst);
hipError_t launch_transpose_out(qhp_ctx* c, const double* src, double* dst, double scale);
hipError_t launch_centroid_of_beads(qhp_ctx* c);

hipError_t launch_nlist(qhp_ctx* c, bool from_step);
hipError_t launch_zero(qhp_ctx* c, void* ptr, size_t bytes);
// zero the contracted-bead terms (all but bonds and angles) of energy rows [r0, r1)
hipError_t launch_clear_slow_energy(qhp_ctx* c, int r0, int r1);
// H u of the intramolecular terms (bonds, angle, exclusion) at c->x: writes (initialises)
// hu; with mix, adds the exclusion part of d(u . grad E)/dq to c->pg_dq
hipError_t launch_bonded_hvp(qhp_ctx* c, const double* u, double* hu, bool mix);
// H u of the reciprocal sum at c->x, added to hu; c->grid must hold the potential grid
// of c->x (left there by launch_spme); with mix, adds d(u . grad E_recip)/dq to c->pg_dq
hipError_t launch_spme_hvp(qhp_ctx* c, const double* u, double* hu, bool mix);
// bead >= 0: one bead of the plain (bead-major) layout; bead < 0: the bead set `bs`
// (nullptr: the full ring polymer of the context)
hipError_t launch_bonded(qhp_ctx* c, bool energy, int bead, const BeadSet* bs = nullptr);
// test-only tether (after launch_bonded, which initialises grad V and the energy rows):
// grad V += k (x - a), bond energy += k/2 |x - a|^2; nothing when tether_k = 0
hipError_t launch_tether(qhp_ctx* c, bool energy, int bead, const BeadSet* bs = nullptr);
hipError_t launch_pair(qhp_ctx* c, bool energy, int bead, const BeadSet* bs = nullptr);
// part: SPME_FRONT (tile binning of the plain layout, spread, transforms and influence
// function), SPME_GATHER (forces into grad V, energies), or both
enum { SPME_FRONT = 1, SPME_GATHER = 2, SPME_ALL = 3 };
hipError_t launch_spme(qhp_ctx* c, bool energy, int bead, const BeadSet* bs = nullptr,
                       int part = SPME_ALL);
BeadSet full_beads(qhp_ctx* c);
hipError_t launch_noise_export(qhp_ctx* c, int stream, int64_t step, double* out);

hipError_t launch_qtb_generate(qhp_ctx* c, int64_t seg);
hipError_t launch_qtb_adapt(qhp_ctx* c);
hipError_t qtb_reset_gamma(qhp_ctx* c);

int forces_all(qhp_ctx* c, bool energy, bool from_step);

// ---------------------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------------------
#define QHP_DEV __device__ __forceinline__

namespace qhp {

// Philox-4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11).
QHP_DEV void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0;
    const uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

// The Gaussian transform below is written with IEEE +,-,*,/ and sqrt only, in a fixed
// order and without contraction, so that every machine produces the same bits:
//   ln u = e ln2 + 2 atanh((m-1)/(m+1)) with the atanh Taylor series;
//   sin/cos(2 pi u) by exact reduction on u and Taylor series on [-pi/4, pi/4].
#pragma clang fp contract(off)
QHP_DEV double u53(uint64_t x) {
  return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

QHP_DEV double exact_log(double u) {
  int e;
  double m = frexp(u, &e);
  if (m < 0.7071067811865476) { m = m * 2.0; e -= 1; }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = 1.0 / 23.0;
  p = p * s2 + 1.0 / 21.0;
  p = p * s2 + 1.0 / 19.0;
  p = p * s2 + 1.0 / 17.0;
  p = p * s2 + 1.0 / 15.0;
  p = p * s2 + 1.0 / 13.0;
  p = p * s2 + 1.0 / 11.0;
  p = p * s2 + 1.0 / 9.0;
  p = p * s2 + 1.0 / 7.0;
  p = p * s2 + 1.0 / 5.0;
  p = p * s2 + 1.0 / 3.0;
  p = p * s2 + 1.0;
  const double r = (2.0 * s) * p;
  return (double)e * 0.6931471805599453 + r;
}

// factorials as exact doubles; coefficients (-1)^k/(2k+1)! and (-1)^k/(2k)!
QHP_DEV void exact_sincos_2pi(double u, double* sn, double* cs) {
  const double q = rint(4.0 * u);
  const double r = u - q * 0.25;
  const double th = 6.283185307179586 * r;
  const double t = th * th;
  double sp = 1.0 / 355687428096000.0;            // +1/17!
  sp = sp * t + (-1.0 / 1307674368000.0);         // -1/15!
  sp = sp * t + (1.0 / 6227020800.0);             // +1/13!
  sp = sp * t + (-1.0 / 39916800.0);              // -1/11!
  sp = sp * t + (1.0 / 362880.0);                 // +1/9!
  sp = sp * t + (-1.0 / 5040.0);                  // -1/7!
  sp = sp * t + (1.0 / 120.0);                    // +1/5!
  sp = sp * t + (-1.0 / 6.0);                     // -1/3!
  sp = sp * t + 1.0;
  const double s = th * sp;
  double cp = -1.0 / 6402373705728000.0;          // -1/18!
  cp = cp * t + (1.0 / 20922789888000.0);         // +1/16!
  cp = cp * t + (-1.0 / 87178291200.0);           // -1/14!
  cp = cp * t + (1.0 / 479001600.0);              // +1/12!
  cp = cp * t + (-1.0 / 3628800.0);               // -1/10!
  cp = cp * t + (1.0 / 40320.0);                  // +1/8!
  cp = cp * t + (-1.0 / 720.0);                   // -1/6!
  cp = cp * t + (1.0 / 24.0);                     // +1/4!
  cp = cp * t + (-1.0 / 2.0);                     // -1/2!
  cp = cp * t + 1.0;
  const int qi = ((int)q) & 3;
  if (qi == 0) { *sn = s; *cs = cp; }
  else if (qi == 1) { *sn = cp; *cs = -s; }
  else if (qi == 2) { *sn = -s; *cs = -cp; }
  else { *sn = -cp; *cs = s; }
}

// Three standard normals from counter (c0, c1, c2, 0) under key (seed, stream):
// Box-Muller on words (0,1) -> (cos, sin), then words (2,3) -> cos.
QHP_DEV void gauss3(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1, uint64_t c2,
                    double* g) {
  uint64_t c[4] = {c0, c1, c2, 0ull};
  philox4x64(c, seed, stream);
  double sn, cs;
  const double r0 = sqrt(-2.0 * exact_log(u53(c[0])));
  exact_sincos_2pi(u53(c[1]), &sn, &cs);
  g[0] = r0 * cs;
  g[1] = r0 * sn;
  const double r1 = sqrt(-2.0 * exact_log(u53(c[2])));
  exact_sincos_2pi(u53(c[3]), &sn, &cs);
  g[2] = r1 * cs;
}
#pragma clang fp contract(fast)

// Position of step t, axis d, atom a in the segment kernels' copy of the adQTB records
// (coloured noise, recorded velocities): eight consecutive steps of one atom and axis are
// contiguous ([t / 8][N][3][8]), so the kernels that work on one atom's whole segment read
// and write 64-byte runs. The per-step copies are [t][3][N] (a step reads one contiguous
// row per axis); a transpose converts between the two once per segment.
QHP_DEV size_t qtb_rec(int t, int d, int a, int N) {
  return (((size_t)(t >> 3) * N + a) * 3 + d) * 8 + (t & 7);
}

// ---- runtime-length transforms in LDS (lengths with prime factors 2, 3, 5, 7) ----
// One Stockham stage of radix R over nser series of length L stored one after another
// (Ns = product of the earlier radices): butterfly j of a series takes a[j + r L/R],
// r = 0..R-1, multiplies operand r by w^(r k L/(Ns R)), k = j mod Ns, takes their DFT of
// length R and writes it to b[(j / Ns) Ns R + k + q Ns] (natural order after the last
// stage). w^m = tw[m] = exp(-2 pi i m / L); the DFT of length R uses the same table at
// multiples of L/R (R = 3, 5, 7: the direct sum).
template <int R>
QHP_DEV void rt_stage(const double2* a, double2* b, int L, int nser, int Ns, bool inv,
                      const double2* tw) {
  const int nb = L / R;
  for (int jj = threadIdx.x; jj < nb * nser; jj += blockDim.x) {
    const int ser = jj / nb, j = jj - ser * nb;
    const double2* as = a + (size_t)ser * L;
    double2* bs = b + (size_t)ser * L;
    const int k = j % Ns;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = as[j + r * nb];
      if (r) {
        double2 t = tw[r * k * (L / (Ns * R))];
        if (inv) t.y = -t.y;
        v[r] = make_double2(v[r].x * t.x - v[r].y * t.y, v[r].x * t.y + v[r].y * t.x);
      }
    }
    const int idx = (j / Ns) * Ns * R + k;
    if constexpr (R == 4) {
      const double2 t0 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
      const double2 t1 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
      const double2 t2 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
      const double2 t3 = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
      const double2 jt3 = inv ? make_double2(-t3.y, t3.x) : make_double2(t3.y, -t3.x);
      bs[idx] = make_double2(t0.x + t2.x, t0.y + t2.y);
      bs[idx + 2 * Ns] = make_double2(t0.x - t2.x, t0.y - t2.y);
      bs[idx + Ns] = make_double2(t1.x + jt3.x, t1.y + jt3.y);
      bs[idx + 3 * Ns] = make_double2(t1.x - jt3.x, t1.y - jt3.y);
    } else if constexpr (R == 2) {
      bs[idx] = make_double2(v[0].x + v[1].x, v[0].y + v[1].y);
      bs[idx + Ns] = make_double2(v[0].x - v[1].x, v[0].y - v[1].y);
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        double2 acc = v[0];
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double2 w = tw[((q * r) % R) * nb];
          if (inv) w.y = -w.y;
          acc.x += v[r].x * w.x - v[r].y * w.y;
          acc.y += v[r].x * w.y + v[r].y * w.x;
        }
        bs[idx + q * Ns] = acc;
      }
    }
  }
}

// Unnormalised transforms (exp(+...) when inv) of nser series of runtime length L between
// two LDS buffers: radix 4 while four divides what is left, then 2, 3, 5 and 7 (L must have
// no other prime factor). Every thread of the block takes part. Returns the buffer
// holding the result.
QHP_DEV double2* fft_rt(double2* a, double2* b, int L, int nser, bool inv, const double2* tw) {
  for (int Ns = 1; Ns < L;) {
    const int left = L / Ns;
    const int R = left % 4 == 0 ? 4 : left % 2 == 0 ? 2 : left % 3 == 0 ? 3 : left % 5 == 0 ? 5 : 7;
    switch (R) {
      case 4: rt_stage<4>(a, b, L, nser, Ns, inv, tw); break;
      case 2: rt_stage<2>(a, b, L, nser, Ns, inv, tw); break;
      case 3: rt_stage<3>(a, b, L, nser, Ns, inv, tw); break;
      case 5: rt_stage<5>(a, b, L, nser, Ns, inv, tw); break;
      default: rt_stage<7>(a, b, L, nser, Ns, inv, tw); break;
    }
    __syncthreads();
    double2* t = a; a = b; b = t;
    Ns *= R;
  }
  return a;
}

constexpr uint64_t STREAM_RPMD_O = 5;
constexpr uint64_t STREAM_QTB_WHITE = 6;

QHP_DEV unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

// wrapped grid coordinate u = K * frac(x / L) in [0, K] and its integer base (for K a power
// of two 1/K is the exact power 2^-log2(K) and no division is needed)
QHP_DEV double grid_coord(double x, double KoL, int K) {
  const double u = x * KoL;
  const double f = (K & (K - 1)) ? floor(u / (double)K)
                                 : floor(u * ldexp(1.0, -__builtin_ctz((unsigned)K)));
  return u - (double)K * f;
}
// Packed centroid records (FP32-pair contexts without contraction): the w of a centroid
// record, otherwise the atom's largest bead-centroid distance d, carries the atom's charge
// as FP32 (low word) and, in the high word, d as FP32 rounded up to a multiple of 8 ulp
// with the type (0..7) in those three low bits, so that the pair kernel reads one 32-byte
// record per neighbour. d only widens the pair reach (rounding it up keeps the test
// conservative); the charge and type are only moved.
QHP_DEV double pack_record(double q, int t, double d) {
  const unsigned db = (__float_as_uint(__double2float_ru(d)) + 7u) & ~7u;
  return __hiloint2double((int)(db | (unsigned)t), __float_as_int((float)q));
}
QHP_DEV float packed_charge(double w) { return __int_as_float(__double2loint(w)); }
QHP_DEV int packed_type(double w) { return __double2hiint(w) & 7; }
QHP_DEV float packed_spread(double w) { return __uint_as_float((unsigned)__double2hiint(w) & ~7u); }
QHP_DEV int base_of(double x, double KoL, int K) {
  const double fl = floor(grid_coord(x, KoL, K));
  return isfinite(fl) ? min(max((int)fl, 0), K) : 0;
}
// signed difference of two grid bases, wrapped into [-K/2, K/2]
QHP_DEV int base_diff(int a, int b, int K) {
  int d = a - b;
  if (d > K / 2) d -= K;
  if (d < -K / 2) d += K;
  return d;
}

// Bins of a centroid: its 8^3-point SPME spreading tile (by the grid base of each axis)
// and its neighbour-list cell (fractional coordinate times the cell count, floored and
// clamped; no contraction of the multiply-add, as in the list's reference form).
struct BinGeom {
  int* tile_of; int* cell_of;     // [N] outputs (nullptr: not written)
  int K[3], nt1, nt2, nc[3];
  double KoL[3], iL[3];
};
QHP_DEV int tile_of_centroid(const BinGeom& G, double cx, double cy, double cz) {
  const double c[3] = {cx, cy, cz};
  int t[3];
  for (int d = 0; d < 3; ++d) {
    const int b = base_of(c[d], G.KoL[d], G.K[d]);
    t[d] = (b >= G.K[d] ? b - G.K[d] : b) / QHP_TB;
  }
  return (t[0] * G.nt1 + t[1]) * G.nt2 + t[2];
}
#pragma clang fp contract(off)
QHP_DEV int cell_coord(double x, double iL, int n) {
  double f = x * iL;
  f = f - floor(f);
  if (!isfinite(f)) return 0;
  const int i = (int)(f * (double)n);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}
QHP_DEV int cell_of_centroid(const BinGeom& G, double cx, double cy, double cz) {
  return (cell_coord(cx, G.iL[0], G.nc[0]) * G.nc[1] + cell_coord(cy, G.iL[1], G.nc[1])) * G.nc[2] +
         cell_coord(cz, G.iL[2], G.nc[2]);
}
#pragma clang fp contract(fast)
QHP_DEV void write_bins(const BinGeom& G, int a, double cx, double cy, double cz) {
  if (G.tile_of) G.tile_of[a] = tile_of_centroid(G, cx, cy, cz);
  if (G.cell_of) G.cell_of[a] = cell_of_centroid(G, cx, cy, cz);
}

}  // namespace qhp

// bin geometry of the context (tile and cell arrays, grid and cell counts)
qhp::BinGeom bin_geom(const qhp_ctx* c);
