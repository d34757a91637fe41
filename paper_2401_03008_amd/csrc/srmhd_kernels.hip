// srmhd_kernels.hip -- HIP kernels (gfx950) of one SSP Runge-Kutta stage of
// 3D ideal SRMHD on a periodic box, following the substep structure of Sec. 3
// of arXiv 2401.03008: INT + Newton inversion (with the learned guess), REC +
// upwind face fluxes with stored fast speeds, UCT edge fields, DER (flux
// divergence and curl, second or sixth order) fused with the Runge-Kutta
// update, and the once-per-step global speed maximum; plus the diagnostics
// reductions and the training-pair harvest.
//
// Layout: structure of arrays, x fastest; a workgroup is a tile of 64 x BY x
// BZ cells, one wavefront per 64 consecutive x cells of a (y, z) row (16 x 4
// cells in the FP64 flux and UCT kernels), so every global access of a
// wavefront is a contiguous 512-byte (FP64) or 256-byte (FP32) segment, or
// four 128-byte ones.  Periodic wrap replaces ghost cells.
#include "srmhd_kernels.hpp"
#include "srmhd_phys.hpp"

#include <float.h>

namespace srmhd {

constexpr unsigned kErrC2P = 1u, kErrNonfinite = 2u, kErrDt = 4u, kErrPressure = 8u;

// --------------------------------------------------------------- helpers
struct Cell {
  int i, j, k, id;
  int li, lj, lk;  // position in the tile
  bool valid;
};

// Tiles of 64 x BY x BZ cells (BY * BZ <= 16 wavefronts), launched as a 1D
// grid.  A kernel with a stencil along y or z uses a tile that is tall in
// that direction, so a workgroup fetches its rows or planes plus a 5-cell
// halo into its XCD's L2 once instead of one halo per row.
//
// Workgroup L runs on XCD L mod 8.  The grid is taken in groups of 8 rows of
// tiles (a row: the nbx tiles of one (y, z) tile row, x fastest): within a
// group, XCD x gets all tiles of row x, in order, so the x halos of
// neighbouring tiles meet in one L2; the groups follow each other in the
// natural row order, so all XCDs sweep the same planes together and the z
// neighbours of a row (nby rows on, nby a multiple of 8 in the cubes used)
// stay on its XCD.  (Giving each XCD one contiguous slab of the box instead
// measured 3-10% slower: eight distant slabs compete for the shared
// last-level cache.)  Lanes past the end of the box have valid = false.
constexpr int kXcds = 8;

// x cells per wavefront (64: a wavefront is one x row of its tile).  The FP64
// flux and UCT kernels use 16x4-cell wavefronts: MP5 needs its limiter near
// the extremum surfaces of each field, and SIMT runs it for a whole
// wavefront if one lane needs it; a compact wavefront crosses such a surface
// less often (on the diagonal Alfven wave at 128^3, 75% of 64x1 wavefronts per field
// and direction contain a limited cell, 23% of 16x4 ones).  Measured: FP64 +4%
// per step at 256^3 (CPA and turbulence); the FP32 passes were 2-6% slower.
constexpr int kWaveX = 64;
template <typename TS>
constexpr int kStencilWaveX = sizeof(TS) == 8 ? 16 : 64;

template <int BY, int BZ>
struct Tile {
  static constexpr int kY = BY, kZ = BZ, kThreads = kBlockX * BY * BZ;
};

template <int BY, int BZ, int WX = kWaveX>
__device__ __forceinline__ Cell cell_of_tile(const GridDims& g) {
  const int nbx = (g.nx + kBlockX - 1) / kBlockX, nby = (g.ny + BY - 1) / BY;
  const int nbz = (g.nz + BZ - 1) / BZ;
  const int L = blockIdx.x;
  const int slot = L / kXcds;
  const int row = (slot / nbx) * kXcds + L % kXcds;  // by + nby bz
  const int bx = slot % nbx;
  const int by = row % nby, bz = row / nby;
  // Wavefront w (hardware lanes threadIdx.x) covers WXE x cells of RW tile
  // rows, or one whole row where the box is thinner than the tile.
  constexpr int R = BY * BZ;
  constexpr int RW = (kBlockX / WX < R) ? kBlockX / WX : R;
  constexpr int WXE = kBlockX / RW;
  const bool blocks = RW > 1 && g.ny >= BY && g.nz >= BZ;
  const int w = threadIdx.y + BY * threadIdx.z, l = threadIdx.x;
  const int dx = blocks ? (w % RW) * WXE + l % WXE : l;
  const int dr = blocks ? (w / RW) * RW + l / WXE : w;
  Cell c;
  c.li = dx;
  c.lj = dr % BY;
  c.lk = dr / BY;
  c.i = bx * kBlockX + c.li;
  c.j = by * BY + c.lj;
  c.k = bz * BZ + c.lk;
  c.valid = bz < nbz && c.i < g.nx && c.j < g.ny && c.k < g.nz;
  c.id = c.valid ? (c.k * g.ny + c.j) * g.nx + c.i : 0;
  return c;
}

__device__ __forceinline__ Cell cell_of(const GridDims& g) { return cell_of_tile<kBlockY, 1>(g); }

__device__ __forceinline__ int block_linear() { return blockIdx.x; }

// wavefront index within the workgroup and number of wavefronts
__device__ __forceinline__ int wave_in_block() { return threadIdx.z * blockDim.y + threadIdx.y; }
__device__ __forceinline__ int waves_in_block() { return blockDim.y * blockDim.z; }

// Grid of whole groups of kXcds tile rows.
template <int BY, int BZ>
inline dim3 tile_grid(const GridDims& g) {
  const long long nbx = (g.nx + kBlockX - 1) / kBlockX;
  const long long rows = (long long)((g.ny + BY - 1) / BY) * ((g.nz + BZ - 1) / BZ);
  return dim3((unsigned)((rows + kXcds - 1) / kXcds * kXcds * nbx));
}

template <int BY, int BZ>
inline dim3 tile_block() {
  return dim3(kBlockX, BY, BZ);
}

inline dim3 cell_grid(const GridDims& g) { return tile_grid<kBlockY, 1>(g); }

__device__ __forceinline__ int lane_id() { return threadIdx.x; }

// Stencil indices along direction dir at offsets first..first+5 (periodic,
// first >= -3).  A direction with fewer than 4 cells (a 2D or 1D box: the
// stencil wraps more than once) takes the general modulo.
// THIN selects the modulo form at compile time (for kernels whose body is
// instantiated for both cases); the untemplated form branches on n.
template <bool THIN>
__device__ __forceinline__ void stencil6_t(const GridDims& g, const Cell& c, int dir, int first,
                                           int* idx) {
  const int n = dir == 0 ? g.nx : (dir == 1 ? g.ny : g.nz);
  const int co = dir == 0 ? c.i : (dir == 1 ? c.j : c.k);
  const int stride = dir == 0 ? 1 : (dir == 1 ? g.nx : g.nx * g.ny);
  const int base = c.id - co * stride;
  if (THIN) {
#pragma unroll
    for (int m = 0; m < 6; ++m) idx[m] = base + ((co + m + first + 3 * n) % n) * stride;
  } else {
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      int cm = co + m + first;
      cm += cm < 0 ? n : 0;
      cm -= cm >= n ? n : 0;
      idx[m] = base + cm * stride;
    }
  }
}

__device__ __forceinline__ void stencil6_from(const GridDims& g, const Cell& c, int dir,
                                              int first, int* idx) {
  const int n = dir == 0 ? g.nx : (dir == 1 ? g.ny : g.nz);
  if (n >= 4) stencil6_t<false>(g, c, dir, first, idx);
  else stencil6_t<true>(g, c, dir, first, idx);
}

// REC stencil of the +face along dir: cells at offsets -2..+3.
__device__ __forceinline__ void stencil6(const GridDims& g, const Cell& c, int dir, int* idx) {
  stencil6_from(g, c, dir, -2, idx);
}

// Sixth-order derivative at a centre of a quantity f_m stored at the +faces
// (edges) at offsets m = -3..+2 along the direction, i.e. at -5/2..+5/2:
// (-9 f_{-5/2} + 125 f_{-3/2} - 2250 f_{-1/2} + 2250 f_{1/2} - 125 f_{3/2}
//  + 9 f_{5/2}) / 1920, times 1/dx by the caller.  This is the difference of
// the corrected fluxes f - D2 f/24 + 3 D4 f/640 at the two faces (HO DER).
__device__ __forceinline__ double der6(double f0, double f1, double f2, double f3, double f4,
                                       double f5) {
  return (2250.0 * (f3 - f2) - 125.0 * (f4 - f1) + 9.0 * (f5 - f0)) * (1.0 / 1920.0);
}

template <typename P>
__device__ __forceinline__ double der6_at(const P* q, const int* s) {
  return der6((double)q[s[0]], (double)q[s[1]], (double)q[s[2]], (double)q[s[3]],
              (double)q[s[4]], (double)q[s[5]]);
}

// Index of the neighbour at offset -1 along dir (periodic).
__device__ __forceinline__ int minus1(const GridDims& g, const Cell& c, int dir) {
  if (dir == 0) return c.i == 0 ? c.id + g.nx - 1 : c.id - 1;
  if (dir == 1) return c.j == 0 ? c.id + (g.ny - 1) * g.nx : c.id - g.nx;
  return c.k == 0 ? c.id + (g.nz - 1) * g.nx * g.ny : c.id - g.nx * g.ny;
}

// INT: centred B_d of the cell from the face array bfd: the mean of the two
// d-faces, or (ho) the sixth-order interpolation of the six nearest faces,
// (3, -25, 150, 150, -25, 3)/256.
__device__ __forceinline__ double centre_b(const GridDims& g, const Cell& c, const double* bfd,
                                           int d, int ho) {
  if (ho) {
    int s[6];
    stencil6_from(g, c, d, -3, s);
    return (150.0 * (bfd[s[2]] + bfd[s[3]]) - 25.0 * (bfd[s[1]] + bfd[s[4]]) +
            3.0 * (bfd[s[0]] + bfd[s[5]])) * (1.0 / 256.0);
  }
  return 0.5 * (bfd[minus1(g, c, d)] + bfd[c.id]);
}

__device__ __forceinline__ unsigned wave_sum_u32(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Per-workgroup counters in LDS, flushed with one global atomic per nonzero
// entry into replica (workgroup mod kReplicas).
struct BlockCounters {
  unsigned* s;
  __device__ void init(unsigned* sm) {
    s = sm;
    const int tid = wave_in_block() * kBlockX + threadIdx.x;
    if (tid < CNT_N) s[tid] = 0;
    __syncthreads();
  }
  // add `v` (per lane) to counter slot `slot` (uniform), one LDS atomic per wave
  __device__ void add_uniform(int slot, unsigned v) {
    const unsigned w = wave_sum_u32(v);
    if (lane_id() == 0 && w) atomicAdd(&s[slot], w);
  }
  // histogram: add 1 to slot base + bin(lane) for lanes with has = true
  __device__ void add_hist(int base, bool has, int bin) {
    unsigned long long pending = __ballot(has);
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int b = __shfl(bin, leader);
      const unsigned long long same = __ballot(has && bin == b);
      if (lane_id() == leader) atomicAdd(&s[base + b], (unsigned)__popcll(same));
      pending &= ~same;
    }
  }
  __device__ void flush(unsigned long long* global) {
    __syncthreads();
    const int tid = wave_in_block() * kBlockX + threadIdx.x;
    if (tid < CNT_N && s[tid])
      atomicAdd(&global[(block_linear() % kReplicas) * CNT_N + tid], (unsigned long long)s[tid]);
  }
};

// ----------------------------------------------------------------- init
__global__ __launch_bounds__(kThreads) void k_init(InitArgs a) {
  const Cell c = cell_of(a.g);
  if (!c.valid) return;
  double bc[3];
  for (int d = 0; d < 3; ++d) bc[d] = centre_b(a.g, c, a.bf_in[d], d, a.ho);
  FaceState<double> s{a.prim5[0][c.id], a.prim5[1][c.id], a.prim5[2][c.id], a.prim5[3][c.id],
                      a.prim5[4][c.id], bc[0], bc[1], bc[2]};
  FaceEval<double> e;
  const double g1 = a.gam / (a.gam - 1.0);
  face_eval(s, a.gam, g1, e);
  for (int n = 0; n < 5; ++n) a.cons[n][c.id] = e.u[n];
  const double v2 = s.vn * s.vn + s.vt1 * s.vt1 + s.vt2 * s.vt2;
  a.W[c.id] = (s.rho + g1 * s.p) / (1.0 - v2);
  for (int d = 0; d < 3; ++d) a.bf[d][c.id] = a.bf_in[d][c.id];
}

void launch_init(const InitArgs& a, hipStream_t s) {
  const dim3 grid = cell_grid(a.g);
  hipLaunchKernelGGL(k_init, grid, dim3(kBlockX, kBlockY), 0, s, a);
}

// ------------------------------------------------------- Newton inversion
// One-unknown Newton iteration in W = rho h Gamma^2 (the paper's first step
// of a substep, Sec. 3).  v^2(W) = [S^2 + tau^2 (2W + B^2)/W^2]/(W + B^2)^2,
// p(W) = (g-1)/g [W (1 - v^2) - D sqrt(1 - v^2)],
// f(W) = W - p + B^2 (1 + v^2)/2 - tau^2/(2 W^2) - U, tau = S.B.
// A guess with W <= 0 or v^2 >= 1 is replaced by U, doubled until usable; an
// iterate leaving that set is halved back toward the previous one; the step
// test is |dW| <= max(tol W, 8 eps fs/|f'|) with fs the sum of |terms| of f.
struct C2PIn {
  double D, U, S2, B2, tau2, gf;
};

// v^2(W), with 1/W and 1/(W + B^2) from one reciprocal (returned for reuse).
__device__ __forceinline__ double c2p_v2(const C2PIn& q, double W, double& iw, double& iwb) {
  const double WB = W + q.B2;
  const double r = 1.0 / (W * WB);
  iw = WB * r;
  iwb = W * r;
  return (q.S2 + q.tau2 * (2.0 * W + q.B2) * iw * iw) * iwb * iwb;
}

__device__ __forceinline__ bool c2p_usable(const C2PIn& q, double W, double& v2, double& iw,
                                           double& iwb) {
  if (!(W > 0.0) || !isfinite(W)) return false;
  v2 = c2p_v2(q, W, iw, iwb);
  return v2 < 1.0;
}

// returns 0 converged, 1 maxit reached, 2 unusable input, 3 p <= 0 (no floor),
// 4 unusable guess with `strict` set (no iteration done)
__device__ int con2prim(const double* u, double bx, double by, double bz, double gam,
                        double& Wio, int maxit, double tol, double pfloor, double* pr,
                        int& iters, bool& floored, bool strict = false) {
  iters = 0;
  floored = false;
  bool finite = true;
  for (int n = 0; n < 5; ++n) finite = finite && isfinite(u[n]);
  finite = finite && isfinite(bx) && isfinite(by) && isfinite(bz);
  C2PIn q;
  q.D = u[0];
  q.U = u[4];
  q.S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
  q.B2 = bx * bx + by * by + bz * bz;
  const double tau = u[1] * bx + u[2] * by + u[3] * bz;
  q.tau2 = tau * tau;
  q.gf = (gam - 1.0) / gam;
  if (!finite || !(q.D > 0.0) || !(q.U > 0.0)) return 2;

  double w = Wio, v2 = 0.0, iw = 0.0, iwb = 0.0;
  if (!c2p_usable(q, w, v2, iw, iwb)) {
    if (strict) return 4;
    w = q.U;
    for (int n = 0; n < 200 && !c2p_usable(q, w, v2, iw, iwb); ++n) w *= 2.0;
  }
  int it = 0;
  bool conv = false;
  while (it < maxit) {
    ++it;
    const double omv = 1.0 - v2;
    const double sqv = sqrt(omv);
    const double p = q.gf * (w * omv - q.D * sqv);
    const double tb = 0.5 * q.B2 * (1.0 + v2);
    const double iw2 = iw * iw;
    const double tt = 0.5 * q.tau2 * iw2;
    const double f = w - p + tb - tt - q.U;
    const double fs = w + fabs(p) + tb + tt + q.U;
    const double tiw3 = q.tau2 * iw2 * iw;
    const double dv2 = -2.0 * tiw3 * iwb - 2.0 * v2 * iwb;
    // 1/sqrt(1 - v^2) only scales a term of f' (the step's convergence rate,
    // not the root), so the hardware reciprocal square root suffices
    const double isqv = __builtin_amdgcn_rsq(omv);
    const double dp = q.gf * (omv - w * dv2 + 0.5 * q.D * dv2 * isqv);
    const double fp = 1.0 - dp + 0.5 * q.B2 * dv2 + tiw3;
    double wn = w - f / fp;
    double v2n = v2, iwn = iw, iwbn = iwb;
    int n = 0;
    for (; n < 100 && !c2p_usable(q, wn, v2n, iwn, iwbn); ++n) wn = 0.5 * (wn + w);
    if (n == 100) {  // no usable point between the iterates: stay
      wn = w;
      v2n = v2;
      iwn = iw;
      iwbn = iwb;
    }
    const double dw = wn - w;
    w = wn;
    v2 = v2n;
    iw = iwn;
    iwb = iwbn;
    if (fabs(dw) <= fmax(tol * w, 8.0 * DBL_EPSILON * fs / fabs(fp))) {
      conv = true;
      break;
    }
  }
  Wio = w;
  iters = it;
  const double sqv = sqrt(1.0 - v2);
  const double aa = tau * iw;
  pr[0] = q.D * sqv;
  pr[1] = (u[1] + aa * bx) * iwb;
  pr[2] = (u[2] + aa * by) * iwb;
  pr[3] = (u[3] + aa * bz) * iwb;
  pr[4] = q.gf * (w * (1.0 - v2) - q.D * sqv);
  if (pfloor > 0.0 && pr[4] < pfloor * pr[0]) {
    pr[4] = pfloor * pr[0];
    floored = true;
  }
  if (!conv) return 1;
  if (!(pr[4] > 0.0)) return 3;
  return 0;
}

// Guess: the previous W (mode 0), a cold start from U (mode 2), or the
// learned guess W0 = D Gamma + g/(g-1) p Gamma^2 from the network's
// (log(p/D), log Gamma).  Mode 1: W0 seeds Newton only where the previous W
// is unusable (W <= 0, not finite, or v^2(W) >= 1: after a restart from
// conserved data alone); elsewhere Newton starts from the previous W as in
// mode 0, and a workgroup evaluates the network only if one of its cells
// needs it.  If Newton from W0 does not converge, or W0 is unusable, the
// cell is redone from U (and counted).  Mode 3: W0 first in every cell,
// redone from the previous W (and counted) where that fails.
// PROBE (with MLP): write the network outputs and W0 of every cell and stop
// before Newton (the same feature and inference code as the inversion).
template <bool STATS, bool MLP, bool PROBE = false>
__global__ __launch_bounds__(kThreads) void k_c2p(C2PArgs a) {
  __shared__ unsigned s_cnt[CNT_N];
  __shared__ __align__(16) uint16_t s_lx[MLP ? kBlockY * 64 * 16 : 4];
  __shared__ float s_ly[MLP ? kBlockY * 128 : 1];
  BlockCounters bc;
  if (STATS) bc.init(s_cnt);
  const Cell c = cell_of(a.g);
  int iters = 0, rc = 0, mlpfb = 0;
  bool floored = false;
  double u[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
  double b[3] = {0.0, 0.0, 0.0};
  double Wprev = 1.0;
  if (c.valid) {
    for (int n = 0; n < 5; ++n) u[n] = a.cons[n][c.id];
    for (int d = 0; d < 3; ++d) b[d] = centre_b(a.g, c, a.bf[d], d, a.ho);
    Wprev = a.guess == 2 ? -1.0 : a.W[c.id];
  }
  double pr[5];
  double W = Wprev;
  bool need = true;  // this lane seeds Newton with the network's guess
  if (MLP && !PROBE && a.guess == 1) {
    C2PIn q;
    q.D = u[0];
    q.U = u[4];
    q.S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    q.B2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double tau = u[1] * b[0] + u[2] * b[1] + u[3] * b[2];
    q.tau2 = tau * tau;
    q.gf = (a.gam - 1.0) / a.gam;
    double v2, iw, iwb;
    need = c.valid && !c2p_usable(q, Wprev, v2, iw, iwb);
  }
  // the inference is workgroup-wide (its LDS hand-offs use barriers)
  if (MLP && (PROBE || a.guess != 1 || __syncthreads_or(need ? 1 : 0))) {
    const double S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    const double B2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double tau = u[1] * b[0] + u[2] * b[1] + u[3] * b[2];
    float fe[kMlpIn];
    mlp_features_f32(u[0], S2, B2, tau, u[4], fe);
    bool fin = true;
    for (int k = 0; k < kMlpIn; ++k) fin = fin && isfinite(fe[k]);
    if (!fin)
      for (int k = 0; k < kMlpIn; ++k) fe[k] = 0.f;
    float out[kMlpOut];
    mlp_wave(a.mlp, fe, &s_lx[threadIdx.y * 64 * 16], &s_ly[threadIdx.y * 128], out,
             []() { __syncthreads(); });
    const double lor = (double)__expf(fmaxf(out[1], 0.f));
    const double pg = u[0] * (double)__expf(out[0]);
    W = fin ? u[0] * lor + a.gam / (a.gam - 1.0) * pg * lor * lor : -1.0;
    if constexpr (PROBE) {
      if (c.valid) {
        const long long nc = (long long)a.g.nx * a.g.ny * a.g.nz;
        a.mlp_out[c.id] = out[0];
        a.mlp_out[nc + c.id] = out[1];
        if (a.mlp_w0) a.mlp_w0[c.id] = W;
      }
      return;
    }
    if (!need) W = Wprev;
    if (c.valid && need) {
      rc = con2prim(u, b[0], b[1], b[2], a.gam, W, a.maxit, a.tol, a.pfloor, pr, iters, floored,
                    true);
      if (rc == 1 || rc == 4) {
        int it2 = 0;
        // mode 3: the previous W; mode 1 (no usable previous W): from U
        W = a.guess == 3 ? Wprev : -1.0;
        rc = con2prim(u, b[0], b[1], b[2], a.gam, W, a.maxit, a.tol, a.pfloor, pr, it2, floored);
        iters += it2;
        mlpfb = 1;
      }
    } else if (c.valid) {
      rc = con2prim(u, b[0], b[1], b[2], a.gam, W, a.maxit, a.tol, a.pfloor, pr, iters, floored);
    }
  } else if (c.valid) {
    rc = con2prim(u, b[0], b[1], b[2], a.gam, W, a.maxit, a.tol, a.pfloor, pr, iters, floored);
  }
  if (c.valid) {
    a.W[c.id] = W;
    if (a.prim64[0]) {
      for (int n = 0; n < 5; ++n) a.prim64[n][c.id] = pr[n];
      for (int d = 0; d < 3; ++d) a.prim64[5 + d][c.id] = b[d];
    }
    if (a.prim32[0]) {
      for (int n = 0; n < 5; ++n) a.prim32[n][c.id] = (float)pr[n];
      for (int d = 0; d < 3; ++d) a.prim32[5 + d][c.id] = (float)b[d];
    }
    if (a.bf32[0])
      for (int d = 0; d < 3; ++d) a.bf32[d][c.id] = (float)a.bf[d][c.id];
    if (rc != 0 && c.k >= a.g.zplo && c.k < a.g.zphi) {
      const unsigned bit = rc == 1 ? kErrC2P : (rc == 2 ? kErrNonfinite : kErrPressure);
      atomicOr(a.err, bit);
    }
  }
  if (STATS) {
    const bool in = c.valid && interior_plane(a.g, c.k);
    bc.add_uniform(CNT_ITERS, in ? (unsigned)iters : 0u);
    bc.add_uniform(CNT_CALLS, in ? 1u : 0u);
    bc.add_uniform(CNT_FAIL, (in && rc != 0) ? 1u : 0u);
    bc.add_uniform(CNT_FLOOR, (in && floored) ? 1u : 0u);
    if (MLP) bc.add_uniform(CNT_MLPFB, (in && mlpfb) ? 1u : 0u);
    bc.add_hist(CNT_HIST0, in, iters < 31 ? iters : 31);
    bc.flush(a.counters);
  }
}

void launch_c2p(const C2PArgs& a, bool stats, hipStream_t s) {
  const dim3 grid = cell_grid(a.g);
  dim3 blk(kBlockX, kBlockY);
  const bool mlp = a.guess == 1 || a.guess == 3;
  if (mlp && a.mlp_out) {
    hipLaunchKernelGGL((k_c2p<false, true, true>), grid, blk, 0, s, a);
    return;
  }
  if (stats) {
    if (mlp) hipLaunchKernelGGL((k_c2p<true, true>), grid, blk, 0, s, a);
    else hipLaunchKernelGGL((k_c2p<true, false>), grid, blk, 0, s, a);
  } else {
    if (mlp) hipLaunchKernelGGL((k_c2p<false, true>), grid, blk, 0, s, a);
    else hipLaunchKernelGGL((k_c2p<false, false>), grid, blk, 0, s, a);
  }
}

// Training pairs from the current state: cells kept with probability frac
// (counter-based hash of the cell index and seed), inverted from the stored
// W (not written back); features as in the learned guess, targets
// (log(p/D), log Gamma) of the converged primitives.
__device__ __forceinline__ unsigned hash_u32(unsigned x, unsigned seed) {
  x ^= seed * 0x9E3779B9u;
  x ^= x >> 16;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  x *= 0xC2B2AE35u;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(kThreads) void k_harvest(HarvestArgs a) {
  const Cell c = cell_of(a.g);
  if (!c.valid || !interior_plane(a.g, c.k)) return;
  const double r = hash_u32((unsigned)c.id, a.seed) * (1.0 / 4294967296.0);
  if (!(r < a.frac)) return;
  double u[5], b[3], pr[5];
  for (int n = 0; n < 5; ++n) u[n] = a.cons[n][c.id];
  for (int d = 0; d < 3; ++d) b[d] = centre_b(a.g, c, a.bf[d], d, a.ho);
  double W = a.W[c.id];
  int it = 0;
  bool fl = false;
  const int rc = con2prim(u, b[0], b[1], b[2], a.gam, W, a.maxit, a.tol, 0.0, pr, it, fl);
  if (rc != 0) return;
  const double S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
  const double B2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  const double tau = u[1] * b[0] + u[2] * b[1] + u[3] * b[2];
  double f[kMlpIn];
  mlp_features(u[0], S2, B2, tau, u[4], f);
  const unsigned slot = atomicAdd(a.count, 1u);
  if ((int)slot >= a.cap) return;
  for (int k = 0; k < kMlpIn; ++k) a.feats[(size_t)slot * kMlpIn + k] = (float)f[k];
  a.targets[(size_t)slot * kMlpOut + 0] = (float)log(pr[4] / u[0]);
  a.targets[(size_t)slot * kMlpOut + 1] = (float)log(u[0] / pr[0]);
}

void launch_harvest(const HarvestArgs& a, hipStream_t s) {
  const dim3 grid = cell_grid(a.g);
  hipLaunchKernelGGL(k_harvest, grid, dim3(kBlockX, kBlockY), 0, s, a);
}

// ------------------------------------------------ REC + face physics + HLL
// One thread per +face along DIR.  MP5 left/right states of rho, v, p and the
// two transverse centred B; the normal B is the staggered face value.  A face
// state with rho <= 0, p <= 0 or v^2 >= 1 is replaced by its cell's values
// (first order) and counted.  HLL: a+ = max(0, l+_L, l+_R), a- = max(0, -l-_L,
// -l-_R), Fhat = (a+ F_L + a- F_R - a+ a- (U_R - U_L))/(a+ + a-); LLF: a+ =
// a- = max |l|.  Outputs the 5 fluid fluxes, a+-, and the left and right
// states of v_DIR and v_{DIR+1}, the two velocity components that the edge
// field E_{DIR+2} needs at these faces.  With CFL, also the workgroup max of sum_d max(a+,a-)_d/dx_d
// (needs the other two directions' speeds already stored).
// The x and y faces run in one kernel (k_flux_xy below: the primitives of a
// 64x4 (FP64) or 64x8 (FP32) tile and its x and y halos staged once, 3% off
// the FP64 step against two passes that staged them twice); the z faces in
// k_flux<2> on 64x1x4 tiles in FP64 and 64x1x8 in FP32 (the wavefronts of a
// z tile share stencil planes; at 256^3 the FP64 z tile took 3% off the z
// pass, the FP32 one 20%; 64x1x8 or 64x1x16 FP64 tiles were slower).
// STAGED: the stencil operands come from LDS (Stage); a box thinner than the
// z tile (nz = 1: a 2D run) takes the z pass unstaged on 64x4x1 tiles, its
// operands read directly through the periodic stencil indices.
template <int DIR, typename TS, bool STAGED = true>
struct FluxTile : Tile<(DIR == 2 && STAGED) ? 1 : 4,
                       (DIR == 2 && STAGED) ? (sizeof(TS) == 4 ? 8 : 4) : 1> {};

__device__ __forceinline__ int wrap_index(int p, int n) {
  int r = p % n;
  return r + (r < 0 ? n : 0);
}

// LDS staging of stencil operands: a tile of 64 x BY x BZ cells extended by
// a 5-cell halo along D (six-point stencils at offsets LO..LO+5: -2..+3 for
// REC, -3..+2 for the sixth-order differences of face values), x fastest.
// Each value is fetched once per workgroup instead of once per stencil lane,
// and the periodic wrap is resolved once per staged cell.  for_each calls
// f(e, id) for every staged slot e inside the box (id: its cell index); rows
// beyond a ragged box edge are skipped (their lanes are invalid).  Stencil
// point m of tile cell c sits at base(c) + m * kStride.
template <int D, int BY, int BZ, int LO = -2>
struct Stage {
  static constexpr int EX = kBlockX + (D == 0 ? 5 : 0);
  static constexpr int EY = BY + (D == 1 ? 5 : 0);
  static constexpr int EZ = BZ + (D == 2 ? 5 : 0);
  static constexpr int N = EX * EY * EZ;
  static constexpr int kStride = D == 0 ? 1 : (D == 1 ? EX : EX * EY);
  static constexpr int kThreads = kBlockX * BY * BZ;

  __device__ static int base(const Cell& c) { return (c.lk * EY + c.lj) * EX + c.li; }

  template <typename F>
  __device__ static void for_each(const GridDims& g, const Cell& c, F&& f) {
    const int x0 = c.i - c.li, y0 = c.j - c.lj, z0 = c.k - c.lk;
    if (!(x0 < g.nx && y0 < g.ny && z0 < g.nz)) return;  // a padding tile
    const int tid = (int)threadIdx.x + kBlockX * ((int)threadIdx.y + BY * (int)threadIdx.z);
#pragma unroll
    for (int k = 0; k < (N + kThreads - 1) / kThreads; ++k) {
      const int e = tid + k * kThreads;
      if (e >= N) break;
      int gx = x0 + e % EX, gy = y0 + (e / EX) % EY, gz = z0 + e / (EX * EY);
      bool in;
      if (D == 0) {
        gx = wrap_index(gx + LO, g.nx);
        in = gy < g.ny && gz < g.nz;
      } else if (D == 1) {
        gy = wrap_index(gy + LO, g.ny);
        in = gx < g.nx && gz < g.nz;
      } else {
        gz = wrap_index(gz + LO, g.nz);
        in = gx < g.nx && gy < g.ny;
      }
      if (in) f(e, (gz * g.ny + gy) * g.nx + gx);
    }
  }
};

// One face of direction DIR at tile cell c: REC of the seven primitives the
// face reads (val(n, m): stencil point m, offset m - 2, of rho, v_n, v_t1,
// v_t2, p, B_t1, B_t2), the first-order fallback, the face physics and the
// HLL/LLF flux; writes the face arrays and returns a+ and a-.
template <int DIR, typename TS, int REC, typename Val>
__device__ __forceinline__ void flux_face(const FluxArgs<TS>& a, const Cell& c, Val&& val, int& nfb,
                                          TS& ap_out, TS& am_out) {
  using T = TS;
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
    FaceState<T> L, R;
    auto rec = [&](int n, T& l, T& r) {
      if (REC == kRecMc)  // the outer two stencil values are not read
        rec_pair<REC, T>(T(0), val(n, 1), val(n, 2), val(n, 3), val(n, 4), T(0), l, r);
      else
        rec_pair<REC, T>(val(n, 0), val(n, 1), val(n, 2), val(n, 3), val(n, 4), val(n, 5), l, r);
    };
    rec(0, L.rho, R.rho);
    rec(1, L.vn, R.vn);
    rec(2, L.vt1, R.vt1);
    rec(3, L.vt2, R.vt2);
    rec(4, L.p, R.p);
    rec(5, L.bt1, R.bt1);
    rec(6, L.bt2, R.bt2);
    const T bn = (T)a.bn[c.id];
    L.bn = R.bn = bn;
    auto cell_state = [&](int m) {  // the unreconstructed state of stencil cell m
      return FaceState<T>{val(0, m), val(1, m), val(2, m), val(3, m),
                          val(4, m), bn,        val(5, m), val(6, m)};
    };
    if (!face_state_ok(L)) {
      L = cell_state(2);
      ++nfb;
    }
    if (!face_state_ok(R)) {
      R = cell_state(3);
      ++nfb;
    }
    const T g = (T)a.gam, g1 = (T)(a.gam / (a.gam - 1.0));
    FaceEval<T> eL, eR;
    face_eval(L, g, g1, eL);
    face_eval(R, g, g1, eR);
    T ap, am;
    if (a.riemann == 1) {
      ap = fmax(fmax(fabs(eL.lm), fabs(eL.lp)), fmax(fabs(eR.lm), fabs(eR.lp)));
      am = ap;
    } else {
      ap = fmax(T(0), fmax(eL.lp, eR.lp));
      am = fmax(T(0), fmax(-eL.lm, -eR.lm));
    }
    ap_out = ap;
    am_out = am;
    const T sum = ap + am;
    T F[5];
    if (sum > T(0)) {
      const T inv = recip(sum), apam = ap * am;
#pragma unroll
      for (int n = 0; n < 5; ++n) F[n] = (ap * eL.f[n] + am * eR.f[n] - apam * (eR.u[n] - eL.u[n])) * inv;
    } else {
#pragma unroll
      for (int n = 0; n < 5; ++n) F[n] = T(0.5) * (eL.f[n] + eR.f[n]);
    }
    a.fhat[0][c.id] = F[0];
    a.fhat[1 + DIR][c.id] = F[1];
    a.fhat[1 + T1][c.id] = F[2];
    a.fhat[1 + T2][c.id] = F[3];
    a.fhat[4][c.id] = F[4];
    a.ap[c.id] = ap;
    a.am[c.id] = am;
    a.fv[0][c.id] = L.vn;
    a.fv[1][c.id] = L.vt1;
    a.fv[2][c.id] = R.vn;
    a.fv[3][c.id] = R.vt1;
}

template <int DIR, typename TS, bool CFL, bool STATS, int REC, bool STAGED>
__global__ __launch_bounds__((FluxTile<DIR, TS, STAGED>::kThreads)) void k_flux(FluxArgs<TS> a) {
  using T = TS;
  using Tl = FluxTile<DIR, TS, STAGED>;
  using St = Stage<DIR, Tl::kY, Tl::kZ>;
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
  __shared__ unsigned s_cnt[CNT_N];
  __shared__ double s_max[16];
  __shared__ TS s_q[STAGED ? 7 : 1][STAGED ? St::N : 1];  // rho, v_n, v_t1, v_t2, p, B_t1, B_t2
  BlockCounters bc;
  if (STATS) bc.init(s_cnt);
  const Cell c = cell_of_tile<Tl::kY, Tl::kZ, kStencilWaveX<TS>>(a.g);
  const TS* q[7] = {a.prim[0], a.prim[1 + DIR], a.prim[1 + T1], a.prim[1 + T2],
                    a.prim[4], a.prim[5 + T1],  a.prim[5 + T2]};
  if constexpr (STAGED) {
    St::for_each(a.g, c, [&](int e, int id) {
#pragma unroll
      for (int n = 0; n < 7; ++n) s_q[n][e] = q[n][id];
    });
    __syncthreads();
  }
  int nfb = 0;
  double cfl_sum = 0.0;
  const bool inner = c.valid && interior_plane(a.g, c.k);
  if (c.valid) {
    // stencil point m (offset m - 2) of primitive n
    int idx[6];
    if constexpr (!STAGED) stencil6(a.g, c, DIR, idx);
    const int b = STAGED ? St::base(c) : 0;
    auto val = [&](int n, int m) -> T {
      if constexpr (STAGED) return s_q[n][b + m * St::kStride];
      else return q[n][idx[m]];
    };
    T ap, am;
    flux_face<DIR, TS, REC>(a, c, val, nfb, ap, am);
    if (CFL && inner) {
      // sum over d = 0, 1, 2 in that order; the other directions' speeds are
      // apm_other = {a+_T1, a-_T1, a+_T2, a-_T2}
      double m[3];
      m[DIR] = (double)fmax(ap, am);
      m[T1] = (double)fmax(a.apm_other[0][c.id], a.apm_other[1][c.id]);
      m[T2] = (double)fmax(a.apm_other[2][c.id], a.apm_other[3][c.id]);
      cfl_sum = m[0] * a.g.inv_dx[0] + m[1] * a.g.inv_dx[1] + m[2] * a.g.inv_dx[2];
    }
  }
  if (CFL) {
    const double w = wave_max_f64(cfl_sum);
    if (lane_id() == 0) s_max[wave_in_block()] = w;
    __syncthreads();
    if (threadIdx.x == 0 && wave_in_block() == 0) {
      double b = s_max[0];
      for (int n = 1; n < waves_in_block(); ++n) b = fmax(b, s_max[n]);
      // +double bit patterns order like unsigned integers; NaN sorts above inf
      atomicMax(a.amax_bits, (unsigned long long)__double_as_longlong(b));
    }
  }
  if (STATS) {
    bc.add_uniform(CNT_FALLBACK, inner ? (unsigned)nfb : 0u);
    bc.flush(a.counters);
  }
}

template <typename TS, int REC, bool ZSTAGED>
void launch_flux_z_rec(const FluxArgs<TS>& a, bool cfl, bool stats, hipStream_t s) {
#define SRMHD_FLUX(C, S)                                                                        \
  hipLaunchKernelGGL((k_flux<2, TS, C, S, REC, ZSTAGED>),                                       \
                     (tile_grid<FluxTile<2, TS, ZSTAGED>::kY, FluxTile<2, TS, ZSTAGED>::kZ>(a.g)), \
                     (tile_block<FluxTile<2, TS, ZSTAGED>::kY, FluxTile<2, TS, ZSTAGED>::kZ>()), 0, s, a)
  if (cfl) {
    if (stats) SRMHD_FLUX(true, true); else SRMHD_FLUX(true, false);
  } else {
    if (stats) SRMHD_FLUX(false, true); else SRMHD_FLUX(false, false);
  }
#undef SRMHD_FLUX
}

template <typename TS, int REC>
void launch_flux_z_rec(const FluxArgs<TS>& a, bool cfl, bool stats, hipStream_t s) {
  if (a.g.nz < FluxTile<2, TS>::kZ)
    launch_flux_z_rec<TS, REC, false>(a, cfl, stats, s);
  else
    launch_flux_z_rec<TS, REC, true>(a, cfl, stats, s);
}

template <typename TS>
void launch_flux_z(const FluxArgs<TS>& a, bool cfl, bool stats, int rec, hipStream_t s) {
  if (rec == kRecMc) launch_flux_z_rec<TS, kRecMc>(a, cfl, stats, s);
  else if (rec == kRecMp5Point) launch_flux_z_rec<TS, kRecMp5Point>(a, cfl, stats, s);
  else launch_flux_z_rec<TS, kRecMp5>(a, cfl, stats, s);
}
template void launch_flux_z<double>(const FluxArgs<double>&, bool, bool, int, hipStream_t);
template void launch_flux_z<float>(const FluxArgs<float>&, bool, bool, int, hipStream_t);

// Primitive of stencil array n (rho, v_n, v_t1, v_t2, p, B_t1, B_t2) for the
// faces of direction dir, in the order rho, vx, vy, vz, p, Bx, By, Bz.
__host__ __device__ constexpr int face_prim(int dir, int n) {
  return n == 0 ? 0 : n == 4 ? 4 : n <= 3 ? 1 + (dir + n - 1) % 3 : 5 + (dir + n - 4) % 3;
}

// The x and the y faces of a 64 x BY tile in one pass: the eight primitives
// are staged once over the tile plus the REC halo in x and y ((64 + 5) x
// (BY + 5) cells, offsets -2..+3; the corners are staged too and not read),
// then each lane evaluates its x face and its y face (flux_face).  Measured
// at 512^3 against two staged passes: FP64 BY = 4 -10% (8: -5%, 16: +6%),
// FP32 BY = 8 -8% (4: -3%, 16: -1%).
template <typename TS, bool STATS, int REC, int BY>
__global__ __launch_bounds__(kBlockX * BY) void k_flux_xy(FluxArgs<TS> ax, FluxArgs<TS> ay) {
  constexpr int EX = kBlockX + 5, EY = BY + 5, N = EX * EY, NT = kBlockX * BY;
  __shared__ unsigned s_cnt[CNT_N];
  __shared__ TS s_p[8][N];
  BlockCounters bc;
  if (STATS) bc.init(s_cnt);
  const GridDims& g = ax.g;
  const Cell c = cell_of_tile<BY, 1, kStencilWaveX<TS>>(g);
  {
    const int x0 = c.i - c.li, y0 = c.j - c.lj, z = c.k - c.lk;
    if (x0 < g.nx && y0 < g.ny && z < g.nz) {  // not a padding tile
      const int tid = (int)threadIdx.x + kBlockX * (int)threadIdx.y;
      const size_t zoff = (size_t)z * g.ny * g.nx;
      for (int e = tid; e < N; e += NT) {
        const int gx = wrap_index(x0 - 2 + e % EX, g.nx);
        const int gy = wrap_index(y0 - 2 + e / EX, g.ny);
        const int id = (int)(zoff + (size_t)gy * g.nx + gx);
#pragma unroll
        for (int n = 0; n < 8; ++n) s_p[n][e] = ax.prim[n][id];
      }
    }
    __syncthreads();
  }
  int nfb = 0;
  const bool inner = c.valid && interior_plane(g, c.k);
  if (c.valid) {
    const int bxs = (c.lj + 2) * EX + c.li;  // x stencil point m: (li + m, lj + 2)
    const int bys = c.lj * EX + c.li + 2;    // y stencil point m: (li + 2, lj + m)
    TS ap, am;
    flux_face<0, TS, REC>(ax, c, [&](int n, int m) -> TS { return s_p[face_prim(0, n)][bxs + m]; },
                          nfb, ap, am);
    flux_face<1, TS, REC>(ay, c,
                          [&](int n, int m) -> TS { return s_p[face_prim(1, n)][bys + m * EX]; },
                          nfb, ap, am);
  }
  if (STATS) {
    bc.add_uniform(CNT_FALLBACK, inner ? (unsigned)nfb : 0u);
    bc.flush(ax.counters);
  }
}

template <typename TS>
void launch_flux_xy(const FluxArgs<TS>& ax, const FluxArgs<TS>& ay, bool stats, int rec,
                    hipStream_t s) {
  constexpr int BY = sizeof(TS) == 8 ? 4 : 8;
#define SRMHD_FXY(ST, R)                                                                   \
  hipLaunchKernelGGL((k_flux_xy<TS, ST, R, BY>), (tile_grid<BY, 1>(ax.g)),                 \
                     (tile_block<BY, 1>()), 0, s, ax, ay)
  if (rec == kRecMc) {
    if (stats) SRMHD_FXY(true, kRecMc); else SRMHD_FXY(false, kRecMc);
  } else if (rec == kRecMp5Point) {
    if (stats) SRMHD_FXY(true, kRecMp5Point); else SRMHD_FXY(false, kRecMp5Point);
  } else {
    if (stats) SRMHD_FXY(true, kRecMp5); else SRMHD_FXY(false, kRecMp5);
  }
#undef SRMHD_FXY
}
template void launch_flux_xy<double>(const FluxArgs<double>&, const FluxArgs<double>&, bool, int,
                                     hipStream_t);
template void launch_flux_xy<float>(const FluxArgs<float>&, const FluxArgs<float>&, bool, int,
                                    hipStream_t);

// ------------------------------------------------------------------- UCT
// Edge field E_K at (+1/2 along P, +1/2 along Q), (P, Q, K) cyclic, in FP64:
// the two P-face velocity states (left/right along P) are MP5-reconstructed
// along Q to the edge (corner states ab), B_P (P faces) along Q, B_Q (Q faces)
// along P; E^{ab} = v_Q^{ab} B_P^b - v_P^{ab} B_Q^a (E = -v x B); edge speeds
// are the maxima over the two adjacent faces of each direction.  REC runs in
// the flux precision (FP32 in the mixed form, like the face reconstructions);
// the edge formula stays FP64.
//
// One kernel per orientation K, on a tile that is long along Q (64x8x1 for
// E_z, 64x1x8 for E_x and E_y): the five arrays reconstructed along Q (the
// four P-face velocities and B_P) are staged in LDS with their Q halo, and
// B_Q along P too where the tile is longer than one cell along P (E_z: x,
// E_y: z); E_x reads B_z along y directly.  A box thinner than the tile
// along Q (nz < 8 for E_x and E_y: a 2D run) takes the unstaged form on
// 64x4x1 tiles, every operand read through the periodic stencil indices.
template <int K, bool STAGED = true>
struct UctTile : Tile<!STAGED ? 4 : (K == 2 ? 8 : 1), (!STAGED || K == 2) ? 1 : 8> {};

__device__ __forceinline__ int plus1(const GridDims& g, const Cell& c, int dir) {
  if (dir == 0) return c.i == g.nx - 1 ? c.id - (g.nx - 1) : c.id + 1;
  if (dir == 1) return c.j == g.ny - 1 ? c.id - (g.ny - 1) * g.nx : c.id + g.nx;
  return c.k == g.nz - 1 ? c.id - (g.nz - 1) * g.nx * g.ny : c.id + g.nx * g.ny;
}

template <int K, typename TS, int REC, bool STAGED>
__global__ __launch_bounds__((UctTile<K, STAGED>::kThreads)) void k_uct(Uct3Args<TS> a) {
  constexpr int P = (K + 1) % 3, Q = (K + 2) % 3;
  using Tl = UctTile<K, STAGED>;
  using SQ = Stage<Q, Tl::kY, Tl::kZ>;
  using SP = Stage<P, Tl::kY, Tl::kZ>;
  constexpr bool kStageP = STAGED && (P == 0 ? kBlockX : (P == 1 ? Tl::kY : Tl::kZ)) > 1;
  __shared__ TS s_q[STAGED ? 5 : 1][STAGED ? SQ::N : 1];  // left v_P, v_Q; right v_P, v_Q; B_P
  __shared__ TS s_p[kStageP ? SP::N : 1];                 // B_Q
  const Cell c = cell_of_tile<Tl::kY, Tl::kZ, kStencilWaveX<TS>>(a.g);
  if constexpr (STAGED) {
    SQ::for_each(a.g, c, [&](int e, int id) {
#pragma unroll
      for (int n = 0; n < 4; ++n) s_q[n][e] = a.fv[P][n][id];
      s_q[4][e] = (TS)a.bf[P][id];
    });
    if constexpr (kStageP) SP::for_each(a.g, c, [&](int e, int id) { s_p[e] = (TS)a.bf[Q][id]; });
    __syncthreads();
  }
  if (!c.valid) return;
  int iq[6], ip[6];
  if constexpr (!STAGED) stencil6(a.g, c, Q, iq);
  if constexpr (!kStageP) stencil6(a.g, c, P, ip);
  const int bq = STAGED ? SQ::base(c) : 0, bp = kStageP ? SP::base(c) : 0;
  // stencil point m (offset m - 2) along Q of array n (0..3: the P-face
  // velocities, 4: B_P), and along P of B_Q
  auto qv = [&](int n, int m) -> TS {
    if constexpr (STAGED) return s_q[n][bq + m * SQ::kStride];
    else return n < 4 ? a.fv[P][n][iq[m]] : (TS)a.bf[P][iq[m]];
  };
  auto pv = [&](int m) -> TS {
    if constexpr (kStageP) return s_p[bp + m * SP::kStride];
    else return (TS)a.bf[Q][ip[m]];
  };
  using R = TS;
  auto rec = [&](auto v, double& l, double& r) {
    R lr, rr;
    if (REC == kRecMc)  // the outer two stencil values are not read
      rec_pair<REC, R>(R(0), v(1), v(2), v(3), v(4), R(0), lr, rr);
    else
      rec_pair<REC, R>(v(0), v(1), v(2), v(3), v(4), v(5), lr, rr);
    l = (double)lr;
    r = (double)rr;
  };
  double vp[2][2], vq[2][2];
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
    rec([&](int m) { return qv(2 * sd, m); }, vp[sd][0], vp[sd][1]);      // v_P
    rec([&](int m) { return qv(2 * sd + 1, m); }, vq[sd][0], vq[sd][1]);  // v_Q, Q = P + 1 cyclically
  }
  double bpL, bpR, bqL, bqR;
  rec([&](int m) { return qv(4, m); }, bpL, bpR);
  rec(pv, bqL, bqR);
  const int iq1 = plus1(a.g, c, Q), ip1 = plus1(a.g, c, P);
  const double app = fmax((double)a.ap[P][c.id], (double)a.ap[P][iq1]);
  const double amp = fmax((double)a.am[P][c.id], (double)a.am[P][iq1]);
  const double aqp = fmax((double)a.ap[Q][c.id], (double)a.ap[Q][ip1]);
  const double aqm = fmax((double)a.am[Q][c.id], (double)a.am[Q][ip1]);
  double E[2][2];
#pragma unroll
  for (int sa = 0; sa < 2; ++sa)
#pragma unroll
    for (int sb = 0; sb < 2; ++sb)
      E[sa][sb] = vq[sa][sb] * (sb ? bpR : bpL) - vp[sa][sb] * (sa ? bqR : bqL);
  a.e[K][c.id] = uct_edge<double>(E[0][0], E[0][1], E[1][0], E[1][1], app, amp, aqp, aqm, bqL,
                                  bqR, bpL, bpR);
}

template <typename TS, int REC>
void launch_uct_rec(const Uct3Args<TS>& a, int k, hipStream_t s) {
#define SRMHD_UCT(K, G)                                                                  \
  hipLaunchKernelGGL((k_uct<K, TS, REC, G>),                                             \
                     (tile_grid<UctTile<K, G>::kY, UctTile<K, G>::kZ>(a.g)),             \
                     (tile_block<UctTile<K, G>::kY, UctTile<K, G>::kZ>()), 0, s, a)
  if (k == 2) {
    if (a.g.ny >= UctTile<2>::kY) SRMHD_UCT(2, true); else SRMHD_UCT(2, false);
  } else if (k == 0) {
    if (a.g.nz >= UctTile<0>::kZ) SRMHD_UCT(0, true); else SRMHD_UCT(0, false);
  } else {
    if (a.g.nz >= UctTile<1>::kZ) SRMHD_UCT(1, true); else SRMHD_UCT(1, false);
  }
#undef SRMHD_UCT
}

template <typename TS>
void launch_uct(const Uct3Args<TS>& a, int k, int rec, hipStream_t s) {
  if (rec == kRecMc) launch_uct_rec<TS, kRecMc>(a, k, s);
  else if (rec == kRecMp5Point) launch_uct_rec<TS, kRecMp5Point>(a, k, s);
  else launch_uct_rec<TS, kRecMp5>(a, k, s);
}
template void launch_uct<double>(const Uct3Args<double>&, int, int, hipStream_t);
template void launch_uct<float>(const Uct3Args<float>&, int, int, hipStream_t);

// -------------------------------------------------- DER + RK stage update
// L(U) at centres: -sum_d (Fhat(+d face) - Fhat(-d face))/dx_d; at faces:
// dB_d/dt = -(d_p E_q - d_q E_p), (d, p, q) cyclic.  HO: the sixth-order
// differences (der6) of the face fluxes and edge fields instead.  SSP-RK3
// (Shu & Osher): stage 1: U1 = U^n + dt L(U^n); stage 2: U2 = 3/4 U^n +
// 1/4 (U1 + dt L(U1)); stage 3: U^{n+1} = 1/3 U^n + 2/3 (U2 + dt L(U2)).
// SSP-RK2: stage 1, then stage 4: U^{n+1} = 1/2 U^n + 1/2 (U1 + dt L(U1)).
// Stage 0 writes L only.  Stage 1 writes U1 to a work register, so U^n stays
// in the caller's arrays and is read back by the later stages (no copy).

// The stage's combination of U^n (u0), the stage input u and L(U) = r.  The
// fused multiply-adds are written out, so every kernel that forms it (the
// update, and the fused update re-deriving a neighbour's face B) rounds it
// the same way.
template <int STAGE>
__device__ __forceinline__ double rk_combine(double u0, double u, double dt, double r) {
  const double e = __builtin_fma(dt, r, u);  // u + dt r
  if (STAGE == 1) return e;
  if (STAGE == 2) return __builtin_fma(0.75, u0, 0.25 * e);
  if (STAGE == 3) return __builtin_fma(1.0 / 3.0, u0, (2.0 / 3.0) * e);
  return __builtin_fma(0.5, u0, 0.5 * e);
}

// The stage's combination of U with L(U) = r (stage 0: store r instead).
template <int STAGE, typename TS>
__device__ __forceinline__ void rk_apply(const UpdArgs<TS>& a, const Cell& c, const double* r) {
  if (STAGE == 0) {
#pragma unroll
    for (int n = 0; n < 8; ++n) a.rhs_out[n][c.id] = r[n];
    return;
  }
  const double dt = a.sc->dt;
#pragma unroll
  for (int n = 0; n < 8; ++n)
    a.uout[n][c.id] =
        rk_combine<STAGE>(STAGE == 1 ? 0.0 : a.u0[n][c.id], a.ucur[n][c.id], dt, r[n]);
}

// -(curl E) on a face from the two edge-field differences across it:
// -((a0 - a1) ia - (b0 - b1) ib), with its one fused multiply-add written out
// (the same rounding wherever it is formed).
__device__ __forceinline__ double curl_face(double a0, double a1, double ia, double b0, double b1,
                                            double ib) {
  return -__builtin_fma(a0 - a1, ia, -((b0 - b1) * ib));
}

// The plain update kernels march each thread along z over kUpdZ planes of
// its (i, j) column (64 x 4 x kUpdZ cells per workgroup): the -z face fluxes
// and the edge fields of the plane below are the ones the thread read as the
// +z values of its previous plane, so each plane reads them once instead of
// twice.  The sums are formed in the same order as with one cell per thread.
constexpr int kUpdZ = 8;

// Second-order DER of the five conserved variables: -sum_d (F(+d face) -
// F(-d face)) / dx_d over d = 0, 1, 2 in that order, with the -z fluxes from
// fzm (updated to this plane's +z fluxes).
template <typename TS>
__device__ __forceinline__ void der2_fluid(const UpdArgs<TS>& a, int id, int im, int jm,
                                           double* fzm, double* r) {
  const double* ix = a.g.inv_dx;
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    double acc = 0.0;
    acc = __builtin_fma((double)a.fhat[0][n][id] - (double)a.fhat[0][n][im], ix[0], acc);
    acc = __builtin_fma((double)a.fhat[1][n][id] - (double)a.fhat[1][n][jm], ix[1], acc);
    const double fz = (double)a.fhat[2][n][id];
    acc = __builtin_fma(fz - fzm[n], ix[2], acc);
    fzm[n] = fz;
    r[n] = -acc;
  }
}

template <int STAGE, typename TS>
__global__ __launch_bounds__(kThreads) void k_update(UpdArgs<TS> a) {
  const Cell c0 = cell_of_tile<kBlockY, kUpdZ>(a.g);
  if (!c0.valid) return;
  const GridDims& g = a.g;
  const int plane = g.nx * g.ny;
  const int di = c0.i == 0 ? g.nx - 1 : -1;
  const int dj = c0.j == 0 ? (g.ny - 1) * g.nx : -g.nx;
  const double* ix = g.inv_dx;
  const double* Ex = a.e[0];
  const double* Ey = a.e[1];
  const double* Ez = a.e[2];
  int id = c0.id;
  const int km = c0.k == 0 ? id + (g.nz - 1) * plane : id - plane;
  double fzm[5];
#pragma unroll
  for (int n = 0; n < 5; ++n) fzm[n] = (double)a.fhat[2][n][km];
  double exm = Ex[km], eym = Ey[km];  // E_x, E_y of the plane below
  const int kend = min(c0.k + kUpdZ, g.nz);
  for (int k = c0.k; k < kend; ++k, id += plane) {
    const int im = id + di, jm = id + dj;
    double r[8];
    der2_fluid(a, id, im, jm, fzm, r);
    const double ex0 = Ex[id], ey0 = Ey[id], ez0 = Ez[id];
    r[5] = curl_face(ez0, Ez[jm], ix[1], ey0, eym, ix[2]);
    r[6] = curl_face(ex0, exm, ix[2], ez0, Ez[im], ix[0]);
    r[7] = curl_face(ey0, Ey[im], ix[0], ex0, Ex[jm], ix[1]);
    exm = ex0;
    eym = ey0;
    Cell c = c0;
    c.id = id;
    rk_apply<STAGE>(a, c, r);
  }
}

// The update of stage STAGE (1 or 2: not the step's last) fused with the
// inversion of its result (the next stage's INT + Newton, as k_c2p with guess
// 0 or 2), for periodic boxes with the face-average INT: the updated state
// never leaves the registers before the inversion reads it.  The face average
// needs the updated B of the three minus faces: B_z at k-1 is the one the
// thread computed on its previous plane; B_x at i-1 and B_y at j-1 (and B_z
// at the first plane) are re-derived with the same curl and the same
// combination as the neighbour that stores them, so the centred B is the one
// k_c2p would read back.  That re-reads the neighbours' input B, so the
// face-B output must not alias the stage's input B (stage 2 writes it to its
// own register).  p carries the inversion's outputs (primitives, W) and
// settings.
template <int STAGE, typename TS, bool STATS>
__global__ __launch_bounds__(kThreads) void k_update_c2p(UpdArgs<TS> a, C2PArgs p) {
  __shared__ unsigned s_cnt[CNT_N];
  BlockCounters bc;
  if (STATS) bc.init(s_cnt);
  const Cell c0 = cell_of_tile<kBlockY, kUpdZ>(a.g);
  const GridDims& g = a.g;
  // every lane of a workgroup runs the same planes (the counters are
  // wavefront-wide); lanes past a ragged x or y edge do no work
  const bool lane_ok = c0.i < g.nx && c0.j < g.ny;
  const int i1 = c0.i == 0 ? g.nx - 1 : c0.i - 1;
  const int j1 = c0.j == 0 ? g.ny - 1 : c0.j - 1;
  const double* ix = g.inv_dx;
  const double* Ex = a.e[0];
  const double* Ey = a.e[1];
  const double* Ez = a.e[2];
  const double dt = a.sc->dt;
  auto at = [&](int i, int j, int k) { return (k * g.ny + j) * g.nx + i; };
  // carried from the plane below: its +z face fluxes, E_x and E_y at (i, j),
  // E_x at (i, j-1), E_y at (i-1, j), and its updated B_z
  double fzm[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double exm = 0.0, eym = 0.0, exjm = 0.0, eyim = 0.0, bzm = 0.0;
  const int k0 = c0.k;
  const int kend = min(k0 + kUpdZ, g.nz);
  if (lane_ok && k0 < g.nz) {
    const int k1 = k0 == 0 ? g.nz - 1 : k0 - 1;
    const int km = at(c0.i, c0.j, k1), imkm = at(i1, c0.j, k1), jmkm = at(c0.i, j1, k1);
#pragma unroll
    for (int n = 0; n < 5; ++n) fzm[n] = (double)a.fhat[2][n][km];
    exm = Ex[km];
    eym = Ey[km];
    exjm = Ex[jmkm];
    eyim = Ey[imkm];
    bzm = rk_combine<STAGE>(STAGE == 1 ? 0.0 : a.u0[7][km], a.ucur[7][km], dt,
                            curl_face(eym, eyim, ix[0], exm, exjm, ix[1]));
  }
  for (int k = k0; k < kend; ++k) {
    int iters = 0, rc = 0;
    bool floored = false;
    if (lane_ok) {
      const int id = at(c0.i, c0.j, k), im = at(i1, c0.j, k), jm = at(c0.i, j1, k);
      const int imjm = at(i1, j1, k);
      double r[8];
      der2_fluid(a, id, im, jm, fzm, r);
      const double ex0 = Ex[id], ey0 = Ey[id], ez0 = Ez[id];
      const double exj = Ex[jm], eyi = Ey[im], ezi = Ez[im], ezj = Ez[jm];
      r[5] = curl_face(ez0, ezj, ix[1], ey0, eym, ix[2]);
      r[6] = curl_face(ex0, exm, ix[2], ez0, ezi, ix[0]);
      r[7] = curl_face(ey0, eyi, ix[0], ex0, exj, ix[1]);
      double un[8];
#pragma unroll
      for (int n = 0; n < 8; ++n) {
        un[n] = rk_combine<STAGE>(STAGE == 1 ? 0.0 : a.u0[n][id], a.ucur[n][id], dt, r[n]);
        a.uout[n][id] = un[n];
      }
      // the updated B_x at i-1 and B_y at j-1, re-derived
      const double ezimjm = Ez[imjm];
      const double bxm = rk_combine<STAGE>(STAGE == 1 ? 0.0 : a.u0[5][im], a.ucur[5][im], dt,
                                           curl_face(ezi, ezimjm, ix[1], eyi, eyim, ix[2]));
      const double bym = rk_combine<STAGE>(STAGE == 1 ? 0.0 : a.u0[6][jm], a.ucur[6][jm], dt,
                                           curl_face(exj, exjm, ix[2], ezj, ezimjm, ix[0]));
      const double b[3] = {0.5 * (bxm + un[5]), 0.5 * (bym + un[6]), 0.5 * (bzm + un[7])};
      exm = ex0;
      eym = ey0;
      exjm = exj;
      eyim = eyi;
      bzm = un[7];
      double W = p.guess == 2 ? -1.0 : p.W[id];
      double pr[5];
      rc = con2prim(un, b[0], b[1], b[2], p.gam, W, p.maxit, p.tol, p.pfloor, pr, iters, floored);
      p.W[id] = W;
      if (p.prim64[0]) {
        for (int n = 0; n < 5; ++n) p.prim64[n][id] = pr[n];
        for (int d = 0; d < 3; ++d) p.prim64[5 + d][id] = b[d];
      }
      if (p.prim32[0]) {
        for (int n = 0; n < 5; ++n) p.prim32[n][id] = (float)pr[n];
        for (int d = 0; d < 3; ++d) p.prim32[5 + d][id] = (float)b[d];
      }
      if (p.bf32[0])
        for (int d = 0; d < 3; ++d) p.bf32[d][id] = (float)un[5 + d];
      if (rc != 0) {
        const unsigned bit = rc == 1 ? kErrC2P : (rc == 2 ? kErrNonfinite : kErrPressure);
        atomicOr(p.err, bit);
      }
    }
    if (STATS) {
      bc.add_uniform(CNT_ITERS, lane_ok ? (unsigned)iters : 0u);
      bc.add_uniform(CNT_CALLS, lane_ok ? 1u : 0u);
      bc.add_uniform(CNT_FAIL, (lane_ok && rc != 0) ? 1u : 0u);
      bc.add_uniform(CNT_FLOOR, (lane_ok && floored) ? 1u : 0u);
      bc.add_hist(CNT_HIST0, lane_ok, iters < 31 ? iters : 31);
    }
  }
  if (STATS) bc.flush(p.counters);
}

template <typename TS>
void launch_update_c2p(int stage, const UpdArgs<TS>& a, const C2PArgs& p, bool stats,
                       hipStream_t s) {
  const dim3 grid = tile_grid<kBlockY, kUpdZ>(a.g);
  const dim3 blk = tile_block<kBlockY, 1>();
#define SRMHD_UC(ST)                                                                     \
  if (stats) hipLaunchKernelGGL((k_update_c2p<ST, TS, true>), grid, blk, 0, s, a, p);    \
  else hipLaunchKernelGGL((k_update_c2p<ST, TS, false>), grid, blk, 0, s, a, p);
  if (stage == 1) {
    SRMHD_UC(1)
  } else {
    SRMHD_UC(2)
  }
#undef SRMHD_UC
}
template void launch_update_c2p<double>(int, const UpdArgs<double>&, const C2PArgs&, bool,
                                        hipStream_t);
template void launch_update_c2p<float>(int, const UpdArgs<float>&, const C2PArgs&, bool,
                                       hipStream_t);

// HO DER: sixth-order differences (der6) of the face fluxes and edge fields.
// Each direction differentiates seven arrays: its five face fluxes and the
// two edge fields it curls (x: E_z, E_y; y: E_z, E_x; z: E_y, E_x).  The x and
// the y arrays pass through one LDS buffer in turn (Stage, offsets -3..+2);
// the z arrays are read through the periodic indices (THINZ: the modulo form,
// for nz < 4).  Each difference is taken once and the terms are summed in a
// fixed order.  Tiles of 64x4x1.
template <int STAGE, typename TS, bool THINZ>
__global__ __launch_bounds__(kThreads) void k_update_ho(UpdArgs<TS> a) {
  using SX = Stage<0, kBlockY, 1, -3>;
  using SY = Stage<1, kBlockY, 1, -3>;
  constexpr int NS = SX::N > SY::N ? SX::N : SY::N;
  __shared__ double s_v[7 * NS];
  const Cell c = cell_of_tile<kBlockY, 1>(a.g);
  const double* ix = a.g.inv_dx;
  double d6[3][7];  // [direction][5 fluxes, then the two edge fields above]
  auto der6_lds = [&](const double* v, int k) {
    return der6(v[0], v[k], v[2 * k], v[3 * k], v[4 * k], v[5 * k]);
  };
  SX::for_each(a.g, c, [&](int e, int id) {
#pragma unroll
    for (int n = 0; n < 5; ++n) s_v[n * NS + e] = (double)a.fhat[0][n][id];
    s_v[5 * NS + e] = a.e[2][id];
    s_v[6 * NS + e] = a.e[1][id];
  });
  __syncthreads();
  if (c.valid) {
    const int b = SX::base(c);
#pragma unroll
    for (int m = 0; m < 7; ++m) d6[0][m] = der6_lds(&s_v[m * NS + b], SX::kStride);
  }
  __syncthreads();
  SY::for_each(a.g, c, [&](int e, int id) {
#pragma unroll
    for (int n = 0; n < 5; ++n) s_v[n * NS + e] = (double)a.fhat[1][n][id];
    s_v[5 * NS + e] = a.e[2][id];
    s_v[6 * NS + e] = a.e[0][id];
  });
  __syncthreads();
  if (!c.valid) return;
  {
    const int b = SY::base(c);
#pragma unroll
    for (int m = 0; m < 7; ++m) d6[1][m] = der6_lds(&s_v[m * NS + b], SY::kStride);
  }
  int sz[6];
  stencil6_t<THINZ>(a.g, c, 2, -3, sz);
#pragma unroll
  for (int n = 0; n < 5; ++n) d6[2][n] = der6_at(a.fhat[2][n], sz);
  d6[2][5] = der6_at(a.e[1], sz);
  d6[2][6] = der6_at(a.e[0], sz);
  double r[8];
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) acc += d6[d][n] * ix[d];
    r[n] = -acc;
  }
  r[5] = -(d6[1][5] * ix[1] - d6[2][5] * ix[2]);
  r[6] = -(d6[2][6] * ix[2] - d6[0][5] * ix[0]);
  r[7] = -(d6[0][6] * ix[0] - d6[1][6] * ix[1]);
  rk_apply<STAGE>(a, c, r);
}

// One staging phase of the 3D HO update: arrays M0..M0+CNT-1 of direction D
// (0..4: the D face fluxes, 5, 6: the two edge fields D curls) through the
// LDS buffer, their sixth-order differences into d6[D][M].
template <int D, int M0, int CNT, int BY, int BZ, typename TS>
__device__ __forceinline__ void ho_phase(const UpdArgs<TS>& a, const Cell& c, double* s_v,
                                         double (&d6)[3][7]) {
  using S = Stage<D, BY, BZ, -3>;
  constexpr int E5 = D == 2 ? 1 : 2, E6 = D == 0 ? 1 : 0;  // x: E_z, E_y; y: E_z, E_x; z: E_y, E_x
  S::for_each(a.g, c, [&](int e, int id) {
#pragma unroll
    for (int j = 0; j < CNT; ++j) {
      const int m = M0 + j;
      s_v[j * S::N + e] = m < 5 ? (double)a.fhat[D][m][id] : a.e[m == 5 ? E5 : E6][id];
    }
  });
  __syncthreads();
  if (c.valid) {
    const int b = S::base(c);
#pragma unroll
    for (int j = 0; j < CNT; ++j) {
      const double* v = &s_v[j * S::N + b];
      constexpr int k = S::kStride;
      d6[D][M0 + j] = der6(v[0], v[k], v[2 * k], v[3 * k], v[4 * k], v[5 * k]);
    }
  }
  __syncthreads();
}

// The HO update on 64x4x4 tiles (boxes with nz >= 4): all three directions
// staged, the y and z arrays in two batches (4 + 3) so that one 72 KB buffer
// serves every phase.  Same differences and the same sums as k_update_ho.
template <int STAGE, typename TS>
__global__ __launch_bounds__(kBlockX * 16) void k_update_ho3(UpdArgs<TS> a) {
  constexpr int NX = Stage<0, 4, 4, -3>::N, NY = Stage<1, 4, 4, -3>::N, NZ = Stage<2, 4, 4, -3>::N;
  constexpr int NXS = 7 * NX, NYS = 4 * NY, NZS = 4 * NZ;
  constexpr int NS = NXS > NYS ? (NXS > NZS ? NXS : NZS) : (NYS > NZS ? NYS : NZS);
  __shared__ double s_v[NS];
  const Cell c = cell_of_tile<4, 4>(a.g);
  double d6[3][7];
  ho_phase<0, 0, 7, 4, 4>(a, c, s_v, d6);
  ho_phase<1, 0, 4, 4, 4>(a, c, s_v, d6);
  ho_phase<1, 4, 3, 4, 4>(a, c, s_v, d6);
  ho_phase<2, 0, 4, 4, 4>(a, c, s_v, d6);
  ho_phase<2, 4, 3, 4, 4>(a, c, s_v, d6);
  if (!c.valid) return;
  const double* ix = a.g.inv_dx;
  double r[8];
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) acc += d6[d][n] * ix[d];
    r[n] = -acc;
  }
  r[5] = -(d6[1][5] * ix[1] - d6[2][5] * ix[2]);
  r[6] = -(d6[2][6] * ix[2] - d6[0][5] * ix[0]);
  r[7] = -(d6[0][6] * ix[0] - d6[1][6] * ix[1]);
  rk_apply<STAGE>(a, c, r);
}

template <typename TS>
void launch_update(int stage, const UpdArgs<TS>& a, bool ho, hipStream_t s) {
  const dim3 grid = ho ? tile_grid<kBlockY, 1>(a.g) : tile_grid<kBlockY, kUpdZ>(a.g);
  const dim3 blk = tile_block<kBlockY, 1>();
#define SRMHD_UPD(K, ...)                                                  \
  switch (stage) {                                                        \
    case 0: hipLaunchKernelGGL((K<0, __VA_ARGS__>), grid, blk, 0, s, a); break; \
    case 1: hipLaunchKernelGGL((K<1, __VA_ARGS__>), grid, blk, 0, s, a); break; \
    case 2: hipLaunchKernelGGL((K<2, __VA_ARGS__>), grid, blk, 0, s, a); break; \
    case 3: hipLaunchKernelGGL((K<3, __VA_ARGS__>), grid, blk, 0, s, a); break; \
    default: hipLaunchKernelGGL((K<4, __VA_ARGS__>), grid, blk, 0, s, a); break; \
  }
  if (!ho) {
    SRMHD_UPD(k_update, TS)
  } else if (a.g.nz < 4) {
    SRMHD_UPD(k_update_ho, TS, true)
  } else {
    const dim3 grid3 = tile_grid<4, 4>(a.g);
    const dim3 blk3 = tile_block<4, 4>();
    switch (stage) {
      case 0: hipLaunchKernelGGL((k_update_ho3<0, TS>), grid3, blk3, 0, s, a); break;
      case 1: hipLaunchKernelGGL((k_update_ho3<1, TS>), grid3, blk3, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_update_ho3<2, TS>), grid3, blk3, 0, s, a); break;
      case 3: hipLaunchKernelGGL((k_update_ho3<3, TS>), grid3, blk3, 0, s, a); break;
      default: hipLaunchKernelGGL((k_update_ho3<4, TS>), grid3, blk3, 0, s, a); break;
    }
  }
#undef SRMHD_UPD
}
template void launch_update<double>(int, const UpdArgs<double>&, bool, hipStream_t);
template void launch_update<float>(int, const UpdArgs<float>&, bool, hipStream_t);

// ------------------------------------------------------------ timestep
// dt = cfl / amax (or dt_fixed) once per step, from the first stage's speeds;
// advances t and the step count and clears the running maximum.
__global__ void k_dt(DevScalars* sc, double cfl, double dt_fixed, const double* amax_in) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double amax = amax_in ? *amax_in : __longlong_as_double((long long)sc->amax_bits);
  const double dt = dt_fixed > 0.0 ? dt_fixed : cfl / amax;
  if (!(dt > 0.0) || !isfinite(dt)) atomicOr(&sc->err, kErrDt);
  sc->dt = dt;
  sc->t = sc->t + dt;
  sc->step = sc->step + 1;
  sc->amax_last = amax;
  sc->amax_bits = 0ull;
}

void launch_dt(DevScalars* sc, double cfl, double dt_fixed, const double* amax_in,
               hipStream_t s) {
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(64), 0, s, sc, cfl, dt_fixed, amax_in);
}

__global__ void k_local_amax(const DevScalars* sc, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    *out = __longlong_as_double((long long)sc->amax_bits);
}

void launch_local_amax(const DevScalars* sc, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_local_amax, dim3(1), dim3(64), 0, s, sc, out);
}

// Ghost planes: G contiguous planes of each of the 9 arrays (z is the
// slowest index), one workgroup row per array.
template <bool PACK>
__global__ __launch_bounds__(256) void k_halo(HaloArgs h) {
  const long long n = (long long)h.G * h.plane;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int a = blockIdx.y;
  double* grid = h.a[a] + (long long)h.z0 * h.plane;
  double* buf = h.buf + (long long)a * n;
  if (PACK) buf[i] = grid[i];
  else grid[i] = buf[i];
}

void launch_halo(const HaloArgs& h, bool pack, hipStream_t s) {
  const long long n = (long long)h.G * h.plane;
  if (n == 0) return;
  const dim3 grid((unsigned)((n + 255) / 256), 9);
  if (pack) hipLaunchKernelGGL(k_halo<true>, grid, dim3(256), 0, s, h);
  else hipLaunchKernelGGL(k_halo<false>, grid, dim3(256), 0, s, h);
}

__global__ void k_zero_u64(unsigned long long* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

void launch_zero_u64(unsigned long long* p, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

__global__ void k_fill_f64(double* p, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_f64(double* p, size_t n, double v, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
}

__global__ void k_set_time(DevScalars* sc, double t, long long step) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  sc->t = t;
  sc->step = step;
}

void launch_set_time(DevScalars* sc, double t, long long step, hipStream_t s) {
  hipLaunchKernelGGL(k_set_time, dim3(1), dim3(64), 0, s, sc, t, step);
}

// ------------------------------------------------------------ diagnostics
// Fixed-order reductions (bitwise reproducible): workgroup b sums a fixed
// contiguous chunk, threads in a fixed stride, then a fixed LDS tree; a single
// workgroup combines the partials in order.  Outputs sums of the 8 state
// arrays and max |div_h B| (div_h B = sum_d (B_d(+) - B_d(-))/dx_d).
constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;

int reduce_blocks(const GridDims&) { return kReduceBlocks; }

__global__ __launch_bounds__(kReduceThreads) void k_reduce_partial(ReduceArgs a) {
  __shared__ double sm[9][kReduceThreads];
  const long long N = (long long)a.g.nx * a.g.ny * a.g.nz;
  const long long chunk = (N + a.nblocks - 1) / a.nblocks;
  const long long beg = (long long)blockIdx.x * chunk;
  const long long end = beg + chunk < N ? beg + chunk : N;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int nxy = a.g.nx * a.g.ny;
  for (long long q = beg + threadIdx.x; q < end; q += kReduceThreads) {
    const int id = (int)q;
    const int i = id % a.g.nx, j = (id / a.g.nx) % a.g.ny, k = id / nxy;
    if (!interior_plane(a.g, k)) continue;
    for (int n = 0; n < 8; ++n) acc[n] += a.a[n][id];
    double dv = 0.0;
    if (a.ho) {
      Cell c{};
      c.i = i;
      c.j = j;
      c.k = k;
      c.id = id;
      c.valid = true;
      int s[6];
      for (int d = 0; d < 3; ++d) {
        stencil6_from(a.g, c, d, -3, s);
        dv += der6_at(a.bf[d], s) * a.g.inv_dx[d];
      }
    } else {
      const int im = i == 0 ? id + a.g.nx - 1 : id - 1;
      const int jm = j == 0 ? id + (a.g.ny - 1) * a.g.nx : id - a.g.nx;
      const int km = k == 0 ? id + (a.g.nz - 1) * nxy : id - nxy;
      dv += (a.bf[0][id] - a.bf[0][im]) * a.g.inv_dx[0];
      dv += (a.bf[1][id] - a.bf[1][jm]) * a.g.inv_dx[1];
      dv += (a.bf[2][id] - a.bf[2][km]) * a.g.inv_dx[2];
    }
    acc[8] = fmax(acc[8], fabs(dv));
  }
  for (int n = 0; n < 9; ++n) sm[n][threadIdx.x] = acc[n];
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int n = 0; n < 8; ++n) sm[n][threadIdx.x] += sm[n][threadIdx.x + w];
      sm[8][threadIdx.x] = fmax(sm[8][threadIdx.x], sm[8][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 9) a.partial[blockIdx.x * 9 + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ __launch_bounds__(kReduceThreads) void k_reduce_final(ReduceArgs a) {
  __shared__ double sm[9][kReduceThreads];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < a.nblocks; b += kReduceThreads) {
    for (int n = 0; n < 8; ++n) acc[n] += a.partial[b * 9 + n];
    acc[8] = fmax(acc[8], a.partial[b * 9 + 8]);
  }
  for (int n = 0; n < 9; ++n) sm[n][threadIdx.x] = acc[n];
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int n = 0; n < 8; ++n) sm[n][threadIdx.x] += sm[n][threadIdx.x + w];
      sm[8][threadIdx.x] = fmax(sm[8][threadIdx.x], sm[8][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 9) a.sc->reduce_out[threadIdx.x] = sm[threadIdx.x][0];
}

void launch_reduce(const ReduceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partial, dim3(a.nblocks), dim3(kReduceThreads), 0, s, a);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kReduceThreads), 0, s, a);
}

}  // namespace srmhd
