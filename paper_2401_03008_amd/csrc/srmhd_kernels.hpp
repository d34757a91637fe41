// srmhd_kernels.hpp -- kernel argument blocks and launchers shared by the
// kernel and C-ABI translation units of libsrmhd.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "srmhd_mlp.hpp"

namespace srmhd {

// Reconstruction kernels: MP5 on the cell-average kernel, linear with the MC
// limiter, MP5 around the point-value interpolation (HO scheme).
constexpr int kRecMp5 = 0, kRecMc = 1, kRecMp5Point = 2;

constexpr int kBlockX = 64;  // one wavefront along x
constexpr int kBlockY = 4;   // four wavefronts per workgroup
constexpr int kThreads = kBlockX * kBlockY;

// Replicated device counters (spread over kReplicas copies so that the
// per-workgroup atomics of 10^5 workgroups do not queue on one address).
constexpr int kReplicas = 64;
enum Counter {
  CNT_ITERS = 0,
  CNT_CALLS = 1,
  CNT_HIST0 = 2,  // 32 bins
  CNT_FAIL = 34,
  CNT_FALLBACK = 35,
  CNT_FLOOR = 36,
  CNT_MLPFB = 37,
  CNT_N = 40
};

// Device-resident scalars at the head of the work buffer.
struct DevScalars {
  unsigned long long amax_bits;  // running max of the CFL sum (bits of a +double)
  double amax_last;
  double dt;
  double t;
  long long step;
  unsigned int err;
  unsigned int pad;
  double reduce_out[16];  // diagnostics results
  unsigned long long harvest;  // slot counter of the training-pair harvest
};

// nz counts every plane of the arrays.  A z-slab context (ghost planes
// below and above its interior) computes on all planes as if they were a
// periodic box and keeps only the interior: the CFL maximum, the counters,
// the diagnostics and the harvest take planes [zlo, zhi), and inversion
// errors count on [zplo, zphi), the planes whose primitives the interior's
// fluxes read (the outermost ghost planes hold wrapped, meaningless data).
// A periodic box has zlo = zplo = 0, zhi = zphi = nz.
struct GridDims {
  int nx, ny, nz;
  double inv_dx[3];
  int zlo, zhi, zplo, zphi;
};

__host__ __device__ inline bool interior_plane(const GridDims& g, int k) {
  return k >= g.zlo && k < g.zhi;
}

struct C2PArgs {
  GridDims g;
  const double* cons[5];
  const double* bf[3];
  double* W;
  double* prim64[8];  // FP64 outputs (or null)
  float* prim32[8];   // FP32 copies for the mixed form (or null)
  float* bf32[3];     // mixed form: FP32 copies of the face B (or null)
  double gam, tol, pfloor;
  int maxit;
  int guess;  // 0 = previous W, 1 = learned guess (fallback previous W), 2 = cold start
  int ho;     // 1: sixth-order INT of the face B
  MlpDev mlp;
  unsigned long long* counters;
  unsigned int* err;
  // Learned-guess probe (guess 1 only): when mlp_out is set the kernel writes
  // the network's de-standardised outputs (log(p/D), log Gamma) of every cell
  // to mlp_out[0..ncell) and mlp_out[ncell..2 ncell), and the guess W0 they
  // give (-1 where the features are not finite) to mlp_w0 if set, and stops
  // there: no Newton, no W, no primitives.
  float* mlp_out;
  double* mlp_w0;
};

struct HarvestArgs {
  GridDims g;
  const double* cons[5];
  const double* bf[3];
  const double* W;
  double gam, tol;
  int maxit;
  float* feats;    // cap x 5
  float* targets;  // cap x 2
  int cap;
  unsigned int* count;
  double frac;
  unsigned int seed;
  int ho;
};

template <typename TS>
struct FluxArgs {
  GridDims g;
  const TS* prim[8];   // rho, vx, vy, vz, p, Bcx, Bcy, Bcz
  const TS* bn;        // face-normal B of this direction (FP32 copy in the mixed form)
  TS* fhat[5];         // D, Sx, Sy, Sz, U fluxes at the +face
  TS* ap;
  TS* am;
  TS* fv[4];           // left v_n, v_t1; right v_n, v_t1 at the +face (t1 = next
                       // direction cyclically: the components the edge fields use)
  const TS* apm_other[4];  // a+/a- of the other two directions (CFL fusion)
  unsigned long long* amax_bits;
  double gam;
  int riemann;
  unsigned long long* counters;
};

// Arrays of the edge-field kernels, for all three orientations (one launch
// per orientation reads its share).
template <typename TS>
struct Uct3Args {
  GridDims g;
  const TS* fv[3][4];  // per face direction d: left v_d, v_{d+1}; right v_d, v_{d+1}
  const TS* ap[3];
  const TS* am[3];
  const TS* bf[3];  // face B (FP32 copies in the mixed form)
  double* e[3];
};

template <typename TS>
struct UpdArgs {
  GridDims g;
  const TS* fhat[3][5];
  const double* e[3];
  const double* ucur[8];  // the stage's input: D, Sx, Sy, Sz, U, Bx, By, Bz
  const double* u0[8];    // U^n (stages 2 and 3)
  double* uout[8];        // the stage's output (may alias ucur or u0 pointwise)
  double* rhs_out[8];     // stage 0: write L(U) here instead of updating
  const DevScalars* sc;
};

struct InitArgs {
  GridDims g;
  const double* prim5[5];
  const double* bf_in[3];
  double* cons[5];
  double* bf[3];
  double* W;
  double gam;
  int ho;
};

struct ReduceArgs {
  GridDims g;
  const double* a[8];
  const double* bf[3];
  double* partial;  // [nblocks][9]
  int nblocks;
  DevScalars* sc;
  int ho;  // 1: div B with the sixth-order differences
};

// Launchers (srmhd_kernels.hip).  All asynchronous on `stream`.
void launch_init(const InitArgs& a, hipStream_t s);
void launch_c2p(const C2PArgs& a, bool stats, hipStream_t s);
void launch_harvest(const HarvestArgs& a, hipStream_t s);
// rec: kRecMp5, kRecMc or kRecMp5Point (srmhd_phys.hpp).  Update stages: 0 =
// L(U) only, 1..3 = SSP-RK3 stages, 4 = second (last) SSP-RK2 stage; ho:
// sixth-order DER.
// The x and the y faces in one pass (primitives staged once per tile).
template <typename TS>
void launch_flux_xy(const FluxArgs<TS>& ax, const FluxArgs<TS>& ay, bool stats, int rec,
                    hipStream_t s);
// The z faces (cfl: also the CFL maximum of the first stage).
template <typename TS>
void launch_flux_z(const FluxArgs<TS>& a, bool cfl, bool stats, int rec, hipStream_t s);
template <typename TS>
void launch_uct(const Uct3Args<TS>& a, int k, int rec, hipStream_t s);  // orientation E_k
template <typename TS>
void launch_update(int stage, const UpdArgs<TS>& a, bool ho, hipStream_t s);
// amax_in (device, or null: the running maximum) is the speed maximum dt
// takes.
// The update of stage 1 or 2 fused with the inversion of its output
// (periodic box, face-average INT, guess 0 or 2); p.cons/p.bf are not read.
template <typename TS>
void launch_update_c2p(int stage, const UpdArgs<TS>& a, const C2PArgs& p, bool stats,
                       hipStream_t s);
void launch_dt(DevScalars* sc, double cfl, double dt_fixed, const double* amax_in, hipStream_t s);
void launch_local_amax(const DevScalars* sc, double* out, hipStream_t s);
// Ghost-plane exchange of a z-slab: 9 arrays, planes [z0, z0 + G) each, to
// (pack) or from (unpack) buf[a * G * plane + ...].
struct HaloArgs {
  double* a[9];
  double* buf;
  long long plane;  // nx * ny
  int z0, G;
};
void launch_halo(const HaloArgs& h, bool pack, hipStream_t s);
void launch_zero_u64(unsigned long long* p, size_t n, hipStream_t s);
void launch_fill_f64(double* p, size_t n, double v, hipStream_t s);
void launch_set_time(DevScalars* sc, double t, long long step, hipStream_t s);
void launch_reduce(const ReduceArgs& a, hipStream_t s);
int reduce_blocks(const GridDims& g);

}  // namespace srmhd
