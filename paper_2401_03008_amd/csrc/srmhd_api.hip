// srmhd_api.hip -- the C ABI of libsrmhd (declared in include/srmhd.h):
// configuration checks, carving of the caller's work buffer, and the launch
// sequence of the SSP-RK stages.  Host code only; every launch goes to the
// caller's stream.
#include "srmhd.h"
#include "srmhd_kernels.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace srmhd;

struct srmhd_ctx {
  srmhd_config cfg;
  srmhd_buffers buf;
  hipStream_t stream;
  int device;
  GridDims g;
  long long ncell;  // cells of every grid array (ghost planes included)
  bool mixed;
  bool initialized;
  // stage sequence of srmhd_stage_begin/_end: the next stage to begin
  // (1-based) and whether its first half ran
  int next_stage;
  bool half_done;
  // the primitives in the work buffer (and W) are the inversion of the
  // current state, done by the last stage's fused update
  bool prims_ready;
  // every cell's W comes from a completed inversion (so it is usable: the
  // learned guess of SRMHD_GUESS_MLP has nothing to seed)
  bool w_complete;
  DevScalars* sc;
  unsigned long long* counters;
  double* partial;
  double* ureg[8];  // RK stage register (U1, then U2; U2's face B in ureg2b)
  double* ureg2b[3];  // face B of U2 (stage 2 must not overwrite U1's B in place)
  double* prim64[8];
  float* prim32[8];
  float* bf32[3];  // mixed form: FP32 copies of the stage's face B (REC operands)
  void* fhat[3][5];
  void* apm[3][2];
  void* fv[3][4];
  double* edge[3];

  std::string err;
  // per-kernel event timing
  bool timing;
  std::vector<hipEvent_t> ev;      // pool, pairs (start, stop)
  std::vector<int> ev_class;       // class of each pair in flight
  int ev_used;
  double kms[SRMHD_NKCLASS];
  long kcount[SRMHD_NKCLASS];
  // learned guess
  bool mlp_set;
  MlpDev mlp;
};

static std::string g_create_error;

namespace srmhd {
// Failure message of a call without a context (srmhd_last_error(NULL)).
void set_call_error(const char* msg) { g_create_error = msg; }
}  // namespace srmhd

#ifndef SRMHD_BUILD_ID
#define SRMHD_BUILD_ID "unknown"
#endif

namespace {

int fail(srmhd_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return code;
}

int hip_check(srmhd_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return SRMHD_OK;
  return fail(c, SRMHD_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int check_launch(srmhd_ctx* c, const char* what) {
  return hip_check(c, hipGetLastError(), what);
}

constexpr int kEventPairs = 2048;

int drain_events(srmhd_ctx* c) {
  if (c->ev_used == 0) return SRMHD_OK;
  int rc = hip_check(c, hipStreamSynchronize(c->stream), "stream sync (timing)");
  if (rc != SRMHD_OK) return rc;
  for (int n = 0; n < c->ev_used; ++n) {
    float ms = 0.f;
    rc = hip_check(c, hipEventElapsedTime(&ms, c->ev[2 * n], c->ev[2 * n + 1]), "event time");
    if (rc != SRMHD_OK) return rc;
    c->kms[c->ev_class[n]] += ms;
    c->kcount[c->ev_class[n]] += 1;
  }
  c->ev_used = 0;
  return SRMHD_OK;
}

// Scoped start/stop events around one launch of class k (no-op if timing off).
struct KTimer {
  srmhd_ctx* c;
  int pair;
  KTimer(srmhd_ctx* cc, int k) : c(cc), pair(-1) {
    if (!c->timing) return;
    if (c->ev_used == kEventPairs) drain_events(c);
    pair = c->ev_used++;
    c->ev_class[pair] = k;
    (void)hipEventRecord(c->ev[2 * pair], c->stream);
  }
  ~KTimer() {
    if (pair >= 0) (void)hipEventRecord(c->ev[2 * pair + 1], c->stream);
  }
};

// Planes of every grid array: the interior plus the ghost planes of a slab.
int planes_of(const srmhd_config* c) { return c->nz + 2 * c->ghost_z; }

std::string validate(const srmhd_config* c) {
  if (!c) return "config is NULL";
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return "nx, ny, nz must each be >= 1";
  if (c->ghost_z < 0 || c->ghost_z > 64) return "ghost_z must be in 0..64";
  if (c->ghost_z > 0) {
    const int need = c->high_order ? 8 : 4;
    if (c->ghost_z < need)
      return c->high_order ? "ghost_z must be >= 8 with high_order" : "ghost_z must be >= 4";
    if (c->nz < c->ghost_z) return "a slab needs nz >= ghost_z interior planes";
  }
  const long long nzp = planes_of(c);
  if ((long long)c->nx * c->ny * nzp >= (1LL << 31)) return "nx*ny*nz must be < 2^31";
  // every launch is a 1D grid of tiles (at most 64 x 8 x 8 cells, tile rows
  // padded to groups of 8): its thread count must stay below 2^32
  if ((double)(c->nx + 63) * (c->ny + 8) * (nzp + 8) + 32768.0 * ((c->nx + 63) / 64) >=
      4294967295.0)
    return "box too large for one launch grid";
  if (!(c->lx > 0 && c->ly > 0 && c->lz > 0)) return "box lengths must be > 0";
  if (!(c->gamma_ad > 1.0 && c->gamma_ad <= 2.0)) return "gamma_ad must be in (1, 2]";
  if (!(c->dt_fixed > 0.0) && !(c->cfl > 0.0 && c->cfl <= 1.0))
    return "cfl must be in (0, 1] unless dt_fixed > 0";
  if (!(c->dt_fixed >= 0.0) || !std::isfinite(c->dt_fixed)) return "dt_fixed must be >= 0";
  if (c->riemann != SRMHD_HLL && c->riemann != SRMHD_LLF) return "riemann must be HLL or LLF";
  if (c->precision != SRMHD_FP64 && c->precision != SRMHD_MIXED) return "bad precision";
  if (c->guess != SRMHD_GUESS_PREV && c->guess != SRMHD_GUESS_COLD &&
      c->guess != SRMHD_GUESS_MLP && c->guess != SRMHD_GUESS_MLP_ALL)
    return "bad guess mode";
  if (c->newton_maxit < 1 || c->newton_maxit > 1000) return "newton_maxit must be in 1..1000";
  if (!(c->newton_tol > 0.0 && c->newton_tol < 1e-3)) return "newton_tol must be in (0, 1e-3)";
  if (!(c->pfloor >= 0.0 && c->pfloor < 1.0)) return "pfloor must be in [0, 1)";
  if (c->recon != SRMHD_REC_MP5 && c->recon != SRMHD_REC_MC) return "recon must be MP5 or MC";
  if (c->time_order != 2 && c->time_order != 3) return "time_order must be 2 or 3";
  if (c->high_order != 0 && c->high_order != 1) return "high_order must be 0 or 1";
  if (c->high_order && c->recon != SRMHD_REC_MP5) return "high_order needs MP5 reconstruction";
  return "";
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Work layout: scalars | counters | reduce partials | arrays.
struct Layout {
  size_t off_sc, off_cnt, off_part, off_arr, total;
  size_t arr_bytes64, arr_bytes32;
  int n64, n32;  // number of FP64 / FP32 arrays
};

Layout layout_of(const srmhd_config* c) {
  Layout L;
  const size_t n = (size_t)c->nx * c->ny * planes_of(c);
  L.off_sc = 0;
  L.off_cnt = align_up(sizeof(DevScalars));
  L.off_part = L.off_cnt + align_up(sizeof(unsigned long long) * kReplicas * CNT_N);
  L.off_arr = L.off_part + align_up(sizeof(double) * 9 * 1024);
  L.arr_bytes64 = align_up(n * sizeof(double));
  L.arr_bytes32 = align_up(n * sizeof(float));
  const bool mixed = c->precision == SRMHD_MIXED;
  // RK register (8 + 3 for U2's face B) + edge E (3) always FP64; prims FP64
  // (8) or FP32 (8, plus FP32 copies of the 3 face B); faces (15 fluxes + 6
  // speeds + 12 velocity states) in the flux precision.
  L.n64 = 8 + 3 + 3 + (mixed ? 0 : 8 + 33);
  L.n32 = mixed ? 8 + 3 + 33 : 0;
  L.total = L.off_arr + L.n64 * L.arr_bytes64 + L.n32 * L.arr_bytes32;
  return L;
}

// The stage's input state: the caller's arrays (U^n) in stage 1 and for the
// stand-alone operator, the work register (U1, U2) in stages 2 and 3.
struct StageState {
  const double* cons[5];
  double* bf[3];
};

StageState stage_state(srmhd_ctx* c, int stage) {
  StageState s;
  const bool reg = stage >= 2;
  for (int n = 0; n < 5; ++n) s.cons[n] = reg ? c->ureg[n] : c->buf.cons[n];
  for (int d = 0; d < 3; ++d)
    s.bf[d] = stage == 3 ? c->ureg2b[d] : (reg ? c->ureg[5 + d] : c->buf.bface[d]);
  return s;
}

// REC kernel of the configuration: MC, or MP5 (point-value form with HO).
int rec_kind(const srmhd_ctx* c) {
  if (c->cfg.recon == SRMHD_REC_MC) return kRecMc;
  return c->cfg.high_order ? kRecMp5Point : kRecMp5;
}

template <typename TS>
void stage_flux(srmhd_ctx* c, const StageState& st, bool cfl) {
  const bool stats = c->cfg.collect_stats != 0;
  FluxArgs<TS> args[3];
  for (int d = 0; d < 3; ++d) {
    FluxArgs<TS>& a = args[d];
    a.g = c->g;
    for (int n = 0; n < 8; ++n)
      a.prim[n] = c->mixed ? (const TS*)c->prim32[n] : (const TS*)c->prim64[n];
    a.bn = c->mixed ? (const TS*)c->bf32[d] : (const TS*)st.bf[d];
    for (int n = 0; n < 5; ++n) a.fhat[n] = (TS*)c->fhat[d][n];
    a.ap = (TS*)c->apm[d][0];
    a.am = (TS*)c->apm[d][1];
    for (int n = 0; n < 4; ++n) a.fv[n] = (TS*)c->fv[d][n];
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    a.apm_other[0] = (const TS*)c->apm[t1][0];
    a.apm_other[1] = (const TS*)c->apm[t1][1];
    a.apm_other[2] = (const TS*)c->apm[t2][0];
    a.apm_other[3] = (const TS*)c->apm[t2][1];
    a.amax_bits = &c->sc->amax_bits;
    a.gam = c->cfg.gamma_ad;
    a.riemann = c->cfg.riemann;
    a.counters = c->counters;
  }
  {
    KTimer kt(c, 1);
    launch_flux_xy<TS>(args[0], args[1], stats, rec_kind(c), c->stream);
  }
  KTimer kt(c, 2);
  launch_flux_z<TS>(args[2], cfl, stats, rec_kind(c), c->stream);
}

C2PArgs c2p_args(srmhd_ctx* c, const StageState& st, double* const* prim64, float* const* prim32,
                 int guess);
int guess_code(const srmhd_ctx* c);

template <typename TS>
void stage_uct_update(srmhd_ctx* c, const StageState& st, int stage, double* const* rhs_out,
                      bool fuse) {
  {
    Uct3Args<TS> a;
    a.g = c->g;
    for (int d = 0; d < 3; ++d) {
      for (int n = 0; n < 4; ++n) a.fv[d][n] = (const TS*)c->fv[d][n];
      a.ap[d] = (const TS*)c->apm[d][0];
      a.am[d] = (const TS*)c->apm[d][1];
      a.bf[d] = c->mixed ? (const TS*)c->bf32[d] : (const TS*)st.bf[d];
      a.e[d] = c->edge[d];
    }
    for (int k = 0; k < 3; ++k) {
      KTimer kt(c, 3 + k);
      launch_uct<TS>(a, k, rec_kind(c), c->stream);
    }
  }
  UpdArgs<TS> u;
  u.g = c->g;
  for (int d = 0; d < 3; ++d)
    for (int n = 0; n < 5; ++n) u.fhat[d][n] = (const TS*)c->fhat[d][n];
  for (int k = 0; k < 3; ++k) u.e[k] = c->edge[k];
  double* state[8];
  for (int n = 0; n < 5; ++n) state[n] = c->buf.cons[n];
  for (int d = 0; d < 3; ++d) state[5 + d] = c->buf.bface[d];
  for (int n = 0; n < 8; ++n) {
    u.ucur[n] = n < 5 ? st.cons[n] : st.bf[n - 5];
    u.u0[n] = state[n];
    // the last stage writes U^{n+1}; stage 2 keeps U1's face B intact
    u.uout[n] = stage >= 3 ? state[n] : (stage == 2 && n >= 5 ? c->ureg2b[n - 5] : c->ureg[n]);
    u.rhs_out[n] = rhs_out ? rhs_out[n] : nullptr;
  }
  u.sc = c->sc;
  if (fuse) {
    // the next stage's inversion of this stage's output
    const C2PArgs p = c2p_args(c, StageState{}, c->mixed ? nullptr : c->prim64,
                               c->mixed ? c->prim32 : nullptr, guess_code(c));
    KTimer kt(c, 8);
    launch_update_c2p<TS>(stage, u, p, c->cfg.collect_stats != 0, c->stream);
  } else {
    KTimer kt(c, 6);
    launch_update<TS>(stage, u, c->cfg.high_order != 0, c->stream);
  }
}

C2PArgs c2p_args(srmhd_ctx* c, const StageState& st, double* const* prim64, float* const* prim32,
                 int guess) {
  C2PArgs a;
  a.g = c->g;
  for (int n = 0; n < 5; ++n) a.cons[n] = st.cons[n];
  for (int d = 0; d < 3; ++d) a.bf[d] = st.bf[d];
  a.W = c->buf.guess_w;
  for (int n = 0; n < 8; ++n) {
    a.prim64[n] = prim64 ? prim64[n] : nullptr;
    a.prim32[n] = prim32 ? prim32[n] : nullptr;
  }
  // the FP32 face B for the mixed form's REC, with the stage's FP32 primitives
  for (int d = 0; d < 3; ++d) a.bf32[d] = prim32 ? c->bf32[d] : nullptr;
  a.gam = c->cfg.gamma_ad;
  a.tol = c->cfg.newton_tol;
  a.pfloor = c->cfg.pfloor;
  a.maxit = c->cfg.newton_maxit;
  a.guess = guess;
  a.ho = c->cfg.high_order;
  a.mlp = c->mlp;
  a.counters = c->counters;
  a.err = &c->sc->err;
  a.mlp_out = nullptr;
  a.mlp_w0 = nullptr;
  return a;
}

void launch_c2p_into(srmhd_ctx* c, const StageState& st, double* const* prim64,
                     float* const* prim32, int guess) {
  const C2PArgs a = c2p_args(c, st, prim64, prim32, guess);
  KTimer kt(c, 0);
  launch_c2p(a, c->cfg.collect_stats != 0, c->stream);
  c->w_complete = true;
}

// Device-to-device copy of one grid array on the context's stream (nothing
// to do when source and destination are the same array).
int copy_grid(srmhd_ctx* c, double* dst, const double* src, const char* what) {
  if (dst == src) return SRMHD_OK;
  return hip_check(c, hipMemcpyAsync(dst, src, (size_t)c->ncell * sizeof(double),
                                     hipMemcpyDeviceToDevice, c->stream), what);
}

// The kernels' guess code of the next inversion: the SRMHD_GUESS_* value
// (see k_c2p), except that SRMHD_GUESS_MLP runs as the previous-W guess once
// every cell has a W from a completed inversion (the network would seed no
// cell).
int guess_code(const srmhd_ctx* c) {
  if (c->cfg.guess == SRMHD_GUESS_MLP && c->w_complete) return SRMHD_GUESS_PREV;
  return c->cfg.guess;
}

bool learned_guess(const srmhd_ctx* c) {
  return c->cfg.guess == SRMHD_GUESS_MLP || c->cfg.guess == SRMHD_GUESS_MLP_ALL;
}

// Whether a stage's update also inverts its output for the next stage
// (k_update_c2p): periodic boxes, face-average INT, previous-W or cold
// guess.  The sequence of inversions (inputs and W chain) is the same as
// with a separate inversion at the start of each stage.
bool fused_update(const srmhd_ctx* c) {
  const int g = guess_code(c);
  return c->cfg.ghost_z == 0 && !c->cfg.high_order &&
         (g == SRMHD_GUESS_PREV || g == SRMHD_GUESS_COLD);
}

// First half of a stage (1..3 of SSP-RK3; 1 and 4 of SSP-RK2; 0 = L(U)):
// INT + inversion (unless the previous stage's update already inverted this
// state), REC + face fluxes and speeds (and the running CFL maximum in
// stage 1 and stage 0).
void stage_first_half(srmhd_ctx* c, int stage) {
  const int guess = guess_code(c);
  const StageState st = stage_state(c, stage);
  if (!(c->prims_ready && fused_update(c) && stage >= 1)) {
    if (c->mixed)
      launch_c2p_into(c, st, nullptr, c->prim32, guess);
    else
      launch_c2p_into(c, st, c->prim64, nullptr, guess);
  }
  c->prims_ready = false;
  const bool cfl = stage <= 1;
  if (c->mixed) stage_flux<float>(c, st, cfl);
  else stage_flux<double>(c, st, cfl);
}

// Second half: dt in stage 1 (from amax_in, device, or the running maximum),
// then UCT, DER and the update.
void stage_second_half(srmhd_ctx* c, int stage, double* const* rhs_out, const double* amax_in) {
  const StageState st = stage_state(c, stage);
  if (stage == 1) {
    KTimer kt(c, 7);
    launch_dt(c->sc, c->cfg.cfl, c->cfg.dt_fixed, amax_in, c->stream);
  }
  // stages 1 and 2 (the last stage writes into U^n's arrays, which its
  // neighbours' re-derived face B would still read)
  const bool fuse = (stage == 1 || stage == 2) && !rhs_out && fused_update(c);
  if (c->mixed) stage_uct_update<float>(c, st, stage, rhs_out, fuse);
  else stage_uct_update<double>(c, st, stage, rhs_out, fuse);
  c->prims_ready = fuse;
  if (fuse) c->w_complete = true;
}

void run_stage(srmhd_ctx* c, int stage, double* const* rhs_out) {
  stage_first_half(c, stage);
  stage_second_half(c, stage, rhs_out, nullptr);
}

// Internal code of stage s (1-based) of a step: SSP-RK3 1, 2, 3; SSP-RK2 1, 4.
int stage_code(const srmhd_ctx* c, int s) { return (c->cfg.time_order == 2 && s == 2) ? 4 : s; }
int stages_per_step(const srmhd_ctx* c) { return c->cfg.time_order == 2 ? 2 : 3; }

// SRMHD_E_STATE while a step driven by srmhd_stage_begin/_end is under way.
int check_between_steps(srmhd_ctx* c, const char* what) {
  if (c->next_stage != 1 || c->half_done)
    return fail(c, SRMHD_E_STATE,
                std::string(what) + " while a step is under way (finish its stages first)");
  return SRMHD_OK;
}

__global__ void k_take_amax(srmhd::DevScalars* sc, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *out = __longlong_as_double((long long)sc->amax_bits);
    sc->amax_bits = 0ull;
  }
}

}  // namespace

extern "C" {

int srmhd_config_default(srmhd_config* cfg) {
  if (!cfg) return SRMHD_E_INVAL;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->nx = cfg->ny = cfg->nz = 32;
  cfg->lx = cfg->ly = cfg->lz = 1.0;
  cfg->gamma_ad = 4.0 / 3.0;
  cfg->cfl = 0.5;
  cfg->dt_fixed = 0.0;
  cfg->riemann = SRMHD_HLL;
  cfg->precision = SRMHD_FP64;
  cfg->guess = SRMHD_GUESS_PREV;
  cfg->newton_maxit = 50;
  cfg->newton_tol = 1e-14;
  cfg->pfloor = 0.0;
  cfg->collect_stats = 1;
  cfg->recon = SRMHD_REC_MP5;
  cfg->time_order = 3;
  cfg->high_order = 0;
  cfg->ghost_z = 0;
  return SRMHD_OK;
}

int srmhd_work_bytes(const srmhd_config* cfg, size_t* bytes) {
  const std::string v = validate(cfg);
  if (!v.empty()) return fail(nullptr, SRMHD_E_INVAL, v);
  if (!bytes) return fail(nullptr, SRMHD_E_INVAL, "bytes is NULL");
  *bytes = layout_of(cfg).total;
  return SRMHD_OK;
}

int srmhd_create(const srmhd_config* cfg, const srmhd_buffers* buf, void* stream,
                 srmhd_ctx** out) {
  if (!out) return fail(nullptr, SRMHD_E_INVAL, "out is NULL");
  *out = nullptr;
  const std::string v = validate(cfg);
  if (!v.empty()) return fail(nullptr, SRMHD_E_INVAL, v);
  if (!buf) return fail(nullptr, SRMHD_E_INVAL, "buffers is NULL");
  for (int n = 0; n < 5; ++n)
    if (!buf->cons[n]) return fail(nullptr, SRMHD_E_INVAL, "cons pointer is NULL");
  for (int d = 0; d < 3; ++d)
    if (!buf->bface[d]) return fail(nullptr, SRMHD_E_INVAL, "bface pointer is NULL");
  if (!buf->guess_w) return fail(nullptr, SRMHD_E_INVAL, "guess_w is NULL");
  const Layout L = layout_of(cfg);
  if (!buf->work || buf->work_bytes < L.total)
    return fail(nullptr, SRMHD_E_INVAL, "work buffer missing or smaller than srmhd_work_bytes");
  if (((uintptr_t)buf->work) % kAlign != 0)
    return fail(nullptr, SRMHD_E_INVAL, "work buffer must be 256-byte aligned");

  srmhd_ctx* c = new srmhd_ctx();
  c->cfg = *cfg;
  c->buf = *buf;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, SRMHD_E_HIP, "hipGetDevice failed");
  }
  c->g.nx = cfg->nx;
  c->g.ny = cfg->ny;
  c->g.nz = planes_of(cfg);
  c->g.inv_dx[0] = cfg->nx / cfg->lx;
  c->g.inv_dx[1] = cfg->ny / cfg->ly;
  c->g.inv_dx[2] = cfg->nz / cfg->lz;
  // interior planes, and the planes whose primitives the interior's fluxes
  // read (3 beyond each edge; 5 with the HO differences)
  const int G = cfg->ghost_z, reach = G > 0 ? (cfg->high_order ? 5 : 3) : 0;
  c->g.zlo = G;
  c->g.zhi = G + cfg->nz;
  c->g.zplo = G - reach;
  c->g.zphi = G + cfg->nz + reach;
  c->ncell = (long long)cfg->nx * cfg->ny * c->g.nz;
  c->next_stage = 1;
  c->half_done = false;
  c->prims_ready = false;
  c->w_complete = false;
  c->mixed = cfg->precision == SRMHD_MIXED;
  c->initialized = false;
  c->timing = false;
  c->ev_used = 0;
  c->mlp_set = false;
  std::memset(&c->mlp, 0, sizeof(c->mlp));
  for (int k = 0; k < SRMHD_NKCLASS; ++k) {
    c->kms[k] = 0.0;
    c->kcount[k] = 0;
  }
  char* w = (char*)buf->work;
  c->sc = (DevScalars*)(w + L.off_sc);
  c->counters = (unsigned long long*)(w + L.off_cnt);
  c->partial = (double*)(w + L.off_part);
  char* p = w + L.off_arr;
  auto take64 = [&]() { double* r = (double*)p; p += L.arr_bytes64; return r; };
  auto take32 = [&]() { float* r = (float*)p; p += L.arr_bytes32; return r; };
  auto takeT = [&]() -> void* { return c->mixed ? (void*)take32() : (void*)take64(); };
  for (int n = 0; n < 8; ++n) c->ureg[n] = take64();
  for (int k = 0; k < 3; ++k) c->edge[k] = take64();
  for (int d = 0; d < 3; ++d) c->ureg2b[d] = take64();
  for (int n = 0; n < 8; ++n) {
    c->prim64[n] = c->mixed ? nullptr : take64();
    c->prim32[n] = c->mixed ? take32() : nullptr;
  }
  for (int d = 0; d < 3; ++d) c->bf32[d] = c->mixed ? take32() : nullptr;
  for (int d = 0; d < 3; ++d) {
    for (int n = 0; n < 5; ++n) c->fhat[d][n] = takeT();
    for (int n = 0; n < 2; ++n) c->apm[d][n] = takeT();
    for (int n = 0; n < 4; ++n) c->fv[d][n] = takeT();
  }
  // clear scalars and counters (a fill kernel, no memset node)
  launch_zero_u64((unsigned long long*)w, L.off_part / sizeof(unsigned long long), c->stream);
  const int rc = check_launch(c, "clearing work scalars");
  if (rc != SRMHD_OK) {
    g_create_error = c->err;
    delete c;
    return rc;
  }
  *out = c;
  return SRMHD_OK;
}

int srmhd_init_from_prims(srmhd_ctx* c, const double* const prim5[5], const double* const bface[3]) {
  if (!c) return SRMHD_E_INVAL;
  if (check_between_steps(c, "init_from_prims") != SRMHD_OK) return SRMHD_E_STATE;
  if (!prim5 || !bface) return fail(c, SRMHD_E_INVAL, "prim5/bface is NULL");
  for (int n = 0; n < 5; ++n)
    if (!prim5[n]) return fail(c, SRMHD_E_INVAL, "prim5 entry is NULL");
  for (int d = 0; d < 3; ++d)
    if (!bface[d]) return fail(c, SRMHD_E_INVAL, "bface entry is NULL");
  InitArgs a;
  a.g = c->g;
  a.ho = c->cfg.high_order;
  for (int n = 0; n < 5; ++n) {
    a.prim5[n] = prim5[n];
    a.cons[n] = c->buf.cons[n];
  }
  for (int d = 0; d < 3; ++d) {
    a.bf_in[d] = bface[d];
    a.bf[d] = c->buf.bface[d];
  }
  a.W = c->buf.guess_w;
  a.gam = c->cfg.gamma_ad;
  // state arrays may alias the inputs only for bface (copied in place)
  launch_init(a, c->stream);
  const Layout L = layout_of(&c->cfg);
  launch_zero_u64((unsigned long long*)c->buf.work, L.off_part / sizeof(unsigned long long),
                  c->stream);
  const int rc = check_launch(c, "init_from_prims");
  if (rc == SRMHD_OK) c->initialized = true;
  c->prims_ready = false;
  c->w_complete = true;  // W = rho h Gamma^2 of the initial data
  return rc;
}

int srmhd_step(srmhd_ctx* c, int nsteps) {
  if (!c) return SRMHD_E_INVAL;
  if (!c->initialized) return fail(c, SRMHD_E_STATE, "step before init_from_prims");
  if (nsteps < 0) return fail(c, SRMHD_E_INVAL, "nsteps < 0");
  if (learned_guess(c) && !c->mlp_set)
    return fail(c, SRMHD_E_STATE, "learned guess selected but no network set");
  if (c->cfg.ghost_z > 0)
    return fail(c, SRMHD_E_STATE,
                "a slab context (ghost_z > 0) steps through srmhd_stage_begin/_end with a "
                "ghost exchange after every stage");
  if (check_between_steps(c, "step") != SRMHD_OK) return SRMHD_E_STATE;
  for (int s = 0; s < nsteps; ++s) {
    run_stage(c, 1, nullptr);
    if (c->cfg.time_order == 2) {
      run_stage(c, 4, nullptr);
    } else {
      run_stage(c, 2, nullptr);
      run_stage(c, 3, nullptr);
    }
  }
  return check_launch(c, "step");
}

int srmhd_rhs(srmhd_ctx* c, double* const rhs[8], double* amax_dev) {
  if (!c) return SRMHD_E_INVAL;
  if (!c->initialized) return fail(c, SRMHD_E_STATE, "rhs before init_from_prims");
  if (check_between_steps(c, "rhs") != SRMHD_OK) return SRMHD_E_STATE;
  if (!rhs || !amax_dev) return fail(c, SRMHD_E_INVAL, "rhs/amax is NULL");
  if (learned_guess(c) && !c->mlp_set)
    return fail(c, SRMHD_E_STATE, "learned guess selected but no network set");
  for (int n = 0; n < 8; ++n)
    if (!rhs[n]) return fail(c, SRMHD_E_INVAL, "rhs entry is NULL");
  // the running CFL maximum belongs to the step sequence: clear, use, clear
  hipLaunchKernelGGL(k_take_amax, dim3(1), dim3(64), 0, c->stream, c->sc, amax_dev);
  run_stage(c, 0, rhs);
  hipLaunchKernelGGL(k_take_amax, dim3(1), dim3(64), 0, c->stream, c->sc, amax_dev);
  return check_launch(c, "rhs");
}

int srmhd_get_primitives(srmhd_ctx* c, double* const prim[8]) {
  if (!c) return SRMHD_E_INVAL;
  if (!c->initialized) return fail(c, SRMHD_E_STATE, "get_primitives before init_from_prims");
  if (check_between_steps(c, "get_primitives") != SRMHD_OK) return SRMHD_E_STATE;
  if (!prim) return fail(c, SRMHD_E_INVAL, "prim is NULL");
  for (int n = 0; n < 8; ++n)
    if (!prim[n]) return fail(c, SRMHD_E_INVAL, "prim entry is NULL");
  if (learned_guess(c) && !c->mlp_set)
    return fail(c, SRMHD_E_STATE, "learned guess selected but no network set");
  launch_c2p_into(c, stage_state(c, 0), prim, nullptr, guess_code(c));
  c->prims_ready = false;  // W moved: the next stage inverts afresh
  return check_launch(c, "get_primitives");
}

int srmhd_get_state(srmhd_ctx* c, double* const cons[5], double* const bface[3], double* w,
                    double* t, long* step) {
  if (!c) return SRMHD_E_INVAL;
  if (!c->initialized) return fail(c, SRMHD_E_STATE, "get_state before the state is set");
  if (check_between_steps(c, "get_state") != SRMHD_OK) return SRMHD_E_STATE;
  if (cons)
    for (int n = 0; n < 5; ++n)
      if (!cons[n]) return fail(c, SRMHD_E_INVAL, "cons entry is NULL");
  if (bface)
    for (int d = 0; d < 3; ++d)
      if (!bface[d]) return fail(c, SRMHD_E_INVAL, "bface entry is NULL");
  int rc = SRMHD_OK;
  for (int n = 0; cons && n < 5 && rc == SRMHD_OK; ++n)
    rc = copy_grid(c, cons[n], c->buf.cons[n], "get_state copy");
  for (int d = 0; bface && d < 3 && rc == SRMHD_OK; ++d)
    rc = copy_grid(c, bface[d], c->buf.bface[d], "get_state copy");
  if (rc == SRMHD_OK && w)
    rc = copy_grid(c, w, c->buf.guess_w, "get_state copy");
  if (rc != SRMHD_OK) return rc;
  double tt = 0.0, dt = 0.0;
  long st = 0;
  rc = srmhd_get_time(c, &tt, &st, &dt);  // syncs: the copies are complete
  if (rc != SRMHD_OK) return rc;
  if (t) *t = tt;
  if (step) *step = st;
  return SRMHD_OK;
}

int srmhd_set_state(srmhd_ctx* c, const double* const cons[5], const double* const bface[3],
                    const double* w, double t, long step) {
  if (!c) return SRMHD_E_INVAL;
  if (check_between_steps(c, "set_state") != SRMHD_OK) return SRMHD_E_STATE;
  if (!cons || !bface) return fail(c, SRMHD_E_INVAL, "cons/bface is NULL");
  for (int n = 0; n < 5; ++n)
    if (!cons[n]) return fail(c, SRMHD_E_INVAL, "cons entry is NULL");
  for (int d = 0; d < 3; ++d)
    if (!bface[d]) return fail(c, SRMHD_E_INVAL, "bface entry is NULL");
  if (!std::isfinite(t) || step < 0) return fail(c, SRMHD_E_INVAL, "bad time or step");
  int rc = SRMHD_OK;
  for (int n = 0; n < 5 && rc == SRMHD_OK; ++n)
    rc = copy_grid(c, c->buf.cons[n], cons[n], "set_state copy");
  for (int d = 0; d < 3 && rc == SRMHD_OK; ++d)
    rc = copy_grid(c, c->buf.bface[d], bface[d], "set_state copy");
  if (rc != SRMHD_OK) return rc;
  if (w) {
    rc = copy_grid(c, c->buf.guess_w, w, "set_state copy");
    if (rc != SRMHD_OK) return rc;
  } else {
    // no previous W: every guess is unusable, so the next inversion starts
    // from the learned guess (learned form) or from U
    launch_fill_f64(c->buf.guess_w, (size_t)c->ncell, -1.0, c->stream);
  }
  // scalars (running max, dt, error word) and counters start afresh
  const Layout L = layout_of(&c->cfg);
  launch_zero_u64((unsigned long long*)c->buf.work, L.off_part / sizeof(unsigned long long),
                  c->stream);
  launch_set_time(c->sc, t, step, c->stream);
  rc = check_launch(c, "set_state");
  if (rc == SRMHD_OK) c->initialized = true;
  c->prims_ready = false;
  c->w_complete = false;  // a given W is checked cell by cell at the next inversion
  return rc;
}

int srmhd_mlp_guess(srmhd_ctx* c, float* out, double* w0) {
  if (!c) return SRMHD_E_INVAL;
  if (!c->initialized) return fail(c, SRMHD_E_STATE, "mlp_guess before the state is set");
  if (check_between_steps(c, "mlp_guess") != SRMHD_OK) return SRMHD_E_STATE;
  if (!c->mlp_set) return fail(c, SRMHD_E_STATE, "mlp_guess needs srmhd_set_mlp first");
  if (!out) return fail(c, SRMHD_E_INVAL, "out is NULL");
  C2PArgs a;
  std::memset(&a, 0, sizeof(a));
  const StageState st = stage_state(c, 0);
  a.g = c->g;
  for (int n = 0; n < 5; ++n) a.cons[n] = st.cons[n];
  for (int d = 0; d < 3; ++d) a.bf[d] = st.bf[d];
  a.W = c->buf.guess_w;
  a.gam = c->cfg.gamma_ad;
  a.tol = c->cfg.newton_tol;
  a.pfloor = c->cfg.pfloor;
  a.maxit = c->cfg.newton_maxit;
  a.guess = 1;
  a.ho = c->cfg.high_order;
  a.mlp = c->mlp;
  a.counters = c->counters;
  a.err = &c->sc->err;
  a.mlp_out = out;
  a.mlp_w0 = w0;
  launch_c2p(a, false, c->stream);
  return check_launch(c, "mlp_guess");
}

int srmhd_stage_begin(srmhd_ctx* c, int stage) {
  if (!c) return SRMHD_E_INVAL;
  if (!c->initialized) return fail(c, SRMHD_E_STATE, "stage_begin before the state is set");
  if (learned_guess(c) && !c->mlp_set)
    return fail(c, SRMHD_E_STATE, "learned guess selected but no network set");
  if (stage < 1 || stage > stages_per_step(c))
    return fail(c, SRMHD_E_INVAL, "stage must be 1..3 (SSP-RK3) or 1..2 (SSP-RK2)");
  if (c->half_done || stage != c->next_stage)
    return fail(c, SRMHD_E_STATE, "stage_begin out of order (expected stage " +
                                      std::to_string(c->next_stage) +
                                      (c->half_done ? "'s end" : "") + ")");
  stage_first_half(c, stage_code(c, stage));
  c->half_done = true;
  return check_launch(c, "stage_begin");
}

int srmhd_local_amax(srmhd_ctx* c, double* amax_dev) {
  if (!c) return SRMHD_E_INVAL;
  if (!amax_dev) return fail(c, SRMHD_E_INVAL, "amax_dev is NULL");
  if (!(c->half_done && c->next_stage == 1))
    return fail(c, SRMHD_E_STATE, "local_amax needs stage_begin(1) first");
  launch_local_amax(c->sc, amax_dev, c->stream);
  return check_launch(c, "local_amax");
}

int srmhd_stage_end(srmhd_ctx* c, int stage, const double* amax_dev) {
  if (!c) return SRMHD_E_INVAL;
  if (!c->half_done || stage != c->next_stage)
    return fail(c, SRMHD_E_STATE, "stage_end without the matching stage_begin");
  const int code = stage_code(c, stage);
  stage_second_half(c, code, nullptr, stage == 1 ? amax_dev : nullptr);
  c->half_done = false;
  const bool last = stage == stages_per_step(c);
  c->next_stage = last ? 1 : stage + 1;
  return check_launch(c, "stage_end");
}

int srmhd_halo_count(const srmhd_ctx* c, size_t* n) {
  if (!c || !n) return SRMHD_E_INVAL;
  *n = (size_t)9 * c->cfg.ghost_z * c->cfg.nx * c->cfg.ny;
  return SRMHD_OK;
}

namespace {
int halo_copy(srmhd_ctx* c, int side, double* buf, bool pack) {
  if (!c) return SRMHD_E_INVAL;
  const char* what = pack ? "halo_pack" : "halo_unpack";
  if (c->cfg.ghost_z == 0)
    return fail(c, SRMHD_E_STATE, std::string(what) + " on a context without ghost planes");
  if (!c->initialized) return fail(c, SRMHD_E_STATE, std::string(what) + " before the state is set");
  if (c->half_done)
    return fail(c, SRMHD_E_STATE, std::string(what) + " between the halves of a stage");
  if (side != 0 && side != 1) return fail(c, SRMHD_E_INVAL, "side must be 0 (below) or 1 (above)");
  if (!buf) return fail(c, SRMHD_E_INVAL, "buf is NULL");
  const int G = c->cfg.ghost_z, nz = c->cfg.nz;
  HaloArgs h;
  // the state the next stage reads (the work registers mid-step, else the
  // caller's arrays), and W
  const StageState st = stage_state(c, stage_code(c, c->next_stage));
  for (int n = 0; n < 5; ++n) h.a[n] = const_cast<double*>(st.cons[n]);
  for (int d = 0; d < 3; ++d) h.a[5 + d] = st.bf[d];
  h.a[8] = c->buf.guess_w;
  h.buf = buf;
  h.plane = (long long)c->cfg.nx * c->cfg.ny;
  h.G = G;
  // pack: the interior's edge planes; unpack: the ghost planes beyond them
  h.z0 = pack ? (side == 0 ? G : nz) : (side == 0 ? 0 : G + nz);
  launch_halo(h, pack, c->stream);
  return check_launch(c, what);
}
}  // namespace

int srmhd_halo_pack(srmhd_ctx* c, int side, double* buf) { return halo_copy(c, side, buf, true); }

int srmhd_halo_unpack(srmhd_ctx* c, int side, const double* buf) {
  return halo_copy(c, side, const_cast<double*>(buf), false);
}

const char* srmhd_build_id(void) { return SRMHD_BUILD_ID; }

int srmhd_get_diagnostics(srmhd_ctx* c, srmhd_diag* out) {
  if (!c) return SRMHD_E_INVAL;
  if (!out) return fail(c, SRMHD_E_INVAL, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (c->initialized) {
    ReduceArgs a;
    a.g = c->g;
    a.ho = c->cfg.high_order;
    for (int n = 0; n < 5; ++n) a.a[n] = c->buf.cons[n];
    for (int d = 0; d < 3; ++d) {
      a.a[5 + d] = c->buf.bface[d];
      a.bf[d] = c->buf.bface[d];
    }
    a.partial = c->partial;
    a.nblocks = reduce_blocks(c->g);
    a.sc = c->sc;
    launch_reduce(a, c->stream);
    int rc = check_launch(c, "diagnostics reduction");
    if (rc != SRMHD_OK) return rc;
  }
  DevScalars sc;
  std::vector<unsigned long long> cnt((size_t)kReplicas * CNT_N);
  int rc = hip_check(c, hipMemcpyAsync(&sc, c->sc, sizeof(sc), hipMemcpyDeviceToHost, c->stream),
                     "copy scalars");
  if (rc != SRMHD_OK) return rc;
  rc = hip_check(c, hipMemcpyAsync(cnt.data(), c->counters, cnt.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream),
                 "copy counters");
  if (rc != SRMHD_OK) return rc;
  rc = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
  if (rc != SRMHD_OK) return rc;
  unsigned long long tot[CNT_N] = {0};
  for (int r = 0; r < kReplicas; ++r)
    for (int n = 0; n < CNT_N; ++n) tot[n] += cnt[r * CNT_N + n];
  out->t = sc.t;
  out->dt = sc.dt;
  out->step = (long)sc.step;
  out->amax = sc.amax_last;
  for (int n = 0; n < 8; ++n) out->sums[n] = sc.reduce_out[n];
  out->divb_max = sc.reduce_out[8];
  out->newton_iters = (long)tot[CNT_ITERS];
  out->newton_calls = (long)tot[CNT_CALLS];
  for (int b = 0; b < 32; ++b) out->newton_hist[b] = (long)tot[CNT_HIST0 + b];
  out->c2p_failures = (long)tot[CNT_FAIL];
  out->recon_fallbacks = (long)tot[CNT_FALLBACK];
  out->floors = (long)tot[CNT_FLOOR];
  out->mlp_fallbacks = (long)tot[CNT_MLPFB];
  out->error_word = sc.err;
  if (sc.err & (SRMHD_ERRBIT_NONFINITE | SRMHD_ERRBIT_DT))
    return fail(c, SRMHD_E_NONFINITE, "non-finite conserved data or timestep on the device");
  if (sc.err & (SRMHD_ERRBIT_C2P | SRMHD_ERRBIT_PRESSURE))
    return fail(c, SRMHD_E_C2P, "Newton inversion failed in some cell");
  return SRMHD_OK;
}

int srmhd_reset_counters(srmhd_ctx* c) {
  if (!c) return SRMHD_E_INVAL;
  launch_zero_u64(c->counters, (size_t)kReplicas * CNT_N, c->stream);
  // the error word (and its padding) lives in the scalars block: clear only
  // that 8-byte word, keeping t, dt and step
  launch_zero_u64((unsigned long long*)&c->sc->err, 1, c->stream);
  return check_launch(c, "reset_counters");
}

int srmhd_get_time(srmhd_ctx* c, double* t, long* step, double* dt) {
  if (!c) return SRMHD_E_INVAL;
  DevScalars sc;
  int rc = hip_check(c, hipMemcpyAsync(&sc, c->sc, sizeof(sc), hipMemcpyDeviceToHost, c->stream),
                     "copy scalars");
  if (rc != SRMHD_OK) return rc;
  rc = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
  if (rc != SRMHD_OK) return rc;
  if (t) *t = sc.t;
  if (step) *step = (long)sc.step;
  if (dt) *dt = sc.dt;
  return SRMHD_OK;
}

int srmhd_set_time(srmhd_ctx* c, double t, long step) {
  if (!c) return SRMHD_E_INVAL;
  if (!std::isfinite(t) || step < 0) return fail(c, SRMHD_E_INVAL, "bad time or step");
  launch_set_time(c->sc, t, step, c->stream);
  return check_launch(c, "set_time");
}

int srmhd_set_mlp(srmhd_ctx* c, const float* params, const uint16_t* w_bf16, const float* norm) {
  if (!c) return SRMHD_E_INVAL;
  c->prims_ready = false;
  if (!params || !w_bf16 || !norm) return fail(c, SRMHD_E_INVAL, "params/w_bf16/norm is NULL");
  if (reinterpret_cast<uintptr_t>(w_bf16) % 8 != 0)
    return fail(c, SRMHD_E_INVAL, "w_bf16 must be 8-byte aligned");
  MlpDev m;
  m.w = w_bf16;
  m.p = params;
  for (int k = 0; k < kMlpIn; ++k) {
    if (!(norm[kMlpIn + k] > 0.f) || !std::isfinite(norm[k]))
      return fail(c, SRMHD_E_INVAL, "feature std must be > 0 and means finite");
    m.fmean[k] = norm[k];
    m.finv[k] = 1.f / norm[kMlpIn + k];
  }
  for (int k = 0; k < kMlpOut; ++k) {
    if (!(norm[2 * kMlpIn + kMlpOut + k] > 0.f) || !std::isfinite(norm[2 * kMlpIn + k]))
      return fail(c, SRMHD_E_INVAL, "output std must be > 0 and means finite");
    m.omean[k] = norm[2 * kMlpIn + k];
    m.ostd[k] = norm[2 * kMlpIn + kMlpOut + k];
  }
  c->mlp = m;
  c->mlp_set = true;
  return SRMHD_OK;
}

int srmhd_set_guess(srmhd_ctx* c, int guess) {
  if (!c) return SRMHD_E_INVAL;
  c->prims_ready = false;
  if (guess != SRMHD_GUESS_PREV && guess != SRMHD_GUESS_COLD && guess != SRMHD_GUESS_MLP &&
      guess != SRMHD_GUESS_MLP_ALL)
    return fail(c, SRMHD_E_INVAL, "bad guess mode");
  if ((guess == SRMHD_GUESS_MLP || guess == SRMHD_GUESS_MLP_ALL) && !c->mlp_set)
    return fail(c, SRMHD_E_STATE, "learned guess needs srmhd_set_mlp first");
  c->cfg.guess = guess;
  return SRMHD_OK;
}

int srmhd_harvest(srmhd_ctx* c, float* feats, float* targets, int cap, double frac, unsigned seed,
                  int* n_out) {
  if (!c) return SRMHD_E_INVAL;
  if (!c->initialized) return fail(c, SRMHD_E_STATE, "harvest before init_from_prims");
  if (check_between_steps(c, "harvest") != SRMHD_OK) return SRMHD_E_STATE;
  if (!feats || !targets || !n_out || cap <= 0 || !(frac > 0.0 && frac <= 1.0))
    return fail(c, SRMHD_E_INVAL, "bad harvest arguments");
  HarvestArgs a;
  a.g = c->g;
  a.ho = c->cfg.high_order;
  for (int n = 0; n < 5; ++n) a.cons[n] = c->buf.cons[n];
  for (int d = 0; d < 3; ++d) a.bf[d] = c->buf.bface[d];
  a.W = c->buf.guess_w;
  a.gam = c->cfg.gamma_ad;
  a.tol = c->cfg.newton_tol;
  a.maxit = c->cfg.newton_maxit;
  a.feats = feats;
  a.targets = targets;
  a.cap = cap;
  // slot counter: the low 32 bits of the scalars block's harvest word
  a.count = (unsigned int*)&c->sc->harvest;
  launch_zero_u64(&c->sc->harvest, 1, c->stream);
  a.frac = frac;
  a.seed = seed;
  launch_harvest(a, c->stream);
  int rc = check_launch(c, "harvest");
  if (rc != SRMHD_OK) return rc;
  unsigned cnt = 0;
  rc = hip_check(c, hipMemcpyAsync(&cnt, a.count, sizeof(unsigned), hipMemcpyDeviceToHost,
                                   c->stream), "copy harvest count");
  if (rc != SRMHD_OK) return rc;
  rc = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
  if (rc != SRMHD_OK) return rc;
  *n_out = (int)(cnt < (unsigned)cap ? cnt : (unsigned)cap);
  return SRMHD_OK;
}

int srmhd_kernel_timing(srmhd_ctx* c, int enable) {
  if (!c) return SRMHD_E_INVAL;
  int rc = drain_events(c);
  if (rc != SRMHD_OK) return rc;
  if (enable && c->ev.empty()) {
    c->ev.resize(2 * kEventPairs);
    c->ev_class.resize(kEventPairs);
    for (auto& e : c->ev) {
      rc = hip_check(c, hipEventCreate(&e), "hipEventCreate");
      if (rc != SRMHD_OK) return rc;
    }
  }
  c->timing = enable != 0;
  for (int k = 0; k < SRMHD_NKCLASS; ++k) {
    c->kms[k] = 0.0;
    c->kcount[k] = 0;
  }
  return SRMHD_OK;
}

int srmhd_get_kernel_times(srmhd_ctx* c, double* ms, long* launches) {
  if (!c) return SRMHD_E_INVAL;
  if (!ms || !launches) return fail(c, SRMHD_E_INVAL, "ms/launches is NULL");
  const int rc = drain_events(c);
  if (rc != SRMHD_OK) return rc;
  for (int k = 0; k < SRMHD_NKCLASS; ++k) {
    ms[k] = c->kms[k];
    launches[k] = c->kcount[k];
  }
  return SRMHD_OK;
}

const char* srmhd_last_error(const srmhd_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

const char* srmhd_strerror(int code) {
  switch (code) {
    case SRMHD_OK: return "ok";
    case SRMHD_E_INVAL: return "invalid argument or configuration";
    case SRMHD_E_HIP: return "HIP runtime error";
    case SRMHD_E_C2P: return "Newton inversion failed";
    case SRMHD_E_NONFINITE: return "non-finite data";
    case SRMHD_E_STATE: return "call out of order";
    default: return "unknown error";
  }
}

void srmhd_destroy(srmhd_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
