// mhd_api.hip -- host runtime of libmhd: argument validation, the context
// and its scratch, and the launch sequence of each integrator.
//
// Step sequence of the VL (MUSCL-Hancock) integrator, paper Sec. 3.2,
// VL steps 1-7, one kernel per stage:
//   k_prim   U^n, B^n            -> W^n (and the CFL maximum for mhd_advance)
//   k_flux   W^n, B^n  (1st ord) -> F      steps 1
//   k_emf    F, W^n              -> E      step 2
//   k_half   U^n, B^n, F, E      -> W^{n+1/2}, B^{n+1/2}   step 3
//   k_flux   W^{n+1/2}, PLM      -> F      steps 4-5
//   k_emf    F, W^{n+1/2}        -> E      step 6
//   k_final  U^n, B^n, F, E      -> U^{n+1}, B^{n+1} in place   step 7
// With a patch-group list every stage covers the groups plus the halo that
// the later stages read (3 ghost cells per side for U^n).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>

#include "../../include/mhd.h"
#include "mhd_kernels.hpp"
#include "mhd_amr.hpp"

using namespace mhd;

// Stage scratch of mhd_step_noalloc: a file-scope device array, one copy per
// device, held until the process ends.  Host code never passes its name to a
// kernel (on the host it is a stand-in, not a device address): mhd_init looks
// up this device's address once with hipGetSymbolAddress and every use goes
// through that pointer.
static __device__ __align__(256) unsigned char scratch[MHD_NOALLOC_SCRATCH_BYTES];

struct mhd_ctx_s {
  mhd_config cfg;
  hipStream_t stream;
  int device;
  size_t elem;            // bytes per state element
  long long cap_cells;    // capacity of the scratch arrays
  long long cap_parts;    // capacity of the reduction partials
  void* W;                // 8 * cap  (W^n, then W^{n+1/2})
  void* Bh;               // 3 * cap
  void* F;                // 21 * cap
  void* E;                // 3 * cap
  void* QL;               // CTU: 21 * cap, states below each face
  void* QR;               // CTU: 21 * cap, states above each face
  void* F2;               // CTU: 21 * cap, corrector fluxes
  void* RF;               // time-averaged final fluxes of a sub-cycled level: 21 * cap_reg
  void* RE;               // time-averaged final EMFs: 3 * cap_reg
  long long cap_reg;
  int* rflags;            // regridding: one flag per candidate fine group
  long long cap_rflags;
  int* occ_old;           // regridding: occupancy of the fine level's previous list
  long long cap_occ_old;
  double* parts;          // reduction partials
  double* dres;           // 8 device doubles of reduction results
  unsigned long long* smax;
  int* flag;
  unsigned long long* nfb;
  double* host;           // pinned host scratch (16 doubles)
  int* occ;               // group occupancy map
  long long cap_occ;
  MlpWeights* mlpw;       // inference weights of the learned flux
  bool mlp_ready;
  Capture capture;        // interface capture (buf == nullptr: off)
  float* mlp_ws;          // training workspace
  long long cap_mlp;      // batch capacity of mlp_ws
  int num_cu;             // compute units of the device
  long long max_blocks;   // cap on stage-kernel grids (0: none)
  int threads;            // threads per block of the stage kernels (64 .. 512)
  int batch;              // group-list batch: groups per launch of the middle stages (0: all)
  int lds_tiles;          // CTU + PPM step 1 on LDS tiles (1) or per cell (0)
  hipGraph_t graph;       // captured mhd_advance
  hipGraphExec_t graph_exec;
  mhd_level graph_key;
  double* graph_dt;
  double* graph_t;
  unsigned char* static_scratch;   // this device's copy of the file-scope scratch array
};

namespace {

bool valid_gamma(double g) { return g > 1.0 && g < 10.0; }

int check_config(const mhd_config* c) {
  if (!c) return MHD_ERR_INVALID_ARG;
  if (c->scheme != MHD_VL && c->scheme != MHD_CTU) return MHD_ERR_INVALID_ARG;
  if (c->recon != MHD_PLM && c->recon != MHD_PPM) return MHD_ERR_INVALID_ARG;
  if (c->riemann < MHD_ROE || c->riemann > MHD_MLP) return MHD_ERR_INVALID_ARG;
  if (c->prec < MHD_F64 || c->prec > MHD_F32_MIXED) return MHD_ERR_INVALID_ARG;
  if (!valid_gamma(c->gamma)) return MHD_ERR_INVALID_ARG;
  if (!(c->courant > 0.0 && c->courant <= 1.0)) return MHD_ERR_INVALID_ARG;
  // the learned flux runs in FP32 inside the CTU Riemann stages
  if (c->riemann == MHD_MLP && (c->scheme != MHD_CTU || c->prec == MHD_F64)) return MHD_ERR_UNSUPPORTED;
  if (c->riemann == MHD_MLP && !(std::isfinite(c->mlp_dp) && std::isfinite(c->mlp_drho))) return MHD_ERR_INVALID_ARG;
  if (c->prec == MHD_F32_MIXED && !(c->beta_fp64 >= 0.0)) return MHD_ERR_INVALID_ARG;
  return MHD_OK;
}

int check_level(const mhd_ctx_s* ctx, const mhd_level* lv) {
  if (!lv) return MHD_ERR_INVALID_ARG;
  if (lv->nx < 4 || lv->ny < 4 || lv->nz < 4) return MHD_ERR_INVALID_ARG;
  if ((long long)lv->nx * lv->ny * lv->nz > (1LL << 34)) return MHD_ERR_INVALID_ARG;
  if (!(lv->dx > 0.0)) return MHD_ERR_INVALID_ARG;
  if (!lv->U || !lv->B) return MHD_ERR_INVALID_ARG;
  if (ctx && ctx->cfg.prec == MHD_F32_MIXED && !lv->E64) return MHD_ERR_INVALID_ARG;
  if (lv->groups || lv->n_groups) {
    if (!lv->groups || lv->n_groups <= 0) return MHD_ERR_INVALID_ARG;
    if (lv->group_edge < 4) return MHD_ERR_INVALID_ARG;
    if (lv->nx % lv->group_edge || lv->ny % lv->group_edge || lv->nz % lv->group_edge)
      return MHD_ERR_INVALID_ARG;
    // the halo of a group must not wrap onto itself
    if (lv->nx < lv->group_edge + 8 || lv->ny < lv->group_edge + 8 || lv->nz < lv->group_edge + 8)
      return MHD_ERR_INVALID_ARG;
  }
  return MHD_OK;
}

#define HIP_TRY(x)                                 \
  do {                                             \
    if ((x) != hipSuccess) return MHD_ERR_HIP;     \
  } while (0)

void free_scratch(mhd_ctx_s* c) {
  void** bufs[] = {&c->W, &c->Bh, &c->F, &c->E, &c->QL, &c->QR, &c->F2};
  for (void** b : bufs) {
    hipFree(*b);
    *b = nullptr;
  }
  c->cap_cells = 0;
}

int ensure_capacity(mhd_ctx_s* c, long long cells) {
  if (cells <= c->cap_cells) return MHD_OK;
  free_scratch(c);
  const size_t e = c->elem;
  bool ok = hipMalloc(&c->W, 8 * cells * e) == hipSuccess && hipMalloc(&c->Bh, 3 * cells * e) == hipSuccess &&
            hipMalloc(&c->F, 21 * cells * e) == hipSuccess && hipMalloc(&c->E, 3 * cells * e) == hipSuccess;
  if (ok && c->cfg.scheme == MHD_CTU)
    ok = hipMalloc(&c->QL, 21 * cells * e) == hipSuccess && hipMalloc(&c->QR, 21 * cells * e) == hipSuccess &&
         hipMalloc(&c->F2, 21 * cells * e) == hipSuccess;
  if (!ok) {
    free_scratch(c);
    return MHD_ERR_OUT_OF_MEMORY;
  }
  c->cap_cells = cells;
  return MHD_OK;
}

int ensure_parts(mhd_ctx_s* c, long long n) {
  if (n <= c->cap_parts) return MHD_OK;
  hipFree(c->parts);
  c->parts = nullptr;
  c->cap_parts = 0;
  if (hipMalloc(&c->parts, n * sizeof(double)) != hipSuccess) return MHD_ERR_OUT_OF_MEMORY;
  c->cap_parts = n;
  return MHD_OK;
}

// Work description of one stage: whole grid, or groups with a halo of lo
// cells below and hi cells above each group in every dimension.
Work make_work(const mhd_level* lv, int lo, int hi) {
  Work w;
  w.nx = lv->nx; w.ny = lv->ny; w.nz = lv->nz;
  w.N = (long long)lv->nx * lv->ny * lv->nz;
  if (lv->groups && lv->n_groups > 0) {
    w.groups = lv->groups;
    w.edge = lv->group_edge;
    w.halo = lo;
    w.box = lv->group_edge + lo + hi;
    w.items = (long long)lv->n_groups * w.box * w.box * w.box;
    w.gnx = lv->nx / lv->group_edge;
    w.gny = lv->ny / lv->group_edge;
    w.gnz = lv->nz / lv->group_edge;
  } else {
    w.groups = nullptr;
    w.edge = 0;
    w.halo = 0;
    w.box = 0;
    w.items = w.N;
    w.gnx = w.gny = w.gnz = 0;
  }
  w.occ = nullptr;
  w.n_dev = (lv->groups && lv->n_groups > 0) ? lv->n_groups_dev : nullptr;
  w.oshift = 0;
  w.gbase = 0;
  w.gcount = 1 << 30;
  w.NS = w.N;
  w.sb = 0;
  w.soff = 0;
  return w;
}

// Work of an update stage whose items reach lo / hi cells below / above each
// group; with a group list the stage scratch is addressed per group, in boxes
// of edge + 2 ghost cells (ghost >= lo, hi).
// ghost cells a step reads around a group: 4 for CTU and for PPM, 3 for VL + PLM
int step_ghost(const mhd_ctx_s* c) { return c->cfg.scheme == MHD_CTU || c->cfg.recon == MHD_PPM ? 4 : 3; }

long long scratch_box(const mhd_level* lv, int ghost) { return (long long)lv->group_edge + 2 * ghost; }
bool list_mode(const mhd_level* lv) { return lv->groups && lv->n_groups > 0; }

long long scratch_cells(const mhd_level* lv, int ghost) {
  if (!list_mode(lv)) return (long long)lv->nx * lv->ny * lv->nz;
  const long long sb = scratch_box(lv, ghost);
  return ((long long)lv->n_groups + 2) * sb * sb * sb;
}

Work stage_work(const mhd_level* lv, int lo, int hi, int ghost) {
  Work w = make_work(lv, lo, hi);
  if (list_mode(lv)) {
    w.sb = (int)scratch_box(lv, ghost);
    w.NS = scratch_cells(lv, ghost);
    w.soff = ghost - lo;
  }
  return w;
}

// groups of a level's occupancy map (list mode)
long long occupancy_cells(const mhd_level* lv) {
  return (long long)(lv->nx / lv->group_edge) * (lv->ny / lv->group_edge) * (lv->nz / lv->group_edge);
}

// fill an occupancy map of occupancy_cells(lv) ints (list mode only): clear
// with a kernel, then mark the listed groups
void fill_occupancy(mhd_ctx_s* c, const mhd_level* lv, int* occ) {
  const long long ng = occupancy_cells(lv);
  k_occ_clear<<<(unsigned)((ng + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(occ, ng);
  k_occ_set<<<(unsigned)((lv->n_groups + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(
      occ, lv->groups, lv->n_groups, lv->n_groups_dev, lv->group_edge, lv->nx / lv->group_edge,
      lv->ny / lv->group_edge, lv->nz / lv->group_edge);
}

// occupancy map of a level's group list (list mode only) into *occ
int build_occupancy_into(mhd_ctx_s* c, const mhd_level* lv, int** occ, long long* cap) {
  if (!lv->groups || lv->n_groups <= 0) return MHD_OK;
  const long long ng = occupancy_cells(lv);
  if (ng > *cap) {
    hipFree(*occ);
    *occ = nullptr;
    *cap = 0;
    if (hipMalloc(occ, ng * sizeof(int)) != hipSuccess) return MHD_ERR_OUT_OF_MEMORY;
    *cap = ng;
  }
  fill_occupancy(c, lv, *occ);
  return MHD_OK;
}

// occupancy map of the level's group list in the context's map
int build_occupancy(mhd_ctx_s* c, const mhd_level* lv) { return build_occupancy_into(c, lv, &c->occ, &c->cap_occ); }

// grid of a reduction kernel: one thread per item (fixed, so results are
// bitwise stable)
unsigned nblocks(const Work& w) { return (unsigned)((w.items + kBlock - 1) / kBlock); }

// grid of a stage kernel: capped by the context's launch shape
thread_local long long g_max_blocks = 0;
thread_local int g_threads = kBlock;
unsigned sblocks(const Work& w, int threads = g_threads) {
  long long b = (w.items + threads - 1) / threads;
  if (g_max_blocks > 0 && b > g_max_blocks) b = g_max_blocks;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// Batches of a group list: the middle stages (between the primitive pass,
// which also reduces the CFL maximum over the whole list, and the final
// update, which writes the level in place) run batch by batch, each batch
// of at most `batch` groups through all of them, so a batch's intermediates
// can still be in the chip's caches when the next stage reads them.  Each
// group's scratch box holds its own halo, so batches are independent.
int num_batches(const Work& w, int batch) {
  if (!w.groups || batch <= 0) return 1;
  const long long n = w.items / ((long long)w.box * w.box * w.box);
  return (int)((n + batch - 1) / batch);
}
Work batch_of(Work w, int b, int batch) {
  if (!w.groups || batch <= 0) return w;
  const long long n = w.items / ((long long)w.box * w.box * w.box);
  w.gbase = b * batch;
  w.gcount = (int)(n - w.gbase < batch ? n - w.gbase : batch);
  w.items = (long long)w.gcount * w.box * w.box * w.box;
  return w;
}

// Stage names in launch order (used by mhd_profile_step).
const char* const kStageNamesVL[] = {"prim", "flux_predict", "emf_predict", "half_step",
                                     "flux_correct", "emf_correct", "final"};
const char* const kStageNamesCTU[] = {"prim", "states", "flux_predict", "emf_predict", "half_step",
                                      "flux_correct", "emf_correct", "final"};
constexpr int kMaxStages = 8;
int num_stages(const mhd_ctx_s* c) { return c->cfg.scheme == MHD_CTU ? 8 : 7; }
const char* stage_name(const mhd_ctx_s* c, int s) {
  return c->cfg.scheme == MHD_CTU ? kStageNamesCTU[s] : kStageNamesVL[s];
}

// Stage scratch of one step: the context's (allocated on demand) or carved
// from the static array of the allocation-free entry point.
struct StepBufs {
  void *W, *Bh, *F, *E, *QL, *QR, *F2;
  int* occ;
};

StepBufs ctx_bufs(const mhd_ctx_s* c) {
  return StepBufs{c->W, c->Bh, c->F, c->E, c->QL, c->QR, c->F2, c->occ};
}

// EMF stage: in double on a whole grid LDS tiles of 16 x 8 x 4 cells (15 %
// faster than one cell per item there); in float, and on group lists, one
// cell per item (in float the tiles were 10-20 % slower for every shape
// tried: 32 x 4 x 2, 32 x 8 x 2, 16 x 8 x 4, 64 x 2 x 2)
template <typename T, bool L>
void launch_emf(const Work& w, const T* F, const T* W, T* E, int nt, hipStream_t st) {
  if constexpr (!L && sizeof(T) == 8) {
    constexpr int TX = 16, TY = 8, TZ = 4;
    const long long nb = (long long)((w.nx + TX - 1) / TX) * ((w.ny + TY - 1) / TY) * ((w.nz + TZ - 1) / TZ);
    k_emf_tiled<T, TX, TY, TZ><<<(unsigned)nb, TX * TY * TZ, 0, st>>>(w, F, W, E);
  } else {
    k_emf<T, L><<<sblocks(w, nt), nt, 0, st>>>(w, F, W, E);
  }
}

// ev (optional): kNumStages + 1 events recorded around the stage kernels.
// R: 1 = PLM (minmod), 2 = PPM at the half step.
template <typename T, int S, int R, bool MIX, bool L>
void launch_step(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev, const StepBufs& sb) {
  const Mix mix{MIX ? lv->E64 : nullptr, c->cfg.beta_fp64};
  hipStream_t st = c->stream;
  T* U = (T*)lv->U;
  T* B = (T*)lv->B;
  T* W = (T*)sb.W;
  T* Bh = (T*)sb.Bh;
  T* F = (T*)sb.F;
  T* E = (T*)sb.E;
  const T gam = (T)c->cfg.gamma;
  const T inv_dx = (T)(1.0 / lv->dx);
  // ghost cells: 3 for PLM (the corrector's faces reach 2 cells below and 1
  // above), 4 for PPM (3 below and 2 above), and one more for each stage back
  constexpr int G = R == 2 ? 4 : 3;
  const Work wp = stage_work(lv, G, G, G), wf1 = stage_work(lv, G, G, G), we1 = stage_work(lv, G - 1, G, G);
  const Work wh = stage_work(lv, G - 1, G - 1, G), wf2 = stage_work(lv, 1, 1, G), we2 = stage_work(lv, 0, 1, G);
  Work wu = stage_work(lv, 0, 0, G);
  wu.occ = sb.occ;
  auto mark = [&](int s) {
    if (ev) (void)hipEventRecord(ev[s], st);
  };
  mark(0);
  if (cfl) {
    k_reset_smax<<<1, 1, 0, st>>>(c->smax);
    k_prim<T, true, MIX, L><<<sblocks(wp), g_threads, 0, st>>>(wp, U, B, mix, W, gam, c->smax, c->flag);
  } else {
    k_prim<T, false, MIX, L><<<sblocks(wp), g_threads, 0, st>>>(wp, U, B, mix, W, gam, c->smax, c->flag);
  }
  mark(1);
  const int nt = g_threads;
  const int batch = ev ? 0 : c->batch;   // profiling times whole stages
  for (int b = 0; b < num_batches(wf1, batch); ++b) {
    const Work f1 = batch_of(wf1, b, batch), e1 = batch_of(we1, b, batch), h = batch_of(wh, b, batch);
    const Work f2 = batch_of(wf2, b, batch), e2 = batch_of(we2, b, batch);
    k_flux<T, 0, S, L><<<sblocks(f1), nt, 0, st>>>(f1, W, B, F, gam, c->nfb);
    mark(2);
    launch_emf<T, L>(e1, F, W, E, nt, st);
    mark(3);
    k_half<T, MIX, L><<<sblocks(h), nt, 0, st>>>(h, U, B, mix, F, E, dts, inv_dx, gam, W, Bh);
    mark(4);
    k_flux<T, R, S, L><<<sblocks(f2), nt, 0, st>>>(f2, W, Bh, F, gam, c->nfb);
    mark(5);
    launch_emf<T, L>(e2, F, W, E, nt, st);
    mark(6);
  }
  k_final<T, MIX, L><<<sblocks(wu), nt, 0, st>>>(wu, U, B, mix, F, E, dts, inv_dx);
  mark(7);
}

// CTU, paper Sec. 3.2 steps 1-8:
//   k_prim         U^n, B^n             -> W^n
//   k_ctu_states   W^n, B^n, dt         -> QL, QR     step 1 (PPM/PLM + tracing)
//   k_flux_q       QL, QR, B^n          -> F1         step 2
//   k_emf          F1, W^n              -> E          step 3
//   k_half         U^n, B^n, F1, E      -> W^{n+1/2}, B^{n+1/2}   step 4
//   k_ctu_correct  QL, QR, F1, E, B^{n+1/2} -> F2     steps 5-6
//   k_emf          F2, W^{n+1/2}        -> E          step 7
//   k_final        U^n, B^n, F2, E      -> U^{n+1}, B^{n+1}   step 8
// Group halos (cells below, above each group): 4,4 / 2,2 / 2,2 / 1,2 / 1,1 /
// 1,1 / 0,1 / 0,0, i.e. 4 ghost cells of U^n.
// CTU step 1 with PPM on LDS tiles: 16 x 4 x 4 cells on a whole grid, 20 x 5
// x 5 on the 20^3 item boxes of 16^3 groups; false (nothing launched) for
// other group boxes, which take the per-cell kernel.  The tile kernels
// have a fixed block of one thread per tile cell.
template <typename T, bool ALLW, bool L, int TX, int TY, int TZ>
void launch_tiles(const Work& w, const T* W, const T* B, T* QL, T* QR, DtSrc dts, T inv_dx, T gam, hipStream_t st) {
  const long long units = L ? w.items / ((long long)w.box * w.box * w.box) : 1;
  long long nb = units * (L ? unit_tiles<TX, TY, TZ>(w.box, w.box, w.box) : unit_tiles<TX, TY, TZ>(w.nx, w.ny, w.nz));
  if (g_max_blocks > 0 && nb > g_max_blocks) nb = g_max_blocks;
  if (nb < 1) nb = 1;
  k_ctu_states_tiled<T, ALLW, L, TX, TY, TZ><<<(unsigned)nb, TX * TY * TZ, 0, st>>>(w, W, B, QL, QR, dts, inv_dx,
                                                                                   gam);
}

template <typename T, bool ALLW, bool L>
bool launch_states_tiled(const Work& w, const T* W, const T* B, T* QL, T* QR, DtSrc dts, T inv_dx, T gam,
                         hipStream_t st) {
  if constexpr (L) {
    if (w.box != 20) return false;
    launch_tiles<T, ALLW, L, 20, 5, 5>(w, W, B, QL, QR, dts, inv_dx, gam, st);
  } else {
    launch_tiles<T, ALLW, L, 16, 4, 4>(w, W, B, QL, QR, dts, inv_dx, gam, st);
  }
  return true;
}

template <typename T, int S, int R, bool MIX, bool L>
void launch_ctu(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev, const StepBufs& sb) {
  const Mix mix{MIX ? lv->E64 : nullptr, c->cfg.beta_fp64};
  hipStream_t st = c->stream;
  T* U = (T*)lv->U;
  T* B = (T*)lv->B;
  T* W = (T*)sb.W;
  T* Bh = (T*)sb.Bh;
  T* F1 = (T*)sb.F;
  T* F2 = (T*)sb.F2;
  T* E = (T*)sb.E;
  T* QL = (T*)sb.QL;
  T* QR = (T*)sb.QR;
  const T gam = (T)c->cfg.gamma;
  const T inv_dx = (T)(1.0 / lv->dx);
  constexpr int G = 4;   // ghost cells of CTU + PPM
  const Work wp = stage_work(lv, 4, 4, G), wq = stage_work(lv, 2, 2, G), wf1 = stage_work(lv, 2, 2, G);
  const Work we1 = stage_work(lv, 1, 2, G), wh = stage_work(lv, 1, 1, G), wf2 = stage_work(lv, 1, 1, G);
  const Work we2 = stage_work(lv, 0, 1, G);
  Work wu = stage_work(lv, 0, 0, G);
  wu.occ = sb.occ;
  auto mark = [&](int s) {
    if (ev) (void)hipEventRecord(ev[s], st);
  };
  mark(0);
  if (cfl) {
    k_reset_smax<<<1, 1, 0, st>>>(c->smax);
    k_prim<T, true, MIX, L><<<sblocks(wp), g_threads, 0, st>>>(wp, U, B, mix, W, gam, c->smax, c->flag);
  } else {
    k_prim<T, false, MIX, L><<<sblocks(wp), g_threads, 0, st>>>(wp, U, B, mix, W, gam, c->smax, c->flag);
  }
  mark(1);
  constexpr bool kMlp = S == 3 && std::is_same<T, float>::value;
  const float dp = (float)c->cfg.mlp_dp, drho = (float)c->cfg.mlp_drho;
  const int nt = g_threads;
  const int batch = ev ? 0 : c->batch;   // profiling times whole stages
  for (int b = 0; b < num_batches(wq, batch); ++b) {
    const Work q = batch_of(wq, b, batch), f1 = batch_of(wf1, b, batch), e1 = batch_of(we1, b, batch);
    const Work h = batch_of(wh, b, batch), f2 = batch_of(wf2, b, batch), e2 = batch_of(we2, b, batch);
    // the HLL-family solvers (HLLE, HLLD, the learned flux standing in for
    // HLLD) take every wave in the tracing, Roe only those moving toward an edge
    if (R != 1 || !c->lds_tiles || !launch_states_tiled<T, S != 0, L>(q, W, B, QL, QR, dts, inv_dx, gam, st))
      k_ctu_states<T, R, S != 0, L><<<sblocks(q), nt, 0, st>>>(q, W, B, QL, QR, dts, inv_dx, gam);
    mark(2);
    if constexpr (kMlp) {
      // the network kernels keep 256-thread blocks (one LDS stage per wave)
      const unsigned nb = sblocks(f1, kBlock);
      const long long n7 = 7LL * f1.NS;
      k_flux_dir_mlp<0, L><<<nb, kBlock, 0, st>>>(f1, QL, QR, B, F1, gam, c->mlpw, dp, drho, c->nfb,
                                                         c->capture);
      k_flux_dir_mlp<1, L><<<nb, kBlock, 0, st>>>(f1, QL + n7, QR + n7, B, F1, gam, c->mlpw, dp, drho,
                                                         c->nfb, c->capture);
      k_flux_dir_mlp<2, L><<<nb, kBlock, 0, st>>>(f1, QL + 2 * n7, QR + 2 * n7, B, F1, gam, c->mlpw, dp,
                                                         drho, c->nfb, c->capture);
    } else
      k_flux_q<T, S, L><<<sblocks(f1), nt, 0, st>>>(f1, QL, QR, B, F1, gam, c->nfb, c->capture);
    mark(3);
    launch_emf<T, L>(e1, F1, W, E, nt, st);
    mark(4);
    k_half<T, MIX, L><<<sblocks(h), nt, 0, st>>>(h, U, B, mix, F1, E, dts, inv_dx, gam, W, Bh);
    mark(5);
    if constexpr (kMlp) {
      const unsigned nb = sblocks(f2, kBlock);
      k_ctu_correct_mlp<0, L><<<nb, kBlock, 0, st>>>(f2, QL, QR, F1, E, B, Bh, F2, dts, inv_dx, gam, c->mlpw, dp,
                                                     drho, c->nfb, c->capture);
      k_ctu_correct_mlp<1, L><<<nb, kBlock, 0, st>>>(f2, QL, QR, F1, E, B, Bh, F2, dts, inv_dx, gam, c->mlpw, dp,
                                                     drho, c->nfb, c->capture);
      k_ctu_correct_mlp<2, L><<<nb, kBlock, 0, st>>>(f2, QL, QR, F1, E, B, Bh, F2, dts, inv_dx, gam, c->mlpw, dp,
                                                     drho, c->nfb, c->capture);
    } else
      k_ctu_correct<T, S, L><<<sblocks(f2), nt, 0, st>>>(f2, QL, QR, F1, E, B, Bh, F2, dts, inv_dx, gam, c->nfb,
                                                          c->capture);
    mark(6);
    launch_emf<T, L>(e2, F2, W, E, nt, st);
    mark(7);
  }
  k_final<T, MIX, L><<<sblocks(wu), nt, 0, st>>>(wu, U, B, mix, F2, E, dts, inv_dx);
  mark(8);
}

template <typename T, int S, bool MIX, bool L>
void launch_method(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev, const StepBufs& sb) {
  if constexpr (S == 3) {
    // learned flux: CTU only (validated at mhd_init)
    if (c->cfg.recon == MHD_PPM) launch_ctu<T, S, 1, MIX, L>(c, lv, dts, cfl, ev, sb);
    else launch_ctu<T, S, 0, MIX, L>(c, lv, dts, cfl, ev, sb);
    return;
  }
  if (c->cfg.scheme == MHD_VL) {
    if (c->cfg.recon == MHD_PPM) launch_step<T, S, 2, MIX, L>(c, lv, dts, cfl, ev, sb);
    else launch_step<T, S, 1, MIX, L>(c, lv, dts, cfl, ev, sb);
  }
  else if (c->cfg.recon == MHD_PPM) launch_ctu<T, S, 1, MIX, L>(c, lv, dts, cfl, ev, sb);
  else launch_ctu<T, S, 0, MIX, L>(c, lv, dts, cfl, ev, sb);
}

// group lists use per-group scratch boxes, whole grids the level's addressing
template <typename T, int S, bool MIX>
void launch_scheme(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev, const StepBufs& sb) {
  if (list_mode(lv)) launch_method<T, S, MIX, true>(c, lv, dts, cfl, ev, sb);
  else launch_method<T, S, MIX, false>(c, lv, dts, cfl, ev, sb);
}

template <typename T, bool MIX>
void launch_step_t(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev, const StepBufs& sb) {
  switch (c->cfg.riemann) {
    case MHD_ROE: launch_scheme<T, 0, MIX>(c, lv, dts, cfl, ev, sb); break;
    case MHD_HLLE: launch_scheme<T, 1, MIX>(c, lv, dts, cfl, ev, sb); break;
    case MHD_HLLD: launch_scheme<T, 2, MIX>(c, lv, dts, cfl, ev, sb); break;
    default: launch_scheme<T, 3, MIX>(c, lv, dts, cfl, ev, sb); break;
  }
}

// the stage kernels of one step on the given scratch
int run_step(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev, const StepBufs& sb) {
  g_max_blocks = c->max_blocks;
  g_threads = c->threads;
  if (c->cfg.prec == MHD_F64) launch_step_t<double, false>(c, lv, dts, cfl, ev, sb);
  else if (c->cfg.prec == MHD_F32) launch_step_t<float, false>(c, lv, dts, cfl, ev, sb);
  else launch_step_t<float, true>(c, lv, dts, cfl, ev, sb);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int do_step(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev = nullptr) {
  int rc = check_level(c, lv);
  if (rc) return rc;
  if (c->cfg.riemann == MHD_MLP && !c->mlp_ready) return MHD_ERR_INVALID_ARG;
  rc = ensure_capacity(c, scratch_cells(lv, step_ghost(c)));
  if (rc) return rc;
  rc = build_occupancy(c, lv);
  if (rc) return rc;
  return run_step(c, lv, dts, cfl, ev, ctx_bufs(c));
}

// ---- allocation-free step: stage scratch in a file-scope device array
constexpr size_t kStaticScratchBytes = (size_t)MHD_NOALLOC_SCRATCH_BYTES;
constexpr size_t kStaticAlign = 256;
constexpr int kMaxDevices = 64;
std::mutex g_static_mutex;
unsigned char* g_static_ptr[kMaxDevices];   // per device: its copy's device address

// scratch words per cell of a context's step (W, Bh, F, E; CTU adds QL, QR, F2)
long long step_words(const mhd_ctx_s* c) {
  long long words = 8 + 3 + 21 + 3;
  if (c->cfg.scheme == MHD_CTU) words += 63;
  return words;
}

size_t align_up(size_t x) { return (x + kStaticAlign - 1) / kStaticAlign * kStaticAlign; }

// carve the step's buffers out of base[0 .. kStaticScratchBytes); returns
// the bytes used (which may exceed the array: then nothing is carved)
size_t carve_static(const mhd_ctx_s* c, const mhd_level* lv, unsigned char* base, StepBufs* sb) {
  const long long cells = scratch_cells(lv, step_ghost(c));
  const size_t e = c->elem;
  const bool ctu = c->cfg.scheme == MHD_CTU;
  const size_t n[7] = {8, 3, 21, 3, ctu ? 21u : 0u, ctu ? 21u : 0u, ctu ? 21u : 0u};
  void** dst[7] = {&sb->W, &sb->Bh, &sb->F, &sb->E, &sb->QL, &sb->QR, &sb->F2};
  size_t off = 0;
  size_t at[8];
  for (int q = 0; q < 7; ++q) {
    at[q] = off;
    off = align_up(off + n[q] * (size_t)cells * e);
  }
  at[7] = off;
  if (list_mode(lv)) off = align_up(off + (size_t)occupancy_cells(lv) * sizeof(int));
  if (off > kStaticScratchBytes) return off;
  for (int q = 0; q < 7; ++q) *dst[q] = n[q] ? (void*)(base + at[q]) : nullptr;
  sb->occ = list_mode(lv) ? (int*)(base + at[7]) : nullptr;
  return off;
}

int read_flag(mhd_ctx_s* c, int* flag) {
  HIP_TRY(hipMemcpyAsync(c->host + 15, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::memcpy(flag, c->host + 15, sizeof(int));
  return MHD_OK;
}

}  // namespace

extern "C" {

int mhd_abi_version(void) { return MHD_ABI_VERSION; }

const char* mhd_strerror(int status) {
  switch (status) {
    case MHD_OK: return "ok";
    case MHD_ERR_INVALID_ARG: return "invalid argument";
    case MHD_ERR_UNSUPPORTED: return "unsupported combination of scheme, reconstruction, solver or precision";
    case MHD_ERR_SCRATCH_LIMIT: return "level needs more stage scratch than the allocation-free step's static array holds";
    case MHD_ERR_HIP: return "HIP runtime error";
    case MHD_ERR_NONPHYSICAL: return "non-physical state (rho <= 0 or p <= 0)";
    case MHD_ERR_NO_DEVICE: return "no HIP device";
    case MHD_ERR_OUT_OF_MEMORY: return "out of device memory";
    default: return "unknown status";
  }
}

int mhd_required_ghost(int scheme, int recon) {
  if (scheme != MHD_VL && scheme != MHD_CTU) return MHD_ERR_INVALID_ARG;
  if (recon == MHD_PLM) return 3;
  if (recon == MHD_PPM) return 4;
  return MHD_ERR_INVALID_ARG;
}

int mhd_workspace_bytes(mhd_ctx c, const mhd_level* lv, size_t* bytes) {
  if (!c || !bytes) return MHD_ERR_INVALID_ARG;
  const int rc = check_level(c, lv);
  if (rc) return rc;
  const int ghost = step_ghost(c);
  long long total = step_words(c) * scratch_cells(lv, ghost) * (long long)c->elem;
  if (list_mode(lv))
    total += (long long)(lv->nx / lv->group_edge) * (lv->ny / lv->group_edge) * (lv->nz / lv->group_edge) *
             (long long)sizeof(int);
  *bytes = (size_t)total;
  return MHD_OK;
}

int mhd_init(const mhd_config* cfg, void* hip_stream, mhd_ctx* out) {
  if (!out) return MHD_ERR_INVALID_ARG;
  *out = nullptr;
  int rc = check_config(cfg);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return MHD_ERR_NO_DEVICE;
  mhd_ctx_s* c = new (std::nothrow) mhd_ctx_s();
  if (!c) return MHD_ERR_OUT_OF_MEMORY;
  c->cfg = *cfg;
  c->stream = (hipStream_t)hip_stream;
  HIP_TRY(hipGetDevice(&c->device));
  c->elem = cfg->prec == MHD_F64 ? sizeof(double) : sizeof(float);
  c->threads = kBlock;
  c->batch = 0;
  c->lds_tiles = 0;
  {
    // this device's copy of the static scratch array, looked up once per device
    std::lock_guard<std::mutex> lock(g_static_mutex);
    if (c->device < 0 || c->device >= kMaxDevices) {
      delete c;
      return MHD_ERR_NO_DEVICE;
    }
    if (!g_static_ptr[c->device]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        delete c;
        return MHD_ERR_HIP;
      }
      g_static_ptr[c->device] = (unsigned char*)ptr;
    }
    c->static_scratch = g_static_ptr[c->device];
  }
  c->capture = Capture{nullptr, 0, nullptr, 1};
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
    if (c->num_cu <= 0) c->num_cu = 256;
  }
  if (hipMalloc(&c->dres, 8 * sizeof(double)) != hipSuccess || hipMalloc(&c->smax, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->flag, sizeof(int)) != hipSuccess || hipMalloc(&c->nfb, sizeof(unsigned long long)) != hipSuccess ||
      hipHostMalloc(&c->host, 16 * sizeof(double)) != hipSuccess) {
    mhd_finalize(c);
    return MHD_ERR_OUT_OF_MEMORY;
  }
  if (hipMemsetAsync(c->flag, 0, sizeof(int), c->stream) != hipSuccess ||
      hipMemsetAsync(c->nfb, 0, sizeof(unsigned long long), c->stream) != hipSuccess ||
      hipMemsetAsync(c->smax, 0, sizeof(unsigned long long), c->stream) != hipSuccess) {
    mhd_finalize(c);
    return MHD_ERR_HIP;
  }
  *out = c;
  return MHD_OK;
}

int mhd_finalize(mhd_ctx c) {
  if (!c) return MHD_ERR_INVALID_ARG;
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  if (c->graph) hipGraphDestroy(c->graph);
  free_scratch(c);
  hipFree(c->mlpw);
  hipFree(c->mlp_ws);
  hipFree(c->RF);
  hipFree(c->RE);
  hipFree(c->rflags);
  hipFree(c->occ_old);
  hipFree(c->parts); hipFree(c->dres); hipFree(c->smax); hipFree(c->flag); hipFree(c->nfb); hipFree(c->occ);
  if (c->host) hipHostFree(c->host);
  delete c;
  return MHD_OK;
}

int mhd_check_level(mhd_ctx ctx, const mhd_level* lv) { return check_level(ctx, lv); }

int mhd_prim_to_cons(mhd_ctx c, const mhd_level* lv, const void* W5) {
  if (!c || !W5) return MHD_ERR_INVALID_ARG;
  int rc = check_level(c, lv);
  if (rc) return rc;
  const Work w = make_work(lv, 0, 0);
  const Mix mix{lv->E64, c->cfg.beta_fp64};
  if (c->cfg.prec == MHD_F64)
    k_prim_to_cons<double, false><<<nblocks(w), kBlock, 0, c->stream>>>(
        w, (const double*)W5, (const double*)lv->B, (double*)lv->U, mix, c->cfg.gamma);
  else if (c->cfg.prec == MHD_F32)
    k_prim_to_cons<float, false><<<nblocks(w), kBlock, 0, c->stream>>>(
        w, (const float*)W5, (const float*)lv->B, (float*)lv->U, mix, (float)c->cfg.gamma);
  else
    k_prim_to_cons<float, true><<<nblocks(w), kBlock, 0, c->stream>>>(
        w, (const float*)W5, (const float*)lv->B, (float*)lv->U, mix, (float)c->cfg.gamma);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int mhd_cfl_dt(mhd_ctx c, const mhd_level* lv, double* dt_host, double* dt_dev) {
  if (!c) return MHD_ERR_INVALID_ARG;
  int rc = check_level(c, lv);
  if (rc) return rc;
  const Work w = make_work(lv, 0, 0);
  k_reset_smax<<<1, 1, 0, c->stream>>>(c->smax);
  const Mix mix{lv->E64, c->cfg.beta_fp64};
  if (c->cfg.prec == MHD_F64)
    k_cfl<double, false><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const double*)lv->U, (const double*)lv->B, mix,
                                                                c->cfg.gamma, c->smax, c->flag);
  else if (c->cfg.prec == MHD_F32)
    k_cfl<float, false><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const float*)lv->U, (const float*)lv->B, mix,
                                                               (float)c->cfg.gamma, c->smax, c->flag);
  else
    k_cfl<float, true><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const float*)lv->U, (const float*)lv->B, mix,
                                                              (float)c->cfg.gamma, c->smax, c->flag);
  const double cdx = c->cfg.courant * lv->dx;
  if (dt_dev) k_publish_dt<<<1, 1, 0, c->stream>>>(c->smax, cdx, dt_dev, nullptr);
  if (hipGetLastError() != hipSuccess) return MHD_ERR_HIP;
  if (dt_host) {
    HIP_TRY(hipMemcpyAsync(c->host, c->smax, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    int flag = 0;
    rc = read_flag(c, &flag);
    if (rc) return rc;
    if (flag) return MHD_ERR_NONPHYSICAL;
    const double smax = c->host[0];
    if (!(smax > 0.0)) return MHD_ERR_NONPHYSICAL;
    *dt_host = cdx / smax;
  }
  return MHD_OK;
}

int mhd_step(mhd_ctx c, const mhd_level* lv, double dt) {
  if (!c || !(dt > 0.0)) return MHD_ERR_INVALID_ARG;
  DtSrc s{dt, nullptr, nullptr, 0.0};
  return do_step(c, lv, s, false);
}

int mhd_step_devdt(mhd_ctx c, const mhd_level* lv, const double* dt_dev) {
  if (!c || !dt_dev) return MHD_ERR_INVALID_ARG;
  DtSrc s{0.0, dt_dev, nullptr, 0.0};
  return do_step(c, lv, s, false);
}

int mhd_step_noalloc(mhd_ctx c, const mhd_level* lv, const double* dt_dev) {
  if (!c || !dt_dev) return MHD_ERR_INVALID_ARG;
  int rc = check_level(c, lv);
  if (rc) return rc;
  if (c->cfg.riemann == MHD_MLP && !c->mlp_ready) return MHD_ERR_INVALID_ARG;
  if (!c->static_scratch) return MHD_ERR_HIP;
  StepBufs sb{};
  if (carve_static(c, lv, c->static_scratch, &sb) > kStaticScratchBytes) return MHD_ERR_SCRATCH_LIMIT;
  if (list_mode(lv)) fill_occupancy(c, lv, sb.occ);
  DtSrc s{0.0, dt_dev, nullptr, 0.0};
  return run_step(c, lv, s, false, nullptr, sb);
}

int mhd_advance(mhd_ctx c, const mhd_level* lv, double* dt_dev, double* t_dev) {
  if (!c || !lv) return MHD_ERR_INVALID_ARG;
  DtSrc s{0.0, nullptr, c->smax, c->cfg.courant * lv->dx};
  int rc = do_step(c, lv, s, true);
  if (rc) return rc;
  if (dt_dev || t_dev) {
    k_publish_dt<<<1, 1, 0, c->stream>>>(c->smax, c->cfg.courant * lv->dx, dt_dev, t_dev);
    if (hipGetLastError() != hipSuccess) return MHD_ERR_HIP;
  }
  return MHD_OK;
}

int mhd_num_stages(mhd_ctx c) {
  if (!c) return MHD_ERR_INVALID_ARG;
  return num_stages(c);
}

const char* mhd_stage_name(mhd_ctx c, int stage) {
  if (!c || stage < 0 || stage >= num_stages(c)) return nullptr;
  return stage_name(c, stage);
}

int mhd_profile_step(mhd_ctx c, const mhd_level* lv, int nrep, double* stage_ms) {
  if (!c || !lv || nrep <= 0 || !stage_ms) return MHD_ERR_INVALID_ARG;
  int rc = check_level(c, lv);
  if (rc) return rc;
  const int ns = num_stages(c);
  hipEvent_t ev[kMaxStages + 1];
  for (int s = 0; s <= ns; ++s)
    if (hipEventCreate(&ev[s]) != hipSuccess) return MHD_ERR_HIP;
  for (int s = 0; s < ns; ++s) stage_ms[s] = 0.0;
  DtSrc dts{0.0, nullptr, c->smax, c->cfg.courant * lv->dx};
  for (int r = 0; r < nrep && rc == MHD_OK; ++r) {
    rc = do_step(c, lv, dts, true, ev);
    if (rc) break;
    if (hipEventSynchronize(ev[ns]) != hipSuccess) { rc = MHD_ERR_HIP; break; }
    for (int s = 0; s < ns; ++s) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[s], ev[s + 1]) != hipSuccess) { rc = MHD_ERR_HIP; break; }
      stage_ms[s] += ms;
    }
  }
  for (int s = 0; s <= ns; ++s) (void)hipEventDestroy(ev[s]);
  if (rc) return rc;
  for (int s = 0; s < ns; ++s) stage_ms[s] /= nrep;
  return MHD_OK;
}

static void drop_graph(mhd_ctx_s* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

int mhd_set_launch(mhd_ctx c, int blocks_per_cu, int threads_per_block, int batch_groups, int lds_tiles) {
  if (!c || blocks_per_cu < 0 || batch_groups < 0 || (lds_tiles != 0 && lds_tiles != 1)) return MHD_ERR_INVALID_ARG;
  if (threads_per_block == 0) threads_per_block = kBlock;
  if (threads_per_block < 64 || threads_per_block > kMaxBlock || threads_per_block % 64) return MHD_ERR_INVALID_ARG;
  c->max_blocks = blocks_per_cu > 0 ? (long long)blocks_per_cu * c->num_cu : 0;
  c->threads = threads_per_block;
  c->batch = batch_groups;
  c->lds_tiles = lds_tiles;
  drop_graph(c);
  return MHD_OK;
}

int mhd_advance_graph(mhd_ctx c, const mhd_level* lv, double* dt_dev, double* t_dev) {
  if (!c || !lv) return MHD_ERR_INVALID_ARG;
  if (!c->stream) return MHD_ERR_INVALID_ARG;   // capture needs a non-default stream
  int rc = check_level(c, lv);
  if (rc) return rc;
  if (c->cfg.riemann == MHD_MLP && !c->mlp_ready) return MHD_ERR_INVALID_ARG;
  const bool same = c->graph_exec && std::memcmp(&c->graph_key, lv, sizeof(mhd_level)) == 0 &&
                    c->graph_dt == dt_dev && c->graph_t == t_dev;
  if (!same) {
    drop_graph(c);
    // allocations happen before the capture
    rc = ensure_capacity(c, scratch_cells(lv, step_ghost(c)));
    if (rc) return rc;
    if (lv->groups && lv->n_groups > 0) {
      const long long ng =
          (long long)(lv->nx / lv->group_edge) * (lv->ny / lv->group_edge) * (lv->nz / lv->group_edge);
      if (ng > c->cap_occ) {
        hipFree(c->occ);
        c->occ = nullptr;
        c->cap_occ = 0;
        if (hipMalloc(&c->occ, ng * sizeof(int)) != hipSuccess) return MHD_ERR_OUT_OF_MEMORY;
        c->cap_occ = ng;
      }
    }
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return MHD_ERR_HIP;
    DtSrc s{0.0, nullptr, c->smax, c->cfg.courant * lv->dx};
    rc = do_step(c, lv, s, true);
    if (rc == MHD_OK && (dt_dev || t_dev))
      k_publish_dt<<<1, 1, 0, c->stream>>>(c->smax, c->cfg.courant * lv->dx, dt_dev, t_dev);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess || !g) return MHD_ERR_HIP;
    c->graph = g;
    if (hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
      drop_graph(c);
      return MHD_ERR_HIP;
    }
    c->graph_key = *lv;
    c->graph_dt = dt_dev;
    c->graph_t = t_dev;
  }
  return hipGraphLaunch(c->graph_exec, c->stream) == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int mhd_cfl_dt_min(mhd_ctx c, const mhd_level* lv, double scale, double* dt_dev) {
  if (!c || !dt_dev || !(scale > 0.0 && std::isfinite(scale))) return MHD_ERR_INVALID_ARG;
  int rc = check_level(c, lv);
  if (rc) return rc;
  const Work w = make_work(lv, 0, 0);
  const Mix mix{lv->E64, c->cfg.beta_fp64};
  k_reset_smax<<<1, 1, 0, c->stream>>>(c->smax);
  if (c->cfg.prec == MHD_F64)
    k_cfl<double, false><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const double*)lv->U, (const double*)lv->B, mix,
                                                                c->cfg.gamma, c->smax, c->flag);
  else if (c->cfg.prec == MHD_F32)
    k_cfl<float, false><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const float*)lv->U, (const float*)lv->B, mix,
                                                               (float)c->cfg.gamma, c->smax, c->flag);
  else
    k_cfl<float, true><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const float*)lv->U, (const float*)lv->B, mix,
                                                              (float)c->cfg.gamma, c->smax, c->flag);
  k_min_dt<<<1, 1, 0, c->stream>>>(c->smax, c->cfg.courant * lv->dx * scale, dt_dev);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

}  // extern "C"

#include "mhd_amr_api.inc"

extern "C" {

int mhd_divB(mhd_ctx c, const mhd_level* lv, double* max_abs, double* l1) {
  if (!c) return MHD_ERR_INVALID_ARG;
  int rc = check_level(c, lv);
  if (rc) return rc;
  const Work w = make_work(lv, 0, 0);
  const unsigned nb = nblocks(w);
  rc = ensure_parts(c, 2LL * nb);
  if (rc) return rc;
  if (c->cfg.prec == MHD_F64)
    k_divb<double><<<nb, kBlock, 0, c->stream>>>(w, (const double*)lv->B, 1.0 / lv->dx, c->parts);
  else
    k_divb<float><<<nb, kBlock, 0, c->stream>>>(w, (const float*)lv->B, 1.0 / lv->dx, c->parts);
  k_finish<<<1, kBlock, 0, c->stream>>>(c->parts, (int)nb, 2, 1, c->dres);
  if (hipGetLastError() != hipSuccess) return MHD_ERR_HIP;
  HIP_TRY(hipMemcpyAsync(c->host, c->dres, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (l1) *l1 = c->host[0] / (double)w.N;
  if (max_abs) *max_abs = c->host[1];
  return MHD_OK;
}

int mhd_sums(mhd_ctx c, const mhd_level* lv, double out[7]) {
  if (!c || !out) return MHD_ERR_INVALID_ARG;
  int rc = check_level(c, lv);
  if (rc) return rc;
  const Work w = make_work(lv, 0, 0);
  const unsigned nb = nblocks(w);
  rc = ensure_parts(c, 7LL * nb);
  if (rc) return rc;
  const double* e64 = c->cfg.prec == MHD_F32_MIXED ? lv->E64 : nullptr;
  if (c->cfg.prec == MHD_F64)
    k_sums<double><<<nb, kBlock, 0, c->stream>>>(w, (const double*)lv->U, (const double*)lv->B, nullptr, c->parts);
  else
    k_sums<float><<<nb, kBlock, 0, c->stream>>>(w, (const float*)lv->U, (const float*)lv->B, e64, c->parts);
  k_finish<<<1, kBlock, 0, c->stream>>>(c->parts, (int)nb, 7, 7, c->dres);
  if (hipGetLastError() != hipSuccess) return MHD_ERR_HIP;
  HIP_TRY(hipMemcpyAsync(c->host, c->dres, 7 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const double dv = lv->dx * lv->dx * lv->dx;
  for (int q = 0; q < 7; ++q) out[q] = c->host[q] * dv;
  return MHD_OK;
}

int mhd_fallback_count(mhd_ctx c, long long* count) {
  if (!c || !count) return MHD_ERR_INVALID_ARG;
  HIP_TRY(hipMemcpyAsync(c->host, c->nfb, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  unsigned long long v;
  std::memcpy(&v, c->host, sizeof v);
  *count = (long long)v;
  HIP_TRY(hipMemsetAsync(c->nfb, 0, sizeof(unsigned long long), c->stream));
  return MHD_OK;
}

// ------------------------------------------------------------ learned flux
int mhd_mlp_set_weights(mhd_ctx c, const float* params_dev) {
  if (!c || !params_dev) return MHD_ERR_INVALID_ARG;
  if (!c->mlpw && hipMalloc(&c->mlpw, sizeof(MlpWeights)) != hipSuccess) return MHD_ERR_OUT_OF_MEMORY;
  k_mlp_pack<<<16, 256, 0, c->stream>>>(params_dev, c->mlpw);
  if (hipGetLastError() != hipSuccess) return MHD_ERR_HIP;
  c->mlp_ready = true;
  return MHD_OK;
}

}  // extern "C"

namespace {
// training workspace: Z1, H1, Z2, H2, dZ2, dZ1 (n x 64 each), Y, dY (n x 7),
// loss partials
constexpr int kSplitK = 256;            // batch rows per split-K chunk of a weight gradient
constexpr int kGradParts = 64 * 64;     // largest weight-gradient tile set

int ensure_mlp_ws(mhd_ctx_s* c, long long n) {
  if (n <= c->cap_mlp) return MHD_OK;
  hipFree(c->mlp_ws);
  c->mlp_ws = nullptr;
  c->cap_mlp = 0;
  const long long words = 6 * 64 * n + 2 * 7 * n + (7 * n + 255) / 256 + 16 + kGradParts * ((n + kSplitK - 1) / kSplitK);
  if (hipMalloc(&c->mlp_ws, words * sizeof(float)) != hipSuccess) return MHD_ERR_OUT_OF_MEMORY;
  c->cap_mlp = n;
  return MHD_OK;
}

struct MlpBufs {
  float *Z1, *H1, *Z2, *H2, *dZ2, *dZ1, *Y, *dY, *part, *gpart;
};

MlpBufs mlp_bufs(mhd_ctx_s* c) {
  const long long n = c->cap_mlp;
  float* b = c->mlp_ws;
  MlpBufs m;
  m.Z1 = b; m.H1 = b + 64 * n; m.Z2 = b + 128 * n; m.H2 = b + 192 * n; m.dZ2 = b + 256 * n; m.dZ1 = b + 320 * n;
  m.Y = b + 384 * n; m.dY = b + 391 * n; m.part = b + 398 * n;
  m.gpart = m.part + (7 * n + 255) / 256 + 16;
  return m;
}

// weight gradient C[M x N] = A^T B over the batch (K = n): split-K on MFMA
// with an ordered sum of the chunks (deterministic), M, N <= 64
void gemm_wgrad(hipStream_t st, int M, int N, int K, const float* A, long long sam, long long sak, const float* Bm,
                long long sbk, long long sbn, float* C, int ldc, float* gpart) {
  const int chunks = (K + kSplitK - 1) / kSplitK;
  const long long waves = (long long)((M + 15) / 16) * ((N + 15) / 16) * chunks;
  k_mlp_gemm_part<<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(M, N, K, kSplitK, A, sam, sak, Bm, sbk, sbn, gpart);
  k_mlp_sum_parts<<<(unsigned)((M * N + 255) / 256), 256, 0, st>>>(M, N, chunks, gpart, C, ldc);
}

template <int EPI>
void gemm(hipStream_t st, int M, int N, int K, const float* A, long long sam, long long sak, const float* Bm,
          long long sbk, long long sbn, const float* bias, const float* Zin, float* C, float* H, int ldc) {
  const long long waves = (long long)((M + 15) / 16) * ((N + 15) / 16);
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  k_mlp_gemm<EPI><<<blocks, 256, 0, st>>>(M, N, K, A, sam, sak, Bm, sbk, sbn, bias, Zin, C, H, ldc);
}

void mlp_forward(mhd_ctx_s* c, const float* P, const float* X, int n, const MlpBufs& b, float* Y) {
  hipStream_t st = c->stream;
  gemm<EPI_BIAS_GELU>(st, n, kNh, kNin, X, kNin, 1, P + oW1, kNh, 1, P + ob1, nullptr, b.Z1, b.H1, kNh);
  gemm<EPI_BIAS_GELU>(st, n, kNh, kNh, b.H1, kNh, 1, P + oW2, kNh, 1, P + ob2, nullptr, b.Z2, b.H2, kNh);
  gemm<EPI_BIAS>(st, n, kNout, kNh, b.H2, kNh, 1, P + oW3, kNout, 1, P + ob3, nullptr, Y, nullptr, kNout);
}

void mlp_backward(mhd_ctx_s* c, const float* P, const float* X, const float* dY, int n, const MlpBufs& b, float* G) {
  hipStream_t st = c->stream;
  gemm_wgrad(st, kNh, kNout, n, b.H2, 1, kNh, dY, kNout, 1, G + oW3, kNout, b.gpart);
  k_mlp_colsum<<<kNout, 256, 0, st>>>(n, kNout, dY, G + ob3);
  gemm<EPI_GELU_PRIME>(st, n, kNh, kNout, dY, kNout, 1, P + oW3, 1, kNout, nullptr, b.Z2, b.dZ2, nullptr, kNh);
  k_mlp_colsum<<<kNh, 256, 0, st>>>(n, kNh, b.dZ2, G + ob2);
  gemm_wgrad(st, kNh, kNh, n, b.H1, 1, kNh, b.dZ2, kNh, 1, G + oW2, kNh, b.gpart);
  gemm<EPI_GELU_PRIME>(st, n, kNh, kNh, b.dZ2, kNh, 1, P + oW2, 1, kNh, nullptr, b.Z1, b.dZ1, nullptr, kNh);
  k_mlp_colsum<<<kNh, 256, 0, st>>>(n, kNh, b.dZ1, G + ob1);
  gemm_wgrad(st, kNin, kNh, n, X, 1, kNin, b.dZ1, kNh, 1, G + oW1, kNh, b.gpart);
}
}  // namespace

extern "C" {

int mhd_mlp_num_params(void) { return kParams; }

int mhd_mlp_forward(mhd_ctx c, const float* params_dev, const float* X_dev, int n, float* Y_dev) {
  if (!c || !params_dev || !X_dev || !Y_dev || n <= 0) return MHD_ERR_INVALID_ARG;
  int rc = ensure_mlp_ws(c, n);
  if (rc) return rc;
  mlp_forward(c, params_dev, X_dev, n, mlp_bufs(c), Y_dev);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int mhd_mlp_backward(mhd_ctx c, const float* params_dev, const float* X_dev, const float* dY_dev, int n,
                     float* grads_dev) {
  if (!c || !params_dev || !X_dev || !dY_dev || !grads_dev || n <= 0) return MHD_ERR_INVALID_ARG;
  int rc = ensure_mlp_ws(c, n);
  if (rc) return rc;
  const MlpBufs b = mlp_bufs(c);
  mlp_forward(c, params_dev, X_dev, n, b, b.Y);
  mlp_backward(c, params_dev, X_dev, dY_dev, n, b, grads_dev);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int mhd_mlp_train_step(mhd_ctx c, float* params_dev, float* adam_m, float* adam_v, float* grads_dev, int step,
                       const float* X_dev, const float* T_dev, int n, float lr, float* loss_dev) {
  if (!c || !params_dev || !adam_m || !adam_v || !grads_dev || !X_dev || !T_dev || n <= 0 || step < 1 ||
      !(lr > 0.f))
    return MHD_ERR_INVALID_ARG;
  int rc = ensure_mlp_ws(c, n);
  if (rc) return rc;
  hipStream_t st = c->stream;
  const MlpBufs b = mlp_bufs(c);
  mlp_forward(c, params_dev, X_dev, n, b, b.Y);
  const long long total = 7LL * n;
  const unsigned nb = (unsigned)((total + 255) / 256);
  k_mlp_mse<<<nb, 256, 0, st>>>(total, b.Y, T_dev, b.dY, b.part);
  if (loss_dev) k_mlp_loss<<<1, 64, 0, st>>>(b.part, (int)nb, total, loss_dev);
  mlp_backward(c, params_dev, X_dev, b.dY, n, b, grads_dev);
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  k_mlp_adam<<<(kParams + 255) / 256, 256, 0, st>>>(params_dev, adam_m, adam_v, grads_dev, kParams, lr, b1, b2, 1e-8f,
                                                    c1, c2);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int mhd_mlp_prepare(mhd_ctx c, const float* samples_dev, int n, float* X_dev, float* T_dev, int* flags_dev) {
  if (!c || !samples_dev || !X_dev || !T_dev || !flags_dev || n <= 0) return MHD_ERR_INVALID_ARG;
  k_mlp_prepare<<<(n + 255) / 256, 256, 0, c->stream>>>(samples_dev, n, (float)c->cfg.gamma, (float)c->cfg.mlp_dp,
                                                        (float)c->cfg.mlp_drho, X_dev, T_dev, flags_dev);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

}  // extern "C"

namespace {
__global__ void __launch_bounds__(kBlock) k_mlp_faces(const float* __restrict__ S, int n, const MlpWeights* mw,
                                                      float gam, float dp, float drho, float* __restrict__ F,
                                                      int* __restrict__ used_hlld) {
  __shared__ MlpShared sh;
  mlp_load_weights(sh, mw);
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < n;
  float wl[7], wr[7], f[7];
  float bn = 1.0f;
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    wl[m] = active ? S[(long long)i * 15 + m] : 1.0f;
    wr[m] = active ? S[(long long)i * 15 + 7 + m] : 1.0f;
  }
  if (active) bn = S[(long long)i * 15 + 14];
  const int h = mlp_or_hlld(sh, active, wl, wr, bn, gam, dp, drho, f, Capture{nullptr, 0, nullptr, 1}, 0);
  if (active) {
#pragma unroll
    for (int m = 0; m < 7; ++m) F[(long long)i * 7 + m] = f[m];
    used_hlld[i] = h;
  }
}
}  // namespace

extern "C" {

int mhd_mlp_face_flux(mhd_ctx c, const float* states_dev, int n, float* flux_dev, int* used_hlld_dev) {
  if (!c || !states_dev || !flux_dev || !used_hlld_dev || n <= 0) return MHD_ERR_INVALID_ARG;
  if (!c->mlp_ready) return MHD_ERR_INVALID_ARG;
  k_mlp_faces<<<(n + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(states_dev, n, c->mlpw, (float)c->cfg.gamma,
                                                                     (float)c->cfg.mlp_dp, (float)c->cfg.mlp_drho,
                                                                     flux_dev, used_hlld_dev);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int mhd_set_capture(mhd_ctx c, float* buf_dev, long long cap, unsigned long long* count_dev, int stride) {
  if (!c) return MHD_ERR_INVALID_ARG;
  if (buf_dev && (cap <= 0 || !count_dev || stride <= 0)) return MHD_ERR_INVALID_ARG;
  if (buf_dev && c->cfg.prec == MHD_F64) return MHD_ERR_UNSUPPORTED;
  // the capture settings are kernel arguments of a captured step graph:
  // drop it, so a replay neither writes to a released buffer nor misses a
  // newly set one
  drop_graph(c);
  c->capture = buf_dev ? Capture{buf_dev, cap, count_dev, stride} : Capture{nullptr, 0, nullptr, 1};
  return MHD_OK;
}

int mhd_sync(mhd_ctx c) {
  if (!c) return MHD_ERR_INVALID_ARG;
  int flag = 0;
  int rc = read_flag(c, &flag);
  if (rc) return rc;
  return flag ? MHD_ERR_NONPHYSICAL : MHD_OK;
}

}  // extern "C"
