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

#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/mhd.h"
#include "mhd_kernels.hpp"

using namespace mhd;

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
  double* parts;          // reduction partials
  double* dres;           // 8 device doubles of reduction results
  unsigned long long* smax;
  int* flag;
  unsigned long long* nfb;
  double* host;           // pinned host scratch (16 doubles)
  int* occ;               // group occupancy map
  long long cap_occ;
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
  // implemented combinations: VL with PLM; CTU with PLM or PPM
  if (c->scheme == MHD_VL && c->recon != MHD_PLM) return MHD_ERR_UNSUPPORTED;
  if (c->riemann == MHD_MLP) return MHD_ERR_UNSUPPORTED;
  if (c->prec == MHD_F32_MIXED) return MHD_ERR_UNSUPPORTED;
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
  return w;
}

// occupancy map of the level's group list (list mode only)
int build_occupancy(mhd_ctx_s* c, const mhd_level* lv) {
  if (!lv->groups || lv->n_groups <= 0) return MHD_OK;
  const long long ng = (long long)(lv->nx / lv->group_edge) * (lv->ny / lv->group_edge) * (lv->nz / lv->group_edge);
  if (ng > c->cap_occ) {
    hipFree(c->occ);
    c->occ = nullptr;
    c->cap_occ = 0;
    if (hipMalloc(&c->occ, ng * sizeof(int)) != hipSuccess) return MHD_ERR_OUT_OF_MEMORY;
    c->cap_occ = ng;
  }
  k_occ_clear<<<(unsigned)((ng + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(c->occ, ng);
  k_occ_set<<<(unsigned)((lv->n_groups + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(
      c->occ, lv->groups, lv->n_groups, lv->group_edge, lv->nx / lv->group_edge, lv->ny / lv->group_edge);
  return MHD_OK;
}

unsigned nblocks(const Work& w) { return (unsigned)((w.items + kBlock - 1) / kBlock); }

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

// ev (optional): kNumStages + 1 events recorded around the stage kernels
template <typename T, int S>
void launch_step(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev = nullptr) {
  hipStream_t st = c->stream;
  T* U = (T*)lv->U;
  T* B = (T*)lv->B;
  T* W = (T*)c->W;
  T* Bh = (T*)c->Bh;
  T* F = (T*)c->F;
  T* E = (T*)c->E;
  const T gam = (T)c->cfg.gamma;
  const T inv_dx = (T)(1.0 / lv->dx);
  const Work wp = make_work(lv, 3, 3), wf1 = make_work(lv, 3, 3), we1 = make_work(lv, 2, 3);
  const Work wh = make_work(lv, 2, 2), wf2 = make_work(lv, 1, 1), we2 = make_work(lv, 0, 1);
  Work wu = make_work(lv, 0, 0);
  wu.occ = c->occ;
  auto mark = [&](int s) {
    if (ev) (void)hipEventRecord(ev[s], st);
  };
  mark(0);
  if (cfl) {
    k_reset_smax<<<1, 1, 0, st>>>(c->smax);
    k_prim<T, true><<<nblocks(wp), kBlock, 0, st>>>(wp, U, B, W, gam, c->smax, c->flag);
  } else {
    k_prim<T, false><<<nblocks(wp), kBlock, 0, st>>>(wp, U, B, W, gam, c->smax, c->flag);
  }
  mark(1);
  k_flux<T, 0, S><<<nblocks(wf1), kBlock, 0, st>>>(wf1, W, B, F, gam, c->nfb);
  mark(2);
  k_emf<T><<<nblocks(we1), kBlock, 0, st>>>(we1, F, W, E);
  mark(3);
  k_half<T><<<nblocks(wh), kBlock, 0, st>>>(wh, U, B, F, E, dts, inv_dx, gam, W, Bh);
  mark(4);
  k_flux<T, 1, S><<<nblocks(wf2), kBlock, 0, st>>>(wf2, W, Bh, F, gam, c->nfb);
  mark(5);
  k_emf<T><<<nblocks(we2), kBlock, 0, st>>>(we2, F, W, E);
  mark(6);
  k_final<T><<<nblocks(wu), kBlock, 0, st>>>(wu, U, B, F, E, dts, inv_dx);
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
template <typename T, int S, int R>
void launch_ctu(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev) {
  hipStream_t st = c->stream;
  T* U = (T*)lv->U;
  T* B = (T*)lv->B;
  T* W = (T*)c->W;
  T* Bh = (T*)c->Bh;
  T* F1 = (T*)c->F;
  T* F2 = (T*)c->F2;
  T* E = (T*)c->E;
  T* QL = (T*)c->QL;
  T* QR = (T*)c->QR;
  const T gam = (T)c->cfg.gamma;
  const T inv_dx = (T)(1.0 / lv->dx);
  const Work wp = make_work(lv, 4, 4), wq = make_work(lv, 2, 2), wf1 = make_work(lv, 2, 2);
  const Work we1 = make_work(lv, 1, 2), wh = make_work(lv, 1, 1), wf2 = make_work(lv, 1, 1);
  const Work we2 = make_work(lv, 0, 1);
  Work wu = make_work(lv, 0, 0);
  wu.occ = c->occ;
  auto mark = [&](int s) {
    if (ev) (void)hipEventRecord(ev[s], st);
  };
  mark(0);
  if (cfl) {
    k_reset_smax<<<1, 1, 0, st>>>(c->smax);
    k_prim<T, true><<<nblocks(wp), kBlock, 0, st>>>(wp, U, B, W, gam, c->smax, c->flag);
  } else {
    k_prim<T, false><<<nblocks(wp), kBlock, 0, st>>>(wp, U, B, W, gam, c->smax, c->flag);
  }
  mark(1);
  k_ctu_states<T, R><<<nblocks(wq), kBlock, 0, st>>>(wq, W, B, QL, QR, dts, inv_dx, gam);
  mark(2);
  k_flux_q<T, S><<<nblocks(wf1), kBlock, 0, st>>>(wf1, QL, QR, B, F1, gam, c->nfb);
  mark(3);
  k_emf<T><<<nblocks(we1), kBlock, 0, st>>>(we1, F1, W, E);
  mark(4);
  k_half<T><<<nblocks(wh), kBlock, 0, st>>>(wh, U, B, F1, E, dts, inv_dx, gam, W, Bh);
  mark(5);
  k_ctu_correct<T, S><<<nblocks(wf2), kBlock, 0, st>>>(wf2, QL, QR, F1, E, B, Bh, F2, dts, inv_dx, gam, c->nfb);
  mark(6);
  k_emf<T><<<nblocks(we2), kBlock, 0, st>>>(we2, F2, W, E);
  mark(7);
  k_final<T><<<nblocks(wu), kBlock, 0, st>>>(wu, U, B, F2, E, dts, inv_dx);
  mark(8);
}

template <typename T, int S>
void launch_scheme(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev) {
  if (c->cfg.scheme == MHD_VL) launch_step<T, S>(c, lv, dts, cfl, ev);
  else if (c->cfg.recon == MHD_PPM) launch_ctu<T, S, 1>(c, lv, dts, cfl, ev);
  else launch_ctu<T, S, 0>(c, lv, dts, cfl, ev);
}

template <typename T>
void launch_step_t(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev) {
  switch (c->cfg.riemann) {
    case MHD_ROE: launch_scheme<T, 0>(c, lv, dts, cfl, ev); break;
    case MHD_HLLE: launch_scheme<T, 1>(c, lv, dts, cfl, ev); break;
    default: launch_scheme<T, 2>(c, lv, dts, cfl, ev); break;
  }
}

int do_step(mhd_ctx_s* c, const mhd_level* lv, DtSrc dts, bool cfl, hipEvent_t* ev = nullptr) {
  int rc = check_level(c, lv);
  if (rc) return rc;
  rc = ensure_capacity(c, (long long)lv->nx * lv->ny * lv->nz);
  if (rc) return rc;
  rc = build_occupancy(c, lv);
  if (rc) return rc;
  if (c->cfg.prec == MHD_F64) launch_step_t<double>(c, lv, dts, cfl, ev);
  else launch_step_t<float>(c, lv, dts, cfl, ev);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
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
    case MHD_ERR_GHOST_TOO_SMALL: return "ghost width smaller than the stencil of one step";
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
  free_scratch(c);
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
  if (c->cfg.prec == MHD_F64)
    k_prim_to_cons<double><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const double*)W5, (const double*)lv->B,
                                                                  (double*)lv->U, c->cfg.gamma);
  else
    k_prim_to_cons<float><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const float*)W5, (const float*)lv->B,
                                                                 (float*)lv->U, (float)c->cfg.gamma);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int mhd_cfl_dt(mhd_ctx c, const mhd_level* lv, double* dt_host, double* dt_dev) {
  if (!c) return MHD_ERR_INVALID_ARG;
  int rc = check_level(c, lv);
  if (rc) return rc;
  const Work w = make_work(lv, 0, 0);
  k_reset_smax<<<1, 1, 0, c->stream>>>(c->smax);
  if (c->cfg.prec == MHD_F64)
    k_cfl<double><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const double*)lv->U, (const double*)lv->B,
                                                         c->cfg.gamma, c->smax, c->flag);
  else
    k_cfl<float><<<nblocks(w), kBlock, 0, c->stream>>>(w, (const float*)lv->U, (const float*)lv->B,
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
  if (c->cfg.prec == MHD_F64)
    k_sums<double><<<nb, kBlock, 0, c->stream>>>(w, (const double*)lv->U, (const double*)lv->B, c->parts);
  else
    k_sums<float><<<nb, kBlock, 0, c->stream>>>(w, (const float*)lv->U, (const float*)lv->B, c->parts);
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

int mhd_sync(mhd_ctx c) {
  if (!c) return MHD_ERR_INVALID_ARG;
  int flag = 0;
  int rc = read_flag(c, &flag);
  if (rc) return rc;
  return flag ? MHD_ERR_NONPHYSICAL : MHD_OK;
}

}  // extern "C"
