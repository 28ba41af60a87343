/*
 * mhd.h -- C ABI of libmhd, an MI355X (gfx950) implementation of the
 * unsplit ideal-MHD update of "Magnetohydrodynamics with GAMER"
 * (Zhang, Schive & Chiueh): the per-patch-group finite-volume update with
 * constrained transport of the face-centred magnetic field.
 *
 * Conventions for every entry point
 *   - All functions return an int status: MHD_OK (0) or a negative MHD_ERR_*
 *     code; mhd_strerror() gives text.  No C++ exception crosses the ABI.
 *   - Arguments are validated before any HIP call, so every invalid-argument
 *     path is testable without a GPU.
 *   - All state pointers are DEVICE memory owned by the caller.  The context
 *     owns its scratch (intermediate fluxes, EMFs, half-step state) and frees
 *     it in mhd_finalize().
 *   - Work is enqueued on the HIP stream given to mhd_init() and is
 *     asynchronous unless a function says it synchronises.  One context per
 *     stream; a context is not thread-safe.
 *   - Units: mu = 1 (paper Sec. 2).  Cells are cubic, dx = dy = dz (Sec. 3.1).
 *
 * Data layout of a level (a dense, periodic grid of nx*ny*nz cells):
 *   U  : 5 components (rho, Mx, My, Mz, e), each nz*ny*nx, x fastest --
 *        volume averages at cell centres (Eqs. 6, 11).
 *   B  : 3 components (Bx, By, Bz), each nz*ny*nx -- face-area averages
 *        (Eq. 14); Bx[k][j][i] sits on the lower x-face of cell (i,j,k),
 *        By on the lower y-face, Bz on the lower z-face.
 *   Element type: double for MHD_F64, float for MHD_F32 and MHD_F32_MIXED.
 *   MHD_F32_MIXED additionally keeps the total energy in double in E64
 *   (nz*ny*nx doubles); the e component of U is then ignored on input and
 *   mirrored (rounded to float) on output.
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MHD_ABI_VERSION 4

/* status codes */
#define MHD_OK 0
#define MHD_ERR_INVALID_ARG -1
#define MHD_ERR_UNSUPPORTED -2
/* -3 is not used: ghost zones are the level's own cells around a listed
 * group (see mhd_level), so a caller cannot hand over too few of them */
#define MHD_ERR_HIP -4
#define MHD_ERR_NONPHYSICAL -5
#define MHD_ERR_NO_DEVICE -6
#define MHD_ERR_OUT_OF_MEMORY -7
#define MHD_ERR_SCRATCH_LIMIT -8   /* mhd_step_noalloc: the level needs more than MHD_NOALLOC_SCRATCH_BYTES */

/* size of the static stage scratch of mhd_step_noalloc, per device */
#define MHD_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* unsplit integrators, paper Sec. 3.2 */
enum { MHD_VL = 0, MHD_CTU = 1 };
/* reconstruction, Sec. 3.2 (CTU step 1, VL step 4); PLM limiter is minmod */
enum { MHD_PLM = 0, MHD_PPM = 1 };
/* Riemann solvers, Sec. 3.2 (CTU step 2); MLP = learned flux with HLLD fallback */
enum { MHD_ROE = 0, MHD_HLLE = 1, MHD_HLLD = 2, MHD_MLP = 3 };
/* arithmetic */
enum { MHD_F64 = 0, MHD_F32 = 1, MHD_F32_MIXED = 2 };

typedef struct mhd_ctx_s* mhd_ctx;

typedef struct {
  int scheme;        /* MHD_VL or MHD_CTU */
  int recon;         /* MHD_PLM or MHD_PPM */
  int riemann;       /* MHD_ROE, MHD_HLLE, MHD_HLLD, MHD_MLP */
  int prec;          /* MHD_F64, MHD_F32, MHD_F32_MIXED */
  double gamma;      /* adiabatic index, 5/3 in the paper (Sec. 5) */
  double courant;    /* Courant factor, 1/2 in the paper (Sec. 5), summed over directions */
  double beta_fp64;  /* MHD_F32_MIXED: cells with 2p/|B|^2 below this recover p in double */
  double mlp_dp;     /* MHD_MLP: relative pressure jump above which HLLD is used (negative: every face) */
  double mlp_drho;   /* MHD_MLP: relative density jump above which HLLD is used (negative: every face) */
} mhd_config;

/* One level: a dense periodic grid plus an optional list of patch groups.
 * groups == NULL (or n_groups == 0) updates every cell.  Otherwise only the
 * cells of the listed groups are updated; each entry is the origin (i0, j0,
 * k0) of a group of group_edge^3 cells (paper Sec. 4: eight patches of N^3
 * cells form a group of (2N)^3), and the cells outside the listed groups act
 * as ghost zones that the caller fills (e.g. by prolongation from the coarser
 * level).  All grid dimensions must then be multiples of group_edge. */
typedef struct {
  int nx, ny, nz;       /* cells; each >= 4 */
  double dx;            /* cell width (Sec. 3.1: x_i = (i + 1/2) dx) */
  int n_groups;         /* number of entries in groups */
  int group_edge;       /* cells per group edge (16 = 2 patches of 8^3) */
  const int* groups;    /* device int32[3 * n_groups] origins, or NULL */
  void* U;              /* device, 5 * N elements, see layout above */
  void* B;              /* device, 3 * N elements */
  double* E64;          /* device, N doubles, MHD_F32_MIXED only */
  const int* n_groups_dev; /* optional device int: the number of listed groups
                              actually used (<= n_groups, which is then the
                              capacity); lets a captured graph replay after
                              the list changed */
} mhd_level;

/* Ghost width a patch group needs for one full step of the given integrator
 * and reconstruction (stencil count: 3 for PLM, 4 for PPM): the cells around
 * a listed group that must hold valid ghost data (mhd_prolong fills them). */
int mhd_required_ghost(int scheme, int recon);

/* Device bytes the context's stage scratch takes to update lv (in
 * *bytes): W, Bh, F, E (35 words per scratch cell; CTU adds QL, QR, F2: 98;
 * the learned flux needs no more) times the scratch cells (the level's cells,
 * or (groups + 2) boxes of (edge + 2 ghost)^3 cells for a group list), plus
 * the group occupancy map.  The context allocates this on the first update
 * of a level that needs more than it holds; the time-mean registers of
 * mhd_accumulate_registers (24 words per scratch cell) come on top.  No
 * HIP call. */
int mhd_workspace_bytes(mhd_ctx ctx, const mhd_level* lv, size_t* bytes);

/* Validate cfg and create a context bound to hip_stream (a hipStream_t, or
 * NULL for the default stream) on the current device. */
int mhd_init(const mhd_config* cfg, void* hip_stream, mhd_ctx* out);
int mhd_finalize(mhd_ctx ctx);

/* Validate a level description (no HIP call).  ctx may be NULL, which skips
 * the checks that depend on the context's precision. */
int mhd_check_level(mhd_ctx ctx, const mhd_level* lv);

/* Conserved state from primitive cell fields (Eq. 5; cell-centred field is
 * the mean of the two opposite faces).  W5: device, 5*N elements of the
 * level's type (rho, vx, vy, vz, p).  Writes lv->U (and E64 when mixed). */
int mhd_prim_to_cons(mhd_ctx ctx, const mhd_level* lv, const void* W5);

/* CFL time step, Sec. 3.2: dt = courant * dx / max over cells of
 * sum_d (|v_d| + c_f,d).  Computed and reduced in double.  dt_dev (device
 * double*) receives it without a host sync; dt_host (host double*) syncs.
 * Either may be NULL.  A cell with rho <= 0 or p <= 0 gives
 * MHD_ERR_NONPHYSICAL (host path) or sets the context's sticky flag. */
int mhd_cfl_dt(mhd_ctx ctx, const mhd_level* lv, double* dt_host, double* dt_dev);

/* One full step of length dt (paper Sec. 3.2: CTU steps 1-8 or VL steps 1-7),
 * updating lv->U and lv->B in place.  Asynchronous. */
int mhd_step(mhd_ctx ctx, const mhd_level* lv, double dt);

/* Same, with dt read from device memory at run time (graph-capturable). */
int mhd_step_devdt(mhd_ctx ctx, const mhd_level* lv, const double* dt_dev);

/* mhd_step_devdt for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the stage scratch taken from a static
 * device array of MHD_NOALLOC_SCRATCH_BYTES (64 MiB) that each device holds
 * from its first mhd_init until the process ends; no hipMalloc, hipFree or
 * allocating library call.  A level whose scratch (mhd_workspace_bytes)
 * exceeds the array returns MHD_ERR_SCRATCH_LIMIT before any HIP call: e.g.
 * FP32 CTU up to about 171k cells (48^3), FP64 VL up to about 240k (32^3
 * and beyond).  Every call on a device shares that device's array, which
 * keeps the last call's contents (each step writes every scratch value it
 * reads; the group occupancy map is cleared by a kernel): calls that
 * overlap on one device race, so serialise them, e.g. on one stream.  The
 * fluxes and EMFs stay in the static array, so mhd_correct and
 * mhd_accumulate_registers (which read the context's scratch) do not follow
 * this step. */
int mhd_step_noalloc(mhd_ctx ctx, const mhd_level* lv, const double* dt_dev);

/* CFL step plus update in one call, with no host synchronisation: computes
 * dt from the current state on the device, writes it to dt_dev (device,
 * may be NULL) and adds it to t_dev (device, may be NULL). */
int mhd_advance(mhd_ctx ctx, const mhd_level* lv, double* dt_dev, double* t_dev);

/* mhd_advance through a HIP graph: the first call for a level description
 * (and the same dt_dev/t_dev) captures the step's kernels on the context's
 * stream and instantiates the graph; later calls replay it.  dt comes from
 * the on-device CFL reduction and a group count from n_groups_dev, so a
 * replay needs no host work.  A different description re-captures. */
int mhd_advance_graph(mhd_ctx ctx, const mhd_level* lv, double* dt_dev, double* t_dev);

/* Launch shape of the stage kernels (the batched level update):
 *   blocks_per_cu      at most this many blocks per compute unit walk the
 *                      work with a grid-wide stride (0 = one thread per work
 *                      item, no cap);
 *   threads_per_block  64 .. 512, a multiple of 64 (0 = 256); the learned
 *                      flux's network kernels keep 256;
 *   batch_groups       with a group list, the stages between the primitive
 *                      pass (which also reduces the CFL maximum over the whole
 *                      list) and the final update run batch by batch, each
 *                      batch of at most this many groups through all of them,
 *                      so its intermediates can stay in the caches (paper
 *                      Sec. 4 sends patch groups to the GPU in batches);
 *                      0 = the whole list in one launch per stage.
 *   lds_tiles          CTU with PPM, step 1 (reconstruction and characteristic
 *                      tracing): 0 = one thread per cell, each computing its
 *                      own stencil's MC slopes and PPM interface values;
 *                      1 = blocks of 16 x 4 x 4 cells (20 x 5 x 5 on the item
 *                      boxes of 16^3 groups; other group sizes keep the
 *                      per-cell form) that stage their primitives with two
 *                      ghost layers per direction in LDS and compute each
 *                      slope and interface value once (fewer VALU
 *                      instructions, but block barriers between the stages);
 *                      other configurations ignore it.  The same arithmetic
 *                      compiled in another code layout: results agree with
 *                      the per-cell form to rounding, not bit for bit.
 * For a given lds_tiles, every shape gives bit-identical results.  Drops any
 * captured graph.  The reduction kernels of mhd_divB and mhd_sums and the
 * AMR transfer kernels keep their fixed shape. */
int mhd_set_launch(mhd_ctx ctx, int blocks_per_cu, int threads_per_block, int batch_groups, int lds_tiles);

/* Minimum of scale times the level's CFL time step and *dt_dev, written to
 * *dt_dev, without a host sync: scale 1 on every level gives a shared step;
 * scale 2^l on level l gives the root step of a hierarchy whose level l takes
 * 2^l sub-steps (paper Sec. 3.3, adaptive time steps).  scale must be
 * positive and finite. */
int mhd_cfl_dt_min(mhd_ctx ctx, const mhd_level* lv, double scale, double* dt_dev);

/* Refinement / derefinement operation of paper Sec. 3.3, step 1: the group
 * list of the level above `coarse`.  A candidate fine group (fine_edge^3
 * fine cells, a block of fine_edge/2 coarse cells per axis) is listed when
 * the criterion |curl B| dx / |B| > threshold holds in a coarse cell of its
 * block widened by `buffer` coarse cells (periodic); it is decided as
 * (jx^2 + jy^2 + jz^2) > threshold^2 (bx^2 + by^2 + bz^2), b the cell-centred
 * field and j = dx curl b by central differences, without contraction.
 * When `coarse` has a group list, only candidates inside listed coarse
 * groups qualify (proper nesting; coarse->group_edge must be a multiple of
 * fine_edge/2).  groups_out (device int32[capacity][3], fine-cell origins)
 * receives the listed candidates in increasing (z, y, x) order, at most
 * `capacity` of them; *count_dev = min(*wanted_dev, capacity) and
 * *wanted_dev = the number that qualified (device int32 each): the caller
 * checks *wanted_dev <= capacity.  0 <= buffer <= fine_edge/2; the coarse
 * dimensions must be multiples of fine_edge/2.  Not for MHD_F32_MIXED. */
int mhd_regrid_flag(mhd_ctx ctx, const mhd_level* coarse, double threshold, int buffer, int fine_edge,
                    int* groups_out, int capacity, int* count_dev, int* wanted_dev);

/* Refinement / derefinement operation of paper Sec. 3.3, step 2: data of
 * the fine groups created by a new list.  fine_new and fine_old describe
 * the same fine arrays (U, B) with the new and the previous group list
 * (fine_old NULL or without a list: nothing existed).  Groups of the new
 * list that the old list does not hold take cells, lower faces and upper
 * boundary faces from `coarse` by the prolongation of mhd_prolong (Balsara's
 * reconstruction, conservative energy); a face whose far side is a fine
 * cell of an old group keeps its value, and the twist of those kept faces
 * (the part of the four values beyond a mean and two slopes) is returned
 * through the created parent's mid-plane faces so that each created cell
 * keeps its parent's divergence.  Everything else is left untouched: old
 * groups keep their data, removed groups need nothing (their parent cells
 * hold the restricted data).  Call it after mhd_restrict so that the coarse
 * faces next to old groups are their fine means.  Not for MHD_F32_MIXED. */
int mhd_prolong_new_groups(mhd_ctx ctx, const mhd_level* coarse, const mhd_level* fine_new,
                           const mhd_level* fine_old);

/* *dt_fine = *dt_coarse / parts on the device (the step of a level that
 * sub-cycles parts times inside its parent's step); parts >= 1. */
int mhd_dt_subdivide(mhd_ctx ctx, const double* dt_coarse, int parts, double* dt_fine);

/* AMR support between a coarse level and a fine level of twice its cells per
 * dimension (paper Sec. 3.3).  The coarse level is read (prolong) or written
 * (restrict) as a whole grid; its own group list, if any, is ignored.
 * mhd_prolong: with no fine group list, fills the whole fine level from the
 * coarse one; with a list, fills the ghost halo (halo cells around each listed
 * group, plus one above) of the listed groups: cells outside every listed
 * group, and faces whose two cells are both outside.  Cell data: each
 * conserved component of a child is the parent's plus a quarter of the
 * minmod-limited slope of the parent's neighbours along each axis (the eight
 * children average to the parent), the energy adding
 * (|b_child|^2 - <|b|^2>)/2 over the eight children; a parent whose children
 * would not all keep rho > 0 and p > 0 injects rho and M with the same energy
 * shift (and keeps its pressure where even that would not be positive, not
 * conservative).  The slopes read the parent's neighbours, so the coarse
 * level needs valid data one cell around the prolonged region.  Face field: Balsara's
 * divergence-free reconstruction -- fine faces on a coarse face follow its
 * MC-limited linear profile, fine faces inside a coarse cell the quadratic
 * field matching the cell's six face profiles with no linear divergence
 * terms -- so each fine cell's divergence equals its parent's and the fine
 * faces on a coarse face average to it.
 * mhd_restrict: coarse cells under the listed fine groups (all cells with no
 * list) take the mean of their eight children, and the coarse faces of those
 * cells, including the faces on the boundary of the refined region, the mean
 * of the four fine faces on them.  Not for MHD_F32_MIXED. */
int mhd_prolong(mhd_ctx ctx, const mhd_level* coarse, const mhd_level* fine, int halo);

/* mhd_prolong from the coarse data interpolated linearly in time,
 * old + alpha (new - old), with coarse_old the parent's state at the start of
 * its step and coarse its state at the end: the ghosts of a fine level at an
 * intermediate time of a sub-cycled step (paper Sec. 3.3: finer levels are
 * evolved until they reach the parent's time).  alpha in [0, 1]; alpha = 0
 * reads coarse_old alone, alpha = 1 coarse alone (coarse_old may then be
 * NULL).  coarse_old must have coarse's shape and cell width; it is read
 * only. */
int mhd_prolong_time(mhd_ctx ctx, const mhd_level* coarse_old, const mhd_level* coarse, double alpha,
                     const mhd_level* fine, int halo);

/* Time-averaged coarse-fine registers of a sub-cycled level: R = weight S
 * (reset != 0) or R + weight S, with S the final fluxes and EMFs of ctx's
 * last update of lv, on the boundary faces and edges of each listed group
 * (every face and edge without a list): the only ones a correction reads,
 * given that the groups of the finer level lie inside listed groups of
 * this one.  After the sub-steps of one parent step
 * (weight 1/parts each, the first with reset), mhd_correct with
 * fine_registers = 1 corrects the parent with the time mean.  The registers
 * live in ctx (21 + 3 arrays of its scratch size, allocated on the first
 * reset call that needs them; a call with reset == 0 before that fails with
 * MHD_ERR_INVALID_ARG).  Not for MHD_F32_MIXED. */
int mhd_accumulate_registers(mhd_ctx ctx, const mhd_level* lv, double weight, int reset);
int mhd_restrict(mhd_ctx ctx, const mhd_level* fine, const mhd_level* coarse);

/* Correction operation of paper Sec. 3.3 across a coarse-fine interface,
 * after the coarse level took one step *dt_dev (device double) and the fine
 * level the same time span, in one step (fine_registers = 0: the fine
 * values are those of ctx_fine's last update) or in sub-steps
 * (fine_registers = 1: the time mean kept by mhd_accumulate_registers): a
 * coarse cell outside the refined region that shares a face with
 * it replaces the coarse flux through that face by the mean of the four fine
 * fluxes; a coarse face with both cells outside takes the CT update of the
 * EMF differences (mean of the two fine EMFs minus the coarse EMF) on its
 * edges that touch the refined region.  Cells and faces inside the refined
 * region are left to mhd_restrict (call it afterwards).  Then the coarse
 * context's stored final fluxes and EMFs on the faces and edges of refined
 * cells become the fine means, so that correcting the next coarser level
 * across a shared interface uses the finest values (no proper-nesting
 * requirement); a sub-cycled coarse level accumulates its registers after
 * this call.  ctx_coarse and
 * ctx_fine must be the contexts that ran those updates (their stage scratch
 * holds the final fluxes and EMFs), on the same stream, with the same scheme
 * and precision; the fine groups must lie inside listed coarse groups when
 * the coarse level has a list.  Not for MHD_F32_MIXED. */
int mhd_correct(mhd_ctx ctx_coarse, const mhd_level* coarse, mhd_ctx ctx_fine, const mhd_level* fine,
                const double* dt_dev, int fine_registers);

/* Discrete divergence of Eq. 16 in double: max |div B| and the mean of
 * |div B| over the level's cells.  Synchronises. */
int mhd_divB(mhd_ctx ctx, const mhd_level* lv, double* max_abs, double* l1);

/* Volume totals in double with a fixed-order reduction (bitwise
 * reproducible): mass, Mx, My, Mz, total energy, magnetic energy (cell-centred
 * field), kinetic energy.  Synchronises. */
int mhd_sums(mhd_ctx ctx, const mhd_level* lv, double out[7]);

/* Number of faces where the Roe solver fell back to HLLE since the last
 * call (resets the counter).  Synchronises. */
int mhd_fallback_count(mhd_ctx ctx, long long* count);

/* Stage timing: runs nrep steps exactly as mhd_advance does (they advance
 * the level), recording HIP events on the context's stream between the stage
 * kernels, and writes the mean milliseconds of each stage to stage_ms
 * (host array of mhd_num_stages() doubles).  Synchronises. */
int mhd_profile_step(mhd_ctx ctx, const mhd_level* lv, int nrep, double* stage_ms);
int mhd_num_stages(mhd_ctx ctx);
/* Name of stage s (static string), or NULL when out of range. */
const char* mhd_stage_name(mhd_ctx ctx, int stage);

/* ---- learned interface flux (an addition to the paper's method) ----
 * A 15 -> 64 -> 64 -> 7 GELU network replaces HLLD (paper Sec. 3.2, CTU
 * step 2 names HLLD) at interfaces whose relative pressure and density jumps
 * are below cfg.mlp_dp / cfg.mlp_drho; stronger jumps keep HLLD.  Inputs (15)
 * come from the face-frame primitive states w = (rho, vn, vt1, vt2, p, Bt1,
 * Bt2) on both sides and Bn, in units sc = (rho0, v0, v0, v0, p0, B0, B0) with
 * rho0 = mean rho, p0 = mean p, v0 = sqrt(p0/rho0), B0 = sqrt(p0): with
 * d = (wR - wL)/sc and s = |d|, x = (mean rho/rho0, mean (vn, vt1, vt2)/v0,
 * s, mean (Bt1, Bt2)/B0, d/s, Bn/B0).  Outputs: the dissipative part of the
 * flux, i.e. the flux minus the central flux (F(wl) + F(wr))/2 computed
 * exactly (Eq. 7), divided by s (rho0 v0, p0, p0, p0, p0 v0, B0 v0, B0 v0).
 * BF16 operands, FP32 accumulation (MFMA).  Parameters: FP32 device
 * array of mhd_mlp_num_params() values, packed W1[15][64] b1[64] W2[64][64]
 * b2[64] W3[64][7] b3[7] ([in][out], row-major).  Usable with MHD_CTU in
 * MHD_F32 or MHD_F32_MIXED; mhd_fallback_count() then counts HLLD faces. */
int mhd_mlp_num_params(void);
/* Load inference weights (device params) into the context; required before a
 * step with MHD_MLP. */
int mhd_mlp_set_weights(mhd_ctx ctx, const float* params_dev);
/* Y[n][7] = network(X[n][15]) for normalised features (device arrays). */
int mhd_mlp_forward(mhd_ctx ctx, const float* params_dev, const float* X_dev, int n, float* Y_dev);
/* Gradient of sum(dY * network(X)) with respect to the parameters. */
int mhd_mlp_backward(mhd_ctx ctx, const float* params_dev, const float* X_dev, const float* dY_dev, int n,
                     float* grads_dev);
/* One Adam step (beta 0.9, 0.999, eps 1e-8, bias-corrected at step >= 1) on
 * the mean squared error over the batch; params, adam_m, adam_v, grads are
 * device arrays of mhd_mlp_num_params() floats, loss_dev (may be NULL)
 * receives the batch loss before the update. */
int mhd_mlp_train_step(mhd_ctx ctx, float* params_dev, float* adam_m, float* adam_v, float* grads_dev, int step,
                       const float* X_dev, const float* T_dev, int n, float lr, float* loss_dev);
/* Captured samples S[n][22] = (wl[7], wr[7], bn, flux[7]) -> features
 * X[n][15], normalised targets T[n][7] = (flux - central flux) / (s scales)
 * and flags: bit 0 = strong jump (HLLD at run time), bit 1 = jump size s below
 * 1e-4, where the target is dominated by float round-off. */
int mhd_mlp_prepare(mhd_ctx ctx, const float* samples_dev, int n, float* X_dev, float* T_dev, int* flags_dev);
/* Learned flux with HLLD fallback for n interfaces S[n][15] = (wl[7], wr[7],
 * bn) in the face frame -> flux[n][7]; used_hlld[n] = 1 where HLLD was used. */
int mhd_mlp_face_flux(mhd_ctx ctx, const float* states_dev, int n, float* flux_dev, int* used_hlld_dev);
/* Interface capture for training data: while set, every stride-th face of the
 * CTU Riemann stages writes (wl, wr, bn, flux) to buf_dev[cap][22] (FP32
 * forms only; in the learned-flux form the flux the face used, network or
 * HLLD); *count_dev counts attempted writes (writes stop at cap).
 * buf_dev == NULL turns capture off.  Every call drops the graph captured by
 * mhd_advance_graph (the capture settings are arguments of its kernels), so
 * the next mhd_advance_graph captures again. */
int mhd_set_capture(mhd_ctx ctx, float* buf_dev, long long cap, unsigned long long* count_dev, int stride);

/* Wait for the context's stream and report sticky device-side errors
 * (MHD_ERR_NONPHYSICAL). */
int mhd_sync(mhd_ctx ctx);

const char* mhd_strerror(int status);
int mhd_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MHD_H */
