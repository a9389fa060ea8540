/*
 * hy.h -- C ABI of the MI355X (gfx950) 3D Newtonian adiabatic hydro update.
 *
 * The library advances the Euler equations dU/dt + div F(W) = 0 with
 * U = [rho, rho v, E], F = [rho v, rho v v + p, (E + p) v], E = u_g + rho v^2/2,
 * W = [rho, v, u_g] and the gamma-law EOS p = (gamma - 1) u_g (Stone et al.
 * 2024, arXiv:2409.16053: Sec. 3, Eq. 1; Sec. 3.1, Eq. 4). The mesh is a
 * uniform Cartesian grid (Sec. 2, "Cartesian coordinates only") cut into
 * equal MeshBlocks that are processed together as one MeshBlockPack
 * (Sec. 2, "MeshBlockPacks"; "Data locality"), optionally with a box of
 * MeshBlocks refined once (static mesh refinement, hy_config.refine). Each step runs the paper's
 * reconstruct-solve-advance sequence (Sec. 3): ghost zones (Sec. 2,
 * "Boundary conditions"), cons-to-prim, PLM, PPM4, PPMX or WENO-Z
 * reconstruction on primitives, HLLC fluxes in x, y and z, flux divergence
 * and a one- to ten-stage low-storage SSP Runge-Kutta update (method of
 * lines), optionally first-order flux correction, then the CFL time step of
 * Sec. 3, Eq. 3 taken as a minimum over all cells and dimensions.
 *
 * Conventions for every call:
 *  - Status codes are returned; nothing throws or aborts across the ABI.
 *    Argument errors are reported at once. Errors raised on the device
 *    (non-finite state, rho <= 0) are reported by the next hy_query or
 *    hy_get_state. hy_last_error() gives a message for the last failure on
 *    the calling thread.
 *  - Streams are hipStream_t passed as void*; NULL means the default stream.
 *    Calls marked "async" only enqueue work on that stream.
 *  - The library allocates no device memory: every problem lives in a
 *    caller-owned device workspace of hy_workspace_bytes() bytes that must
 *    outlive the handle. The library owns only host-side metadata.
 *  - A handle is used by one thread at a time; distinct handles may be used
 *    concurrently.
 */
#ifndef HY_H
#define HY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hy_problem hy_problem; /* opaque, library-owned host object */

typedef enum {
  HY_OK = 0,
  HY_ERR_ARG = 1,    /* invalid argument or configuration                    */
  HY_ERR_NOMEM = 2,  /* workspace too small or host allocation failed         */
  HY_ERR_HIP = 3,    /* a HIP runtime call failed                             */
  HY_ERR_STATE = 4,  /* a non-finite value or rho <= 0 was seen on the device */
  HY_ERR_BUDGET = 5  /* never returned by the library: the serving layer
                        (serve.py) marks requests it refuses by budget      */
} hy_status;

enum { HY_BC_PERIODIC = 0, HY_BC_OUTFLOW = 1 };
enum { HY_PLM = 0, HY_PPM4 = 1, HY_WENOZ = 2, HY_PPMX = 3 };
enum { HY_FP64 = 0, HY_MIXED = 1 };
#define HY_MAX_REFINE_BOXES 8

/* Problem definition (Sec. 2 mesh and boundaries; Sec. 3 algorithms).
 *  n[3]        global interior cells (nx, ny, nz), each >= 1.
 *  block[3]    MeshBlock interior size; must divide n and be >= the ghost
 *              depth (2 for PLM, 3 for PPM4, PPMX and WENO-Z).
 *  lo[3],hi[3] domain extents; dx_d = (hi_d - lo_d) / n_d > 0.
 *  bc[3][2]    lower/upper boundary per axis: HY_BC_PERIODIC (both sides of
 *              an axis must then be periodic) or HY_BC_OUTFLOW (zero-gradient
 *              copy of the nearest interior cell).
 *  gamma > 1; cfl in (0, 1].
 *  recon       HY_PLM (van Leer limited slopes), HY_PPM4 (Colella &
 *              Woodward 1984 limiters) or HY_WENOZ (fifth-order WENO-Z:
 *              Jiang-Shu smoothness indicators, weights
 *              d_k (1 + (tau5 / (beta_k + 1e-36))^2) with the ratio capped at
 *              1e15, linear weights 1/10, 6/10, 3/10) or HY_PPMX (PPM
 *              with the extremum-preserving limiters of Colella & Sekora:
 *              fourth-order interface values, limited second differences
 *              with C = 1.25), all on primitive variables.
 *  precision   HY_FP64 (all arithmetic in FP64) or HY_MIXED (reconstruction
 *              and the Riemann solve in FP32; cons-to-prim, flux divergence,
 *              the RK accumulation and the time step in FP64; U stays FP64).
 *  fofc        1: first-order flux correction in every RK stage (Sec. 3):
 *              a cell whose updated density or pressure is not positive has
 *              the fluxes on all its faces replaced by LLF fluxes of the
 *              first-order states and its stage update recomputed; 0: off.
 *              Adds 1 byte per (leaf) cell to the workspace. On a refined
 *              mesh the finest level goes first: its flagged cells' faces
 *              change (also in a same-level neighbour leaf), then a coarse
 *              cell is tested with the fine side's fluxes, as they now
 *              stand, on its level faces, and a flagged coarse cell keeps
 *              them there (LLF on its other faces).
 *  rk          order of the low-storage SSP Runge-Kutta integrator (Sec. 3):
 *              1 (forward Euler), 2 (SSPRK(2,2)), 3 (SSPRK(3,3)) or 4
 *              (the ten-stage SSPRK(10,4) of Ketcheson); 0 selects 2. RK3
 *              and RK4 add a third state register to the workspace.
 *  rho_floor, p_floor  floors applied to the primitive state only (U is
 *              never modified by a floor); each firing is counted.
 *  nrefine, refine[HY_MAX_REFINE_BOXES][2][3]  static mesh refinement
 *              (Sec. 2: MeshBlocks of equal cell count on a tree of levels):
 *              a root block (of the n / block grid) is refined once, into 8
 *              blocks of block[] cells at half the cell width, when it lies
 *              in any of the first nrefine boxes, box b covering the root
 *              indices refine[b][0][d] <= index < refine[b][1][d] on every
 *              axis d. nrefine = 0 means no refinement; each box must be
 *              non-empty and inside the root grid; boxes may overlap or
 *              touch (two levels keep face neighbours within one level of
 *              each other for any union). With refinement,
 *              block[] must be even and >= twice the ghost depth. Ghost cells across a level change hold the coarse
 *              mean of the 8 fine cells (restriction) or, on the fine side,
 *              the coarse value plus a quarter of the minmod-limited coarse
 *              slope per axis towards the fine cell (prolongation); the flux
 *              through a coarse face next to 4 fine faces is their mean, so
 *              the update is conservative. The state is then exchanged per
 *              leaf block (hy_leaves, hy_set_state).                        */
typedef struct {
  int32_t n[3];
  int32_t block[3];
  double lo[3], hi[3];
  int32_t bc[3][2];
  double gamma;
  double cfl;
  int32_t recon;
  int32_t precision;
  int32_t fofc;
  int32_t rk;
  double rho_floor, p_floor;
  int32_t nrefine;
  int32_t refine[HY_MAX_REFINE_BOXES][2][3];
} hy_config;

/* Leaf blocks of a configuration's mesh, in the order of the leaf-major
 * state: root blocks with x fastest, then y, then z; a refined root block
 * stands for its 8 children, child x offset fastest, then y, then z. Returns
 * the number of leaves (the root block count without refinement), and, when
 * out != NULL, writes per leaf 4 int32: level (0 or 1) and the block's x, y, z
 * coordinates in blocks of its level. Returns -1 for an invalid configuration
 * (message in hy_last_error). */
int32_t hy_leaves(const hy_config* cfg, int32_t* out);

/* Device bytes one problem needs (the MeshBlockPack of Sec. 2, "Data
 * locality", with no stored ghost cells): two FP64 state registers of
 * 5 x cells doubles each (the step-start state and the RK stage state; three
 * with rk = 3 or 4), a 1024-byte header, and with fofc one byte of flag per
 * cell (per leaf cell with refinement). With refinement each register also
 * holds, per leaf face that meets a different level, the ghost cells there
 * (its ghost slab: ghost depth x the largest block face cells, packed into
 * whole blocks after the leaves), and the workspace holds the leaf, root and
 * face tables.
 * Returns 0 for an invalid configuration (message in hy_last_error). */
size_t hy_workspace_bytes(const hy_config* cfg);

/* Create a problem (a mesh of equal MeshBlocks, Sec. 2) in the caller's
 * device workspace `dev_ws` (256-byte aligned, at least hy_workspace_bytes(cfg)
 * bytes, on the current device; the caller keeps ownership and must keep it
 * alive until hy_destroy). Writes the header synchronously. *out receives the
 * handle. The state is undefined until hy_set_state. Errors: HY_ERR_ARG for an
 * invalid configuration or workspace pointer, HY_ERR_NOMEM for a workspace
 * smaller than hy_workspace_bytes, HY_ERR_HIP if the header upload fails. */
hy_status hy_create(const hy_config* cfg, void* dev_ws, size_t ws_bytes, hy_problem** out);

/* Where a state buffer lives (the `where` argument of hy_set_state and
 * hy_get_state). */
enum {
  HY_HOST = 0,        /* pageable host memory; the call waits for the copy     */
  HY_DEVICE = 1,      /* device memory; the call only enqueues work            */
  HY_HOST_PINNED = 2  /* page-locked host memory; the call only enqueues work
                         and the caller keeps the buffer untouched until the
                         stream has passed this point                         */
};

/* Load the conserved state. U is the GLOBAL interior state as
 * double[5][nz][ny][nx], x fastest, variables rho, Mx, My, Mz, E, located as
 * `where` says. The library scatters it into its MeshBlocks (host data is
 * staged through the problem's second state register) and computes the first
 * time step from it (Eq. 3). On a refined mesh U is instead the leaf-major
 * state double[leaf][5][bz][by][bx] in hy_leaves order, each leaf at its own
 * resolution, copied as is. Clears the bad-state flag. Resets neither t nor
 * the step count. */
hy_status hy_set_state(hy_problem* p, const double* U, int where, void* hip_stream);

/* Store the conserved state into U (same layout as hy_set_state). For
 * HY_HOST and HY_DEVICE it waits for the stream and then reports HY_ERR_STATE
 * if the device flagged a bad state; for HY_HOST_PINNED it only enqueues the
 * copy (check the flag later with hy_query). */
hy_status hy_get_state(hy_problem* p, double* U, int where, void* hip_stream);

/* Advance nsteps >= 0 full time steps (async): the reconstruct-solve-advance
 * update of Sec. 3 in each stage of the configured SSP-RK integrator (method
 * of lines), FOFC after each stage when enabled, and the CFL time step of
 * Eq. 3 for the next step. Each step uses the time step computed on the
 * device at the end of the previous one; the host never reads it back.
 * Errors on the device (non-finite state, rho <= 0) surface at the next
 * hy_query or hy_get_state. */
hy_status hy_advance(hy_problem* p, int32_t nsteps, void* hip_stream);

/* Advance n problems together (async): problem q runs nsteps[q] steps (the
 * MeshBlockPack of Sec. 2 extended to the blocks of many meshes). For every
 * step index, one launch per RK stage covers the tiles of all problems still
 * running that share a (reconstruction, precision) pair; problems of
 * different integrators share the stages they have in common. No problem
 * may appear twice; all must live on the current device. Per-cell
 * arithmetic is identical to hy_advance, so results are bitwise equal to
 * running each problem alone. */
hy_status hy_batch_advance(hy_problem* const* ps, const int32_t* nsteps, int32_t n,
                           void* hip_stream);

/* Same as hy_batch_advance, replayed from a captured HIP graph (async).
 * The first call for a given (problems, nsteps, launch shapes, step parity)
 * captures the launch sequence on `hip_stream` and instantiates it; later calls
 * with the same signature replay it with one graph launch, which removes the
 * per-kernel launch cost for small problems. Every time step stays on the
 * device, so replays need no host input. The graph holds kernel launches only
 * (no memset or copy nodes). `hip_stream` must not be the default (NULL)
 * stream, which cannot be captured. Results are bitwise equal to
 * hy_batch_advance. Graphs that involve a problem are released by its
 * hy_destroy; hy_set_launch on a problem also invalidates them. */
hy_status hy_batch_advance_graph(hy_problem* const* ps, const int32_t* nsteps, int32_t n,
                                 void* hip_stream);

/* Wait for the problem's last stream, then read its time, the time step the
 * next step will take (Eq. 3), the steps taken, the floor hits and the cells
 * corrected by FOFC (Sec. 3; summed over stages; any pointer may be NULL). Returns HY_ERR_STATE
 * if the device flagged a bad state. */
hy_status hy_query(hy_problem* p, double* t, double* dt_next, int64_t* steps,
                   int64_t* floor_hits, int64_t* fofc_cells);

/* Set the simulation time (for resuming from a stored state). */
hy_status hy_set_time(hy_problem* p, double t);

/* Release the handle (not the workspace). Waits for the last stream. */
hy_status hy_destroy(hy_problem* p);

/* Message for the last failed call on this thread ("" if none). */
const char* hy_last_error(void);

/* ---------------- launch shapes and tuning -------------------------------
 * The stage kernel works on x-y tiles of a MeshBlock, marching along z over
 * chunks of kc planes. The compiled variants -- tile shape (tx, ty) and the
 * occupancy (waves per SIMD) the register allocator targets -- are listed by
 * hy_num_variants/hy_variant_info (any out pointer may be NULL); kc is any
 * value >= 1. Results do not depend on the variant or on kc. */
int32_t hy_num_variants(void);
hy_status hy_variant_info(int32_t variant, int32_t* tx, int32_t* ty, int32_t* waves_per_simd);
hy_status hy_set_launch(hy_problem* p, int32_t variant, int32_t kc);
hy_status hy_get_launch(const hy_problem* p, int32_t* variant, int32_t* kc);

/* Time every compiled tile shape and a few z-chunk lengths on this problem's
 * own state, keep the fastest for this problem and cache it for its (block
 * size, recon, precision) class. Each candidate is timed three times and its
 * best time kept. With full_steps == 0 only stage-1 launches are timed, which
 * leave the state unchanged; with full_steps > 0 each timing runs that many
 * complete RK steps (FOFC and counters included), after one warm-up step,
 * which ADVANCES the state (tune a scratch copy). Synchronous. Returns the chosen
 * shape in *variant and *kc (either may be NULL) and its time per stage in
 * *us_per_stage. */
hy_status hy_autotune(hy_problem* p, void* hip_stream, int32_t full_steps, int32_t* variant,
                      int32_t* kc, double* us_per_stage);

/* ---------------- measurement helpers ------------------------------------- */
/* Copy `bytes` (a multiple of 16) from device src to device dst with a plain
 * streaming kernel (async). Used to calibrate HBM byte counters and measure
 * achievable bandwidth. */
hy_status hy_copy_probe(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Record HIP events around hy_advance launches: hy_advance_timed runs nsteps
 * steps on the stream and returns the elapsed device time of the first RK
 * stage's launches and of the later stages' launches (stage 2, and stage 3
 * with RK3) separately (milliseconds), measured with HIP events recorded on
 * that same stream. Synchronous. */
hy_status hy_advance_timed(hy_problem* p, int32_t nsteps, void* hip_stream, double* ms_stage1,
                           double* ms_stage2);

/* ---------------- allocation-free entry point ------------------------------ */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc). Same update
 * as hy_create + hy_set_state(HY_DEVICE) + hy_advance + hy_get_state(HY_DEVICE)
 * with the workspace in a library-owned device array of HY_NOALLOC_MAX_BYTES
 * per GPU (taken when the library is loaded, held until the process ends).
 *  cfg     as for hy_create; refined meshes are not accepted.
 *  U       device pointer, double[5][nz][ny][nx] (the hy_set_state layout):
 *          read as the initial state, overwritten with the state after
 *          nsteps steps.
 *  t0      simulation time of the initial state.
 *  out     NULL, or a device pointer to double[3] that receives the time
 *          after the steps, the next time step and 1.0 if a non-finite state
 *          or rho <= 0 was seen (else 0.0).
 * Async on `hip_stream`; calls no hipMalloc/hipFree, no memset or host copy
 * (graph-capturable). The launch shape is the one hy_create would pick.
 * Errors: HY_ERR_ARG (bad config, NULL U, nsteps < 0, refinement),
 * HY_ERR_NOMEM if hy_workspace_bytes(cfg) exceeds HY_NOALLOC_MAX_BYTES,
 * HY_ERR_HIP. Every call on one GPU uses that GPU's single array, which keeps
 * the last call's contents: calls that overlap on one GPU (other threads,
 * other streams without ordering) race and must not be issued. */
#define HY_NOALLOC_MAX_BYTES (256ull << 20)
hy_status hy_advance_noalloc(const hy_config* cfg, double* U, int32_t nsteps, double t0, double* out,
                             void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* HY_H */
