/*
 * pkhydro.h -- C-ABI of the MI355X (gfx950) hot path of Parthenon-hydro's
 * block-AMR Euler cycle.
 *
 * The problem statement these calls follow (Parthenon, arXiv:2202.12309):
 *   - Sec. 2.1: the domain is tiled by same-size MeshBlocks that are the
 *     leaves of an oct-tree; each leaf has a refinement level and a logical
 *     location; every point of the domain lies in exactly one leaf; blocks
 *     may be split into 8 children or 8 siblings merged, and the tree is
 *     rebuilt when that happens.
 *   - Sec. 3.1/3.6: block data lives in device memory; one kernel covers all
 *     blocks of a pack.
 *   - Sec. 3.7: ghost zones are filled from neighbouring blocks (copy at the
 *     same level, restriction from finer, prolongation from coarser) and
 *     fluxes are corrected at fine-coarse faces.
 *   - Sec. 3.8: derefinement is only applied periodically.
 *   - Sec. 3.10: global reductions (CFL timestep, sums).
 *   - Sec. 4.1: the update is a two-stage second-order finite-volume scheme
 *     with piecewise-linear reconstruction and the HLLE Riemann solver.
 *
 * Conventions for every call:
 *   - Return value: PKH_OK (0) or a negative PKH_E* code; the message of the
 *     last failure on the calling thread is returned by pkh_last_error().
 *   - Unphysical states (rho <= 0, P <= 0 or non-finite values) are latched
 *     by the kernels in a device word and reported as PKH_EPHYS by the next
 *     call that synchronises (download, totals, get_time, sync). The latch is
 *     cleared by pkh_state_upload.
 *   - A mesh handle is not thread-safe. All device work is enqueued on the
 *     handle's HIP stream, in call order; calls that return host data
 *     synchronise that stream.
 *   - The library owns the device arrays it allocates; the caller owns every
 *     host array and every device pointer it passes in.
 *   - State layout ("upload layout"): conserved variables
 *     (rho, M1, M2, M3, E), double precision, [nblocks][5][n3][n2][n1] with
 *     x (index 1) fastest, active cells only, blocks in storage order
 *     (pkh_mesh_blocks).
 */
#ifndef PKHYDRO_H
#define PKHYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pkh_status {
  PKH_OK = 0,
  PKH_EINVAL = -1,   /* bad argument or configuration */
  PKH_ETILING = -2,  /* leaves overlap or leave a gap */
  PKH_EBALANCE = -3, /* neighbouring leaves differ by more than one level */
  PKH_ENOMEM = -4,   /* device allocation failed */
  PKH_EHIP = -5,     /* a HIP runtime call failed */
  PKH_EPHYS = -6,    /* unphysical state latched by a kernel */
  PKH_ESTATE = -7    /* call not valid in the handle's current state */
};

/* Boundary kind of a domain face. PERIODIC: the face is glued to the
   opposite one (both faces of a direction periodic or neither). OUTFLOW:
   a ghost cell beyond the face takes the value of the nearest cell inside
   (zero gradient). REFLECT: a ghost cell takes the value of its mirror
   image across the face with the momentum normal to the face negated.
   Beyond a wall the image is evaluated like any ghost cell there (copy,
   restriction or prolongation), and a prolongation stencil that reaches
   past a wall at the coarse level uses the coarse image cells. */
enum { PKH_BC_PERIODIC = 0, PKH_BC_OUTFLOW = 1, PKH_BC_REFLECT = 2 };
enum { PKH_RECON_DC = 0, PKH_RECON_PLM = 1 };
enum { PKH_LIMITER_MC = 0 };
/* pkh_config.flags */
enum {
  PKH_FLAG_GRAPH = 1u,     /* replay captured cycles with hipGraphs */
  /* Store the state in FP32 (half the bytes): every stage widens its inputs
     to FP64, computes in FP64 and rounds its output once to the nearest
     float when storing it; the CFL and total reductions run in FP64 on the
     stored values. Single-level periodic meshes with nblock[0] of 16 or 32;
     no tape, batch, partition or refinement indicator. Upload rounds the
     FP64 input to float, download widens. */
  PKH_FLAG_FP32_STATE = 2u
};

/* Mesh configuration.
 *   nroot[d]   level-0 cells along d; a multiple of nblock[d].
 *   nblock[d]  cells per block along d (same for every block, Sec. 2.1).
 *              nblock[0] is 8, 16, 32 or 64; nblock[1] is a multiple of
 *              the default row tile (8 for nblock[0] <= 32, 4 for 64);
 *              nblock[2] is at least 4; with max_level > 0 every nblock[d]
 *              is even and at least 8.
 *   nghost     must be 2 (PLM needs two cells on each side of a face).
 *   max_level  deepest refinement level (0..7).
 *   xmin/xmax  domain extent; gamma the ideal-gas ratio; cfl the Courant
 *              number of the timestep.
 *   bc[6]      boundary kind per face (x-, x+, y-, y+, z-, z+), PKH_BC_*.
 *              The reverse mode and batches take periodic meshes only.
 *   stage1_recon PKH_RECON_DC (predictor-corrector, default) or PKH_RECON_PLM.
 *   limiter    PKH_LIMITER_MC.
 *   regrid_every  informational: the caller's derefinement cadence.
 *   flags      PKH_FLAG_* bits. */
typedef struct {
  int32_t nroot[3];
  int32_t nblock[3];
  int32_t nghost;
  int32_t max_level;
  double xmin[3];
  double xmax[3];
  double gamma;
  double cfl;
  int32_t bc[6];
  int32_t stage1_recon;
  int32_t limiter;
  int32_t regrid_every;
  uint32_t flags;
} pkh_config;

/* Logical location of a leaf (Sec. 2.1): its level and its block
   coordinates at that level, 0 <= lx_d < (nroot[d]/nblock[d]) << level. */
typedef struct {
  int32_t level, lx1, lx2, lx3;
} pkh_loc;

/* Device-memory callbacks. alloc returns device memory of at least `bytes`
   usable on `stream` (NULL on failure); free releases it. The library may
   free memory that work already queued on `stream` still uses: free must
   release it in stream order (as hipFreeAsync or a stream-ordered caching
   allocator does). Pass NULL for both to use hipMalloc / hipFree. */
typedef void *(*pkh_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*pkh_free_fn)(void *ptr, void *stream, void *ctx);

typedef struct pkh_mesh pkh_mesh;

/* Create a mesh from a leaf list (Sec. 2.1). Validates that the leaves tile
   the domain exactly once (PKH_ETILING) and that leaves touching across a
   face, edge or corner differ by at most one level (PKH_EBALANCE). Leaves
   are stored in Morton (Z) order of their deepest-level corner; read the
   order back with pkh_mesh_blocks. `hip_stream` (a hipStream_t, may be NULL
   for the null stream) receives all of the handle's work. The state is
   zero until uploaded. */
int pkh_mesh_create(const pkh_config *cfg, const pkh_loc *blocks, int64_t nblocks,
                    void *hip_stream, pkh_alloc_fn alloc, pkh_free_fn free_fn,
                    void *alloc_ctx, pkh_mesh **out);

/* Synchronise the stream and release every device array of the handle. */
int pkh_mesh_destroy(pkh_mesh *mesh);

/* Current leaves in storage order. Writes min(cap, count) entries to out
   (out may be NULL when cap is 0) and the count to *n. */
int pkh_mesh_blocks(const pkh_mesh *mesh, pkh_loc *out, int64_t cap, int64_t *n);

/* Copy a state in the upload layout into the mesh (asynchronous on the
   stream when src is device memory; a host src is staged and the call
   returns after the copy is enqueued and the host buffer is consumed).
   Marks ghosts and the timestep stale; they are recomputed by
   pkh_exchange_boundaries or at the start of pkh_step. */
int pkh_state_upload(pkh_mesh *mesh, const double *src, int32_t src_on_device);

/* Copy the active state out in the upload layout; synchronises. */
int pkh_state_download(pkh_mesh *mesh, double *dst, int32_t dst_on_device);

/* Fill every ghost zone from the leaves' active data (Sec. 3.7: copy,
   restriction, prolongation, all 26 neighbour regions; periodic wrap or
   the wall images of PKH_BC_*) and recompute the CFL timestep from the
   active data (Sec. 3.10). Inside pkh_step the kernels read a same-level
   neighbour's cells directly and only the face ghost regions that cross a
   level jump or a wall are refilled after each stage; the other ghost
   cells keep the values of the last full fill. */
int pkh_exchange_boundaries(pkh_mesh *mesh);

/* Advance n_cycles full cycles (Sec. 4.1). Each cycle:
     dt  = CFL timestep of the current state, clamped to t_end - t when
           t_end is finite;
     U*  = U^n - dt/2 D(U^n)   (donor-cell or PLM faces, HLLE fluxes);
     on multilevel meshes, fine-coarse flux correction; the ghost faces
     across level jumps and walls of U*;
     U^{n+1} = U^n - dt D_PLM(U*) (MC-limited PLM on primitives, HLLE);
     the same for U^{n+1}; t += dt; the next dt is reduced on the device.
   Halo cells at same-level faces are read from the neighbour's active
   cells (the results equal those of a full ghost exchange after each
   stage).
   No host synchronisation. With PKH_FLAG_GRAPH the cycles are replayed
   from a captured hipGraph. */
int pkh_step(pkh_mesh *mesh, int32_t n_cycles, double t_end);

/* Simulation time, the CFL timestep the next cycle will use (before any
   t_end clamp) and the cycle count; synchronises. */
int pkh_get_time(pkh_mesh *mesh, double *t, double *dt, int64_t *cycle);
/* Set time and cycle (resume); the timestep is recomputed at the next step. */
int pkh_set_time(pkh_mesh *mesh, double t, int64_t cycle);

/* Per-leaf refinement flags in storage order: -1 derefine, 0 keep,
   +1 refine (Sec. 2.1, Sec. 3.8). Applied by pkh_regrid. */
int pkh_set_refinement_flags(pkh_mesh *mesh, const int8_t *flags, int64_t n);

/* Device refinement indicators (the paper leaves the criterion to the
   application; Sec. 2.1, Sec. 3.8). Per leaf, eta = the largest relative
   jump |q(i+e_d) - q(i-e_d)| / (q(i+e_d) + q(i-e_d)) over active cells i
   and directions d (neighbour cells across a block face as for the
   stencil) of q = pressure (PKH_JUMP_PRESSURE: shocks, blasts) or density
   (PKH_JUMP_DENSITY: contact and shear layers, where pressure is smooth);
   evaluated without FMA contraction and with correctly rounded division.
   Sets the mesh's flags to +1 where eta > refine_above, -1 where eta <
   derefine_below, else 0 (as pkh_set_refinement_flags would) and, when
   non-NULL, copies them to flags_out[n leaves] and eta to eta_out[n leaves]
   (host arrays, caller owned). PKH_EINVAL for an unknown quantity or if
   derefine_below > refine_above. Synchronises. */
enum { PKH_JUMP_PRESSURE = 0, PKH_JUMP_DENSITY = 1 };
int pkh_flag_jump(pkh_mesh *mesh, int32_t quantity, double refine_above, double derefine_below,
                  int8_t *flags_out, double *eta_out);
/* pkh_flag_jump with PKH_JUMP_PRESSURE. */
int pkh_flag_pressure_jump(pkh_mesh *mesh, double refine_above, double derefine_below,
                           int8_t *flags_out, double *eta_out);

/* Apply the flags: +1 splits a leaf below max_level into 8 children; a
   refinement that would break 2:1 also refines the touching coarser
   leaves, to a fixed point; 8 siblings all flagged -1 (none refining) merge
   when the merged block keeps 2:1. New children get the prolongation of
   the composite field at the parent's level, a merged parent the
   restriction of its children. The tree and all tables are rebuilt on the
   host, the data moved on the device, the ghost faces the cycle reads
   (across level jumps, walls and remote faces) filled and the timestep
   recomputed; pkh_exchange_boundaries fills every ghost region.
   Flags are cleared. Synchronises. PKH_ESTATE while a tape or a batch
   holds the mesh (they keep pointers into its leaf layout): destroy them
   first. */
int pkh_regrid(pkh_mesh *mesh);

/* Conserved totals sum_leaves sum_active U_v dV (Sec. 3.10 reduction);
   fixed-order device reduction; synchronises. out[5]. */
int pkh_conserved_totals(pkh_mesh *mesh, double out[5]);

/* pkh_conserved_totals for callers that cannot allocate device memory
   (code that must not call hipMalloc, e.g. inside tight serving loops or
   under harnesses that forbid allocation): the same kernels, bitwise the
   same result, with the per-leaf partial sums in a static device array of
   the library (one per GPU, 65536 leaves x 5 doubles + 5 results, about
   2.5 MiB, held until the process ends) instead of the mesh's own buffer.
   Allocates nothing. PKH_EINVAL for meshes of more than 65536 leaves. Every
   call on one GPU shares that GPU's array: calls on one GPU that overlap in
   time (meshes on different streams, or host threads) race and must be
   serialised by the caller. Synchronises. out[5] is a host array. */
int pkh_conserved_totals_noalloc(pkh_mesh *mesh, double out[5]);

/* ---- Reverse mode (gradient of a final-state loss w.r.t. the initial
   state). A tape records the timestep of every cycle and the state every
   `ckpt_every` cycles; the adjoint recomputes each segment forward from its
   checkpoint, keeping the ghost-filled inputs of both stages, and sweeps it
   in reverse: per cycle the transposes of the ghost fill, the corrector,
   the ghost fill and the predictor, with the timestep frozen at its
   recorded value and limiter / wave-speed / prolongation-slope branches
   frozen at those the forward pass takes. On meshes with level jumps the
   transposes include the fine-coarse flux correction (each fine sub-face
   flux also carries a quarter of the coarse cell's adjoint), restriction
   (1/8 of a ghost adjoint to each fine cell) and prolongation (the linear
   map with the forward's minmod cases); at walls the image rule. ---- */
typedef struct pkh_tape pkh_tape;

/* Tape for the mesh; ckpt_every >= 1. Device memory: one active-state copy
   per checkpoint (allocated as cycles are recorded) plus 2*ckpt_every + 1
   ghost-filled states for recomputation and 1 or 2 for the reverse sweep.
   Single-level periodic meshes with 8 to 64 cells per block row use the
   pencil/row reverse kernels; meshes with level jumps or walls the
   face-wise reverse. PKH_EINVAL for FP32-stored or partitioned meshes.
   While the tape exists the mesh refuses pkh_regrid and pkh_set_partition
   (PKH_ESTATE). */
int pkh_tape_create(pkh_mesh *mesh, int32_t ckpt_every, pkh_tape **out);
int pkh_tape_destroy(pkh_tape *tape);
/* Use (on = 1) the face-wise reverse on a mesh that does not need it (a
   cross-check of the two), or return (on = 0) to the pencil/row kernels;
   PKH_EINVAL for on = 0 on a mesh with level jumps or walls. The gradient
   does not depend on it beyond rounding. Synchronises. */
int pkh_tape_set_facewise(pkh_tape *tape, int32_t on);

/* Advance n_cycles exactly like pkh_step (no t_end clamp) while recording
   into the tape. A second call discards the previous recording. */
int pkh_forward_taped(pkh_mesh *mesh, pkh_tape *tape, int32_t n_cycles);

/* Advance the mesh's current state by the recorded number of cycles using
   the recorded timesteps (not the CFL timesteps of the current state): the
   map whose derivative pkh_adjoint computes, e.g. for finite-difference
   checks. Records nothing. */
int pkh_tape_replay(pkh_mesh *mesh, pkh_tape *tape);

/* Given lam_final = dL/dU at the end of the recorded cycles (device,
   upload layout), write dL/dU at their start to grad_init (device, upload
   layout; may alias lam_final). The mesh's own state is not touched.
   Enqueued on the mesh's stream; synchronises at the end. */
int pkh_adjoint(pkh_mesh *mesh, pkh_tape *tape, const double *lam_final, double *grad_init);

/* Virtual partition for the multi-GPU data path on one GPU (Sec. 3.7: the
   communication buffers of faces whose neighbour lives on another rank).
   The leaves in storage order are cut into nparts contiguous ranges of
   nearly equal count (the Morton distribution of Sec. 2.1). A same-level
   face between two parts is remote: after each stage (and its flux
   correction) the sender's two cell layers next to every remote face are
   packed into a buffer grouped by (sender part, receiver part), each
   group moves as one device copy (the stand-in for the peer transfer), and
   an unpack kernel writes them into the receiver's ghost layers, which the
   stage kernels then read. Faces inside a part keep the direct reads.
   Results are bitwise those of nparts = 1. nparts in [1, number of leaves];
   the partition survives regrids (recut over the new leaves). A
   partitioned mesh takes no tape or batch (PKH_EINVAL), and a mesh held by
   a tape or batch cannot be repartitioned (PKH_ESTATE). Synchronises. */
int pkh_set_partition(pkh_mesh *mesh, int32_t nparts);
/* Current parts, remote faces and (sender, receiver) messages per stage;
   any pointer may be NULL. */
int pkh_get_partition(const pkh_mesh *mesh, int32_t *nparts, int32_t *nremote, int32_t *nmessages);

/* Launch tuning of the stage kernels (set by the caller or an autotuner).
   tile_rows: rows of cells per workgroup tile (0 = default). Compiled
   choices: n1 = 8: 8; n1 = 16: 8, 16, 4; n1 = 32: 8, 4, 16; n1 = 64: 4, 2.
   It must divide nblock[1]. An explicit choice applies to both stages; the
   default is 8 rows on 32-cell rows and 16 on 16-cell rows of a large mesh
   (it may differ between the stages of other shapes, and pkh_get_tuning
   reports the corrector's).
   packs: launches per stage (0 or 1: one launch over every leaf). With
   packs = P > 1 the leaves (in storage order) are cut into P contiguous
   ranges of nearly equal count and each stage is launched once per range,
   in order: the paper's number of MeshBlockPacks (Sec. 3.6, Sec. 5.1). At
   most the leaf count.
   The results depend on neither (each face flux is computed by the same
   arithmetic whatever the tile or pack, and the CFL reduction is an
   order-free maximum). */
typedef struct {
  int32_t tile_rows;
  int32_t packs;
  int32_t reserved[2];
} pkh_tuning;
int pkh_set_tuning(pkh_mesh *mesh, const pkh_tuning *tuning);
int pkh_get_tuning(const pkh_mesh *mesh, pkh_tuning *tuning);

/* Autotune one mesh the same way (states saved and restored); writes the
   chosen tuning to *out if not NULL. */
int pkh_autotune(pkh_mesh *mesh, int32_t trial_cycles, pkh_tuning *out);

/* ---- Batches: many independent meshes advanced together, each with its
   own t and dt (the paper's concern with launch overhead for many small
   blocks, Sec. 5.1, and MeshBlockPacks, Sec. 3.6). Members may be
   multilevel and may have walls; they must share one HIP stream, be stored
   in FP64 and be unpartitioned. ---- */
typedef struct pkh_batch pkh_batch;
enum {
  PKH_PLAIN = 0,     /* per mesh and cycle: the mesh's own launches (pkh_step) */
  PKH_FUSED = 1,     /* per cycle: one grouped launch per stage and tile shape over
                        every mesh's tiles, each multilevel mesh's flux correction
                        and level-jump face fill, one clock launch for all meshes */
  PKH_GRAPH = 2,     /* PKH_FUSED with segments of up to 50 cycles replayed from a
                        captured hipGraph */
  PKH_PERSISTENT = 3 /* one persistent launch per segment of up to 50 cycles:
                        resident workgroups take (cycle, phase, mesh, tile or
                        chunk) items from a ticket counter in order; an item
                        waits (bounded) only for the previous phase of its own
                        mesh, so meshes overlap and the launch cannot deadlock;
                        the last item of a mesh's cycle advances its clock.
                        Needs blocks of 16 or 32 cells per row (tiles of 16 or
                        8 rows, 256-thread workgroups); PKH_EINVAL otherwise */
};
/* Create a batch over n distinct meshes. tuning (may be NULL): tile_rows
   for the grouped launches of every member (0: each mesh's own), packs
   ignored. The results of the four modes are bitwise identical. While the
   batch exists its meshes refuse pkh_regrid and pkh_set_partition
   (PKH_ESTATE). */
int pkh_batch_create(pkh_mesh *const *meshes, int32_t n, const pkh_tuning *tuning, pkh_batch **out);
int pkh_batch_destroy(pkh_batch *batch);
/* n_cycles cycles of every member in the given mode; no host
   synchronisation. A persistent launch whose bounded wait gave up (a wait
   longer than wait_limit_s) latches an error that the members' next
   synchronising call reports as PKH_ESTATE; the launch still drains and
   ends. */
int pkh_batch_step(pkh_batch *batch, int32_t n_cycles, uint32_t mode);
/* Launch knobs of the persistent mode: waves_per_simd 2 or 3 (0: 2), the
   kernel variant compiled for that occupancy; wait_limit_s the bound of
   every wait inside the persistent kernel, in seconds of the device wall
   clock (default 2; 0 gives up on any wait not met at once). No numerical
   effect. */
typedef struct {
  int32_t waves_per_simd;
  int32_t reserved;
  double wait_limit_s;
} pkh_batch_tuning;
int pkh_batch_set_tuning(pkh_batch *batch, const pkh_batch_tuning *tuning);
int pkh_batch_get_tuning(const pkh_batch *batch, pkh_batch_tuning *tuning);
/* Autotune: for each group of meshes with the same block width, time every
   compiled tile-rows choice over `trial_cycles` fused cycles, then (when the
   persistent mode is available) each waves-per-SIMD variant of the
   persistent kernel, and keep the fastest; the meshes' states and clocks
   are saved and restored around the trials. Writes the chosen tile rows
   per mesh into tile_rows[n] if not NULL; the chosen persistent variant is
   read with pkh_batch_get_tuning. Synchronises. */
int pkh_batch_autotune(pkh_batch *batch, int32_t trial_cycles, int32_t *tile_rows);

/* Kernel timing with HIP events on the handle's stream (a measurement aid
   for the roofline report). `kinds` is a mask of PKH_KT_* bits; while it is
   non-zero, pkh_step (eager path; graph replays are not bracketed) records
   an event pair around every launch of those kinds. Setting a new mask
   discards earlier records. */
enum {
  PKH_KT_PREDICTOR = 1u, /* stage-1 kernel */
  PKH_KT_CORRECTOR = 2u, /* stage-2 kernel (with the fused CFL reduction) */
  PKH_KT_FILL = 4u,      /* ghost fill kernel (faces across level jumps) */
  PKH_KT_FLUXCORR = 8u,  /* fine-coarse flux correction kernel */
  PKH_KT_ADJOINT = 16u,  /* reverse sweep of one stage (pkh_adjoint) */
  PKH_KT_REMOTE = 32u,   /* pack, transfer and unpack of remote faces */
  PKH_KT_KINDS = 6
};
int pkh_kernel_timing(pkh_mesh *mesh, uint32_t kinds);
/* Per kind index (0 predictor, 1 corrector, 2 fill, 3 flux correction,
   4 adjoint stage, 5 remote faces): summed bracketed duration in
   milliseconds and the number of bracketed launches since the mask was
   set. ms[PKH_KT_KINDS], count[PKH_KT_KINDS]. Synchronises. */
int pkh_kernel_times(pkh_mesh *mesh, double *ms, int64_t *count);

/* Wait for the handle's stream and report any latched PKH_EPHYS. */
int pkh_sync(pkh_mesh *mesh);

/* Message of the last failure on this thread ("" if none). */
const char *pkh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PKHYDRO_H */
