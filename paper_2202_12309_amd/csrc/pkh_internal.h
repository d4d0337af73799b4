// pkh_internal.h -- types shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pkh_tiles.h"

namespace pkh {

constexpr int NV = 5;  // rho, M1, M2, M3, E
constexpr int NG = 2;  // ghost width (PLM needs two cells beside a face)

// Face slots of a block: 2*d + s, d = 0 (x), 1 (y), 2 (z); s = 0 low, 1 high.
enum : int { XLO = 0, XHI = 1, YLO = 2, YHI = 3, ZLO = 4, ZHI = 5 };
// Boundary kinds of a domain face (the values of pkh_config.bc).
enum : int { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2 };

// Per-leaf data the kernels read.
struct BlockInfo {
  int32_t level, lx, ly, lz;
  double idx[3];        // 1 / dx_d at the leaf's level
  // Face-buffer slot (in units of one face of n_t1 x n_t2 x 5 doubles) where
  // the stage kernels store this leaf's fluxes on each face; -1 where the
  // face is not a fine-coarse face.
  int32_t fslot[6];
  // bit f set: face f borders finer leaves (this leaf's flux there is
  // replaced by the restricted fine flux after each stage).
  int32_t finer_mask;
};

// Device-resident clock of a mesh; only kernels write it during a step.
struct DevTime {
  double t;            // simulation time
  double dt;           // timestep of the current cycle (after the t_end clamp)
  double dt_next;      // CFL timestep of the current state (before the clamp)
  double cfl;
  unsigned long long smax_bits;  // running max of (|v_d| + c) / dx_d, as bits of a
                                 // non-negative double (ordered like integers)
  long long cycle;
  int err;             // latched PKH_EPHYS (1) / table error (2)
  int pad;
};

// Level maps: dense arrays, one per level, block location -> leaf id or -1.
struct LevelMaps {
  const int32_t* map;   // concatenated
  int64_t off[9];       // start of each level
  int32_t nb[9][3];     // blocks per dim at each level
  int32_t maxl;
};

// Geometry every kernel needs.
struct Geom {
  int32_t n1, n2, n3;   // active cells per block
  int32_t p1, p2, p3;   // padded extents (n + 4)
  int64_t vstride;      // doubles per variable of one padded block
  int64_t bstride;      // doubles per padded block (5 * vstride)
  int32_t nrb[3];       // level-0 blocks per dim
  int32_t bc[6];        // boundary kind per face (x-, x+, y-, y+, z-, z+)
  double gamma;
};

// Coarse-face correction record: one per (coarse leaf, face bordering finer).
struct FineFace {
  int32_t block;        // coarse leaf id
  int32_t face;         // face slot 0..5
  int32_t own_slot;     // face-buffer slot holding the coarse leaf's flux
  int32_t fine_slot[4]; // face-buffer slots of the 4 fine leaves, quadrant (h1 + 2*h2)
};

// ---- launch wrappers (defined in pkh_kernels.hip) ----
struct StageLaunch {
  // state arrays: double, or float when fp32 is set (storage precision;
  // the arithmetic is FP64 either way)
  const void* uin;
  const void* ubase;
  void* uout;
  int32_t fp32;
  const BlockInfo* blocks;
  int32_t nblocks;    // leaves this launch covers: b0 .. b0 + nblocks - 1
  int32_t b0;
  Geom g;
  DevTime* tm;
  double beta;
  int32_t recon;      // 0 DC, 1 PLM
  int32_t do_dt;      // accumulate the CFL reduction from the updated state
  double* fbuf;       // face buffers (may be null on single-level meshes)
  // Same-level neighbour of each leaf per direction, [leaf][27] with index
  // (dz+1)*9 + (dy+1)*3 + (dx+1), -1 where the neighbour is not a same-level
  // leaf. The stage kernel reads halo cells beyond a block face from the
  // neighbour's active cells through it (from the leaf's own ghost zone
  // where it is -1).
  const int32_t* nbr;
  int32_t tj;         // rows per tile (0: default)
};

hipError_t launch_stage(const StageLaunch& a, hipStream_t s);

// A same-level face between leaves of different parts of a partitioned mesh:
// the receiving leaf, its face slot, the sending leaf. Its two ghost layers
// travel through a buffer slot of 2 * 5 * (largest face area) doubles.
struct RemoteFace {
  int32_t recv, face, send, pad;
};
// Copy the sending leaves' two cell layers next to each remote face into
// buf[rec * slot ...], layout [var][layer][t2][t1].
hipError_t launch_remote_pack(const double* u, const RemoteFace* rf, int32_t nrf, const Geom& g, double* buf,
                              int64_t slot, hipStream_t s);
// Write buf[rec * slot ...] into the receiving leaves' ghost layers.
hipError_t launch_remote_unpack(double* u, const RemoteFace* rf, int32_t nrf, const Geom& g, const double* buf,
                                int64_t slot, hipStream_t s);
// One work item of a grouped stage launch over many meshes.
struct GroupItem {
  int32_t inst, blk, j0, pad;
};
// Grouped launch of the stage over the items of meshes that share block
// width n1 and tile rows tj; insts/items are device arrays.
hipError_t launch_stage_group(int recon, int n1, int tj, const StageLaunch* insts,
                              const GroupItem* items, int nitems, hipStream_t s);
// ---- Persistent batch launch: one kernel advances many independent
// meshes by several cycles. Every instance is pinned to one XCD (a GPU
// chiplet with its own L2); the workgroups running on that XCD take the
// items of its instances from that XCD's ticket counter in order (cycle,
// phase, instance) and wait only for items with smaller tickets of the same
// counter, so the launch cannot deadlock whatever its grid, and an item's
// producers wrote through the same L2. ----
// Phases of a cycle: 0 predictor tiles, 1 flux correction of U*, 2 ghost
// faces of U* across level jumps and walls, 3 corrector tiles, 4 flux
// correction of U^{n+1}, 5 ghost faces of U^{n+1}; then the instance's clock.
constexpr int PPHASES = 6;
struct PInst {
  StageLaunch st[2];       // predictor, corrector
  const FineFace* ff;      // flux-correction records (multilevel)
  const int32_t* ff_first;
  const int32_t* cblocks;
  const int32_t* jf;       // ghost face records
  const uint2* plan;       // their fill plan
  int32_t cnt[PPHASES];    // items of each phase in one cycle
  int32_t last;            // last phase with items (its end closes the cycle)
  int32_t n1;              // block width: 16 (16-row tiles) or 32 (8-row tiles)
};
// Monotonic per-instance progress within one launch: items done per phase
// (all cycles so far) and cycles whose clock has been advanced.
struct PSync {
  unsigned int done[PPHASES];
  unsigned int clock;
  unsigned int pad;
};
// One work item: phases 0 and 3 a tile (a = leaf, b = first row); 1 and 4
// a 256-cell chunk a of coarse block b of the flux-correction list; 2 and 5
// a 256-cell chunk a of ghost face record b.
struct PItem {
  int32_t inst, phase, a, b;
};
// Per XCD slot: next ticket, the slot's items (offset into the item array,
// count per cycle); err is shared (slot 0's) and set when a bounded wait
// gave up.
struct PCtl {
  unsigned int ticket;
  int err;
  int32_t off, nper;
};
// XCD ids an XCC_ID register can report (4 bits).
constexpr int PMAX_XCC = 16;
// Rows per tile of the persistent launch (256-thread workgroups).
constexpr int persistent_tile_rows(int n1) { return n1 == 32 ? 8 : (n1 == 16 ? 16 : -1); }
// Resident 256-thread workgroups of the persistent kernel with `waves`
// waves per SIMD (2 or 3), or -1.
int persistent_grid(int waves);
// Reset the progress counters and run `ncycles` cycles of every instance;
// a wait longer than wait_ticks of the device wall clock gives up, latches
// ctl->err and error bit 4 of every instance's clock, and the launch drains.
// slot_of[PMAX_XCC]: the queue slot of each XCD id (-1: none); ctl[nslots].
hipError_t launch_persistent(const PInst* insts, int32_t ninst, PSync* sync, const PItem* items,
                             const int32_t* slot_of, PCtl* ctl, int32_t nslots, int32_t ncycles, int waves,
                             int grid, long long wait_ticks, hipStream_t s);
// XCD ids the workgroups of a launch of 4096 workgroups run on:
// out_host[PMAX_XCC] = 1 for each id seen; dev_buf holds PMAX_XCC ints of
// device memory; synchronises.
hipError_t probe_xcc(int32_t* dev_buf, int32_t* out_host, hipStream_t s);

// Ghost face regions of the (leaf, face) pairs jf[2 njf] (faces whose
// neighbour is on another level).
// Threads per ghost-face record of the face fill (two cell layers of the
// largest face, whole 256-thread workgroups).
__host__ __device__ inline int fill_faces_stride(const Geom& g) {
  const int a01 = g.n1 * g.n2, a02 = g.n1 * g.n3, a12 = g.n2 * g.n3;
  const int area = a01 > a02 ? (a01 > a12 ? a01 : a12) : (a02 > a12 ? a02 : a12);
  return (2 * area + 255) / 256 * 256;
}

// Ghost faces of the records jf (leaf, face | wall kind << 3 | coarser
// neighbour << 6); plan from launch_fill_plan on the same tables,
// njf * fill_faces_stride(g) locations of 8 bytes.
hipError_t launch_fill_faces(double* u, const Geom& g, DevTime* tm, const int32_t* jf, const uint2* plan,
                             int32_t njf, hipStream_t s);
hipError_t launch_fill_plan(uint2* plan, const BlockInfo* blocks, const Geom& g, const LevelMaps& maps,
                            const int32_t* jf, int32_t njf, hipStream_t s);
// skip_same: leave ghost cells whose source is a same-level leaf alone
// (the stage kernels already wrote them).
hipError_t launch_fill(double* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                       const LevelMaps& maps, DevTime* tm, int32_t skip_same, hipStream_t s);
hipError_t launch_flux_correct(double* u, const BlockInfo* blocks, const FineFace* ff,
                               const int32_t* ff_first, const int32_t* cblocks, int32_t ncblocks,
                               const Geom& g, DevTime* tm, double beta, int32_t do_dt,
                               const double* fbuf, const int32_t* nbr, hipStream_t s);
hipError_t launch_dt(const double* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                     DevTime* tm, hipStream_t s);
hipError_t launch_dt(const float* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                     DevTime* tm, hipStream_t s);
hipError_t launch_clock(DevTime* tm, int32_t mode, double t_end, hipStream_t s);
// Upload (double -> stored type), download (stored type -> double), totals;
// the float forms serve meshes whose state is stored in FP32.
hipError_t launch_scatter(double* u, const double* src, int32_t nblocks, const Geom& g, hipStream_t s);
hipError_t launch_scatter(float* u, const double* src, int32_t nblocks, const Geom& g, hipStream_t s);
hipError_t launch_gather(double* dst, const double* u, int32_t nblocks, const Geom& g, hipStream_t s);
hipError_t launch_gather(double* dst, const float* u, int32_t nblocks, const Geom& g, hipStream_t s);
hipError_t launch_totals(double* partial, double* out, const double* u, const BlockInfo* blocks,
                         int32_t nblocks, const Geom& g, hipStream_t s);
hipError_t launch_totals(double* partial, double* out, const float* u, const BlockInfo* blocks,
                         int32_t nblocks, const Geom& g, hipStream_t s);
// The same with the partial sums in the library's static device scratch
// (leaves at most TOTALS_SCRATCH_LEAVES); the five results land at
// scr + TOTALS_SCRATCH_LEAVES * NV. totals_scratch gives the scratch's
// device address on `device` (looked up once per device).
constexpr int32_t TOTALS_SCRATCH_LEAVES = 65536;
hipError_t totals_scratch(int device, double** ptr);
hipError_t launch_totals_scratch(const double* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                                 double* scr, hipStream_t s);
hipError_t launch_totals_scratch(const float* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                                 double* scr, hipStream_t s);
// Pressure-jump indicator per leaf into eta[nblocks] (ghost-filled u).
hipError_t launch_eta(double* eta, const double* u, const int32_t* nbr, int32_t nblocks, const Geom& g,
                      int32_t quantity, hipStream_t s);
// Regrid: new leaf r takes kind[r] (0 copy, 1 child of a refined leaf,
// 2 merged parent) from old leaf src[r].
hipError_t launch_regrid_data(double* unew, const BlockInfo* bnew, const int32_t* kind,
                              const int32_t* src, int32_t nnew, const double* uold,
                              const BlockInfo* bold, const LevelMaps& old_maps, const Geom& g,
                              DevTime* tm, hipStream_t s);

// Reverse mode of one stage U_out = U_base - beta*dt*D(U_in) w.r.t. U_in
// (same-level meshes): out = add0 + add1 + (dD/dU_in)^T-term of lam;
// U is the padded U_in (halos read from the face neighbours); wyz scratch
// for two padded states (the y and z primitive adjoints); xside scratch of
// 20 doubles per x-row (the parts across x faces); dt is read from dtp on
// the device.
hipError_t launch_adj_stage(int recon, const double* U, const double* lam, double* wyz, double* xside,
                            const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                            const int32_t* nbr, const double* dtp, double beta, double* out,
                            const double* add0, const double* add1, hipStream_t s);
// Block widths the row kernels of launch_adj_stage cover.
bool adj_xrow_supported(int n1);
// The same stage reverse face by face, for meshes with level jumps or
// walls (also valid without): gw scratch of one padded state; the
// transposed flux correction and ghost fill of the face records jf[2 njf]
// are included. Lookup failures latch error bit 2 in tm.
hipError_t launch_adj_stage_facewise(int recon, const double* U, const double* lam, double* gw,
                                     const BlockInfo* blocks, int32_t nblocks, const Geom& g, const int32_t* nbr,
                                     const LevelMaps& maps, const int32_t* jf, int32_t njf, const double* dtp,
                                     double beta, double* out, const double* add0, const double* add1,
                                     DevTime* tm, hipStream_t s);
// record: dts[c] = tm->dt; else tm->dt = dts[c].
hipError_t launch_tape_dt(DevTime* tm, double* dts, int32_t c, int32_t record, hipStream_t s);

// Clocks of many meshes in one launch; tms is a device array of n pointers.
hipError_t launch_clock_group(DevTime* const* tms, int32_t n, int32_t mode, double t_end,
                              hipStream_t s);

// Clock modes
enum : int { CLOCK_END = 1, CLOCK_BEGIN = 2, CLOCK_FROM_SMAX = 4 };

}  // namespace pkh
