// hy_internal.h -- types shared by the host runtime and the gfx950 kernels.
//
// A problem's device workspace starts with a 1024-byte header: the descriptor
// below (read by every workgroup with scalar loads) and its counters. Two FP64
// state registers follow (three for RK3 and RK4), each a MeshBlockPack laid
// out as [block m][variable v][k][j][i] with i (x) fastest and no ghost cells:
// ghost zones are filled into each tile's LDS halo directly from the
// neighbouring block's interior or from the physical boundary condition (on a
// refined mesh, from a ghost slab where the neighbour is on the other level).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hy {

constexpr int kHeaderBytes = 1024;
constexpr int kMaxBatch = 48;   // problems per launch (kernel-argument budget)
constexpr int kFixPlanes = 1;   // z-planes of one MeshBlock per FOFC correction unit
constexpr int kWave = 64;       // CDNA wavefront width

// One low-storage SSP-RK stage: dst = a U + b src + c dt L(src), evaluated as
// src + c dt L(src) when a == 0 (the "first" kind of stage kernel).
struct RkStage {
  const double* src;
  double* dst;
  double a, b, c;
};

constexpr int kMaxStages = 10;  // SSPRK(10,4)

// Per-problem descriptor in device memory (first bytes of the workspace).
struct DevProblem {
  double* U;                 // register A: state at the start of a step / result
  double* V;                 // register B: state after RK stage 1 (and staging)
  double* W;                 // register C: state after RK3 stage 2 (RK3 only)
  unsigned long long* dtmin; // [2] min over cells of dx_d/lambda_d as ordered bits
  double* time;              // simulation time
  unsigned long long* floor_hits;
  unsigned int* err;         // bit 0: non-finite state or rho <= 0 seen
  int32_t bx, by, bz;        // MeshBlock interior size
  int32_t nbx, nby, nbz;     // MeshBlocks per axis
  int32_t periodic[3];       // 1 if the axis is periodic
  int32_t nblocks;
  int64_t vstride;           // doubles per variable inside a block
  int64_t bstride;           // doubles per block (5 * vstride)
  double dx[3];
  double gamma, cfl, rho_floor, p_floor;
  uint8_t* flags;            // per-cell FOFC flag of the latest counted stage
  uint8_t* fixmask;          // per (leaf, kFixPlanes-plane unit of it): bit 0 set if
                             // a cell in it is flagged, bits 1-4 if a flagged cell
                             // lies on its -x, +x, -y, +y face (set before each
                             // correction pass)
  unsigned long long* fofc_cnt;  // [2] cells flagged in the stages of sequence parity 0/1
  unsigned long long* fofc_total;
  int32_t fofc;              // 1: first-order flux correction enabled
  int32_t nstages;           // SSP-RK stages per step: 1, 2, 3 or 10 (RK4)
  RkStage rk[kMaxStages];    // rk_stage_of(*this, s) at [s - 1], filled at creation
  // Static refinement (all null / 0 without it). nblocks counts leaves; each
  // register holds nblocks + nvirt blocks, the extra ones ghost slabs.
  const int32_t* binfo;      // per leaf kLeafInts: level, neighbour per face
                             // (-x,+x,-y,+y,-z,+z: leaf, nblocks + slab, or -1)
  const int32_t* vinfo;      // per slab 2: owner leaf, face (2 d + side)
  const int32_t* rinfo;      // per root block 2: refined, leaf or first child
  const int32_t* cfinfo;     // per coarse face next to finer leaves 2: leaf, face
  int32_t nvirt, ncf;
  int32_t nroot[3];          // root blocks per axis
  int32_t slab_k2;           // log2 of the ghost slabs packed into one block
  int32_t slab_cells;        // cells per variable of a packed slab (ghost depth
                             // x largest block face); a slab's layer l along
                             // its face normal, tangential cell (a1, a2) (axes
                             // in x, y, z order) sits at slot * slab_cells +
                             // (l * n2 + a2) * n1 + a1 within its block
  int32_t cfarea;            // cells per slot row of cfsave (largest block face)
  double* cfsave;            // FOFC on a refined mesh: per coarse face row,
                             // cfarea x 5 step-start values of its level-face
                             // cells, saved before a stage that updates U in place
};

constexpr int kLeafInts = 12;  // level, neighbour per face (6), x, y, z at its level, 2 unused

// The stage table (Sec. 3: low-storage SSP-RK of the Ketcheson family).
//  RK1: U -> V, then V is copied to U.
//  RK2 SSPRK(2,2): U -> V (0, 1, 1); V -> U (1/2, 1/2, 1/2).
//  RK3 SSPRK(3,3): U -> V (0, 1, 1); V -> W (3/4, 1/4, 1/4);
//                  W -> U (1/3, 2/3, 2/3).
//  RK4 SSPRK(10,4): U keeps q2; q1 runs U -> V -> W -> V ... through stages
//  1-9 as q1 + dt/6 L(q1); after stage 5 (q1 in V) U <- U/25 + 9 V/25 and
//  V <- 15 U - 5 V; stage 10: V -> U with (1, 3/5, 1/10).
// Kernels read the copy in DevProblem::rk: a table load schedules better than
// this chain of selects.
__host__ __device__ inline RkStage rk_stage_of(const DevProblem& P, int stage) {
  RkStage s{P.U, P.V, 0.0, 1.0, 1.0};
  if (P.nstages == 2) {
    if (stage == 2) s = RkStage{P.V, P.U, 0.5, 0.5, 0.5};
  } else if (P.nstages == 3) {
    if (stage == 2) s = RkStage{P.V, P.W, 0.75, 0.25, 0.25};
    if (stage == 3) s = RkStage{P.W, P.U, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0};
  } else if (P.nstages == 10) {
    if (stage == 10) {
      s = RkStage{P.V, P.U, 1.0, 3.0 / 5.0, 1.0 / 10.0};
    } else {
      s.c = 1.0 / 6.0;
      if (stage > 1) {
        s.src = (stage & 1) ? P.W : P.V;
        s.dst = (stage & 1) ? P.V : P.W;
      }
    }
  }
  return s;
}

// Pointwise step after a stage: 1 copies V to U (RK1, after its stage);
// 2 is the RK4 mix after stage 5. 0: none.
__host__ __device__ inline int rk_combine_after(const DevProblem& P, int stage) {
  if (P.nstages == 1 && stage == 1) return 1;
  if (P.nstages == 10 && stage == 5) return 2;
  return 0;
}

// Stage-kernel kind: 1 for a stage with no step-start term that is not the
// last one, 2 otherwise (the last stage of a step also reduces the next time
// step; with a == 0, b == 1 its update equals the kind-1 one exactly).
__host__ __device__ inline int rk_stage_kind(const DevProblem& P, int stage) {
  return rk_stage_of(P, stage).a == 0.0 && stage != P.nstages ? 1 : 2;
}

// Counters that follow the descriptor in the header.
struct DevCounters {
  unsigned long long dtmin[2];
  double time;
  unsigned long long floor_hits;
  unsigned long long fofc_cnt[2];
  unsigned long long fofc_total;
  unsigned int err;
  unsigned int pad;
};

static_assert(sizeof(DevProblem) + sizeof(DevCounters) <= kHeaderBytes, "header too large");

// A whole header as a kernel argument (see k_put_header).
struct HeaderBytes {
  unsigned char b[kHeaderBytes];
};

// One problem's share of a batched stage launch (kernel arguments).
struct BatchEntry {
  const DevProblem* p;
  int32_t tile0;    // first logical tile of this problem in the launch
  int32_t ntx, nty, ntz;  // tiles per block along x, y, z
  int32_t kc;       // planes per z-chunk
  int32_t parity;   // step index mod 2: which dtmin slot the step reads
  int32_t flags;    // bit 0: count floors, flag bad states, flag FOFC cells
  uint32_t seq;     // nstages * step + stage - 1: running stage number (parity
                    // selects the FOFC counter slot)
  int32_t stage;    // RK stage, 1-based
};

struct StageArgs {
  int32_t nprob;
  int32_t ntiles;   // total logical tiles
  BatchEntry e[kMaxBatch];
};

static_assert(sizeof(StageArgs) <= 3072, "kernel arguments too large");

// First-order flux correction pass after a stage (problems with fofc on).
struct FixEntry {
  const DevProblem* p;
  uint32_t seq;
  int32_t parity;
  int32_t stage;    // RK stage, 1-based
  int32_t last;     // 1 if this is the problem's last stage (time step follows)
};

struct FixArgs {
  int32_t nprob;
  int32_t any_last; // 1 if some entry is at its last stage
  FixEntry e[kMaxBatch];
};

static_assert(sizeof(FixArgs) <= 3072, "kernel arguments too large");

}  // namespace hy
