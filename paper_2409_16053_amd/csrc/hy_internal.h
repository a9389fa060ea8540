// hy_internal.h -- types shared by the host runtime and the gfx950 kernels.
//
// A problem's device workspace starts with a 512-byte header: the descriptor
// below (read by every workgroup with scalar loads) and its counters. Two FP64
// state registers follow (three for RK3), each a MeshBlockPack laid out as
// [block m][variable v][k][j][i] with i (x) fastest and no ghost cells:
// ghost zones are filled into each tile's LDS halo directly from the
// neighbouring block's interior or from the physical boundary condition.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hy {

constexpr int kHeaderBytes = 512;
constexpr int kMaxBatch = 48;   // problems per launch (kernel-argument budget)
constexpr int kWave = 64;       // CDNA wavefront width

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
  unsigned long long* fofc_cnt;  // [2] cells flagged in the stages of sequence parity 0/1
  unsigned long long* fofc_total;
  int32_t fofc;              // 1: first-order flux correction enabled
  // Low-storage SSP-RK stage s (1-based) forms
  //   dst[s-1] = a[s-1] U + b[s-1] src[s-1] + c[s-1] dt L(src[s-1])
  // (stage 1 has a = 0, b = c = 1 and is evaluated as src + dt L).
  int32_t nstages;           // 2 or 3
  const double* src[3];
  double* dst[3];
  double rk_a[3], rk_b[3], rk_c[3];
};

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
