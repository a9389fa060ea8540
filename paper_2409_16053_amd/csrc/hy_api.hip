// hy_api.hip -- host runtime behind the C ABI of include/hy.h.
//
// Owns host metadata only: the problem's workspace (two FP64 MeshBlockPack
// registers, three for RK3 and RK4, a 1024-byte header, and the tables of a
// refined mesh) is provided by the caller. Launch planning
// turns a set of problems into per-stage launch arguments: every problem's
// MeshBlocks are cut into x-y tiles and z-chunks, and one launch per RK
// stage covers the tiles of all problems that share a compiled kernel
// (the paper's MeshBlockPack, Sec. 2, generalised to many problems).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hy.h"
#include "hy_internal.h"
#include "hy_launch.h"

using namespace hy;

struct hy_problem {
  hy_config cfg;
  int ng;
  int nblk[3];
  int64_t ncell;
  char* ws;
  size_t ws_bytes;
  DevProblem* dp;      // descriptor in device memory
  DevCounters* dc;     // counters in device memory
  DevProblem hp;       // host copy of the descriptor
  int64_t steps;
  int variant;
  int kc;
  hipStream_t last;
  int device;
};

namespace {

thread_local std::string g_err;

hy_status fail(hy_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HY_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(HY_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr unsigned long long kInf = 0x7FF0000000000000ull;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int ghost_depth(int recon) { return recon == HY_PLM ? 2 : 3; }

// RK stages per step and state registers per problem for each integrator.
int stages_of(const hy_config* c) {
  return c->rk == 1 ? 1 : (c->rk == 3 ? 3 : (c->rk == 4 ? 10 : 2));
}
int registers_of(const hy_config* c) { return c->rk >= 3 ? 3 : 2; }

// Static refinement: at least one box of refined root blocks.
bool has_refine(const hy_config* c) { return c->nrefine > 0; }

// Root block (rx, ry, rz) lies in one of the refined boxes.
bool root_refined(const hy_config* c, int rx, int ry, int rz) {
  const int r[3] = {rx, ry, rz};
  for (int b = 0; b < c->nrefine; ++b) {
    bool in = true;
    for (int d = 0; d < 3; ++d) in = in && r[d] >= c->refine[b][0][d] && r[d] < c->refine[b][1][d];
    if (in) return true;
  }
  return false;
}

bool validate(const hy_config* c, std::string& msg) {
  if (!c) { msg = "config is NULL"; return false; }
  if (c->recon != HY_PLM && c->recon != HY_PPM4 && c->recon != HY_WENOZ && c->recon != HY_PPMX) {
    msg = "recon must be HY_PLM, HY_PPM4, HY_WENOZ or HY_PPMX";
    return false;
  }
  if (c->rk < 0 || c->rk > 4) { msg = "rk must be 1, 2, 3 or 4 (0 selects 2)"; return false; }
  if (c->precision != HY_FP64 && c->precision != HY_MIXED) { msg = "precision must be HY_FP64 or HY_MIXED"; return false; }
  if (c->fofc != 0 && c->fofc != 1) { msg = "fofc must be 0 or 1"; return false; }
  const int ng = ghost_depth(c->recon);
  for (int d = 0; d < 3; ++d) {
    if (c->n[d] < 1 || c->block[d] < 1) { msg = "n and block must be >= 1"; return false; }
    if (c->n[d] % c->block[d]) { msg = "block must divide n on every axis"; return false; }
    if (c->block[d] < ng) { msg = "block must be >= the ghost depth (2 PLM, 3 PPM4/PPMX/WENO-Z)"; return false; }
    if (!(c->hi[d] > c->lo[d]) || !std::isfinite(c->hi[d] - c->lo[d])) { msg = "need hi > lo"; return false; }
    for (int s = 0; s < 2; ++s)
      if (c->bc[d][s] != HY_BC_PERIODIC && c->bc[d][s] != HY_BC_OUTFLOW) { msg = "bad boundary code"; return false; }
    if ((c->bc[d][0] == HY_BC_PERIODIC) != (c->bc[d][1] == HY_BC_PERIODIC)) {
      msg = "periodic boundaries must be paired on an axis";
      return false;
    }
  }
  if (!(c->gamma > 1.0) || !std::isfinite(c->gamma)) { msg = "gamma must be > 1"; return false; }
  if (!(c->cfl > 0.0 && c->cfl <= 1.0)) { msg = "cfl must be in (0, 1]"; return false; }
  if (!(c->rho_floor >= 0.0) || !(c->p_floor >= 0.0) || !std::isfinite(c->rho_floor) ||
      !std::isfinite(c->p_floor)) {
    msg = "floors must be finite and >= 0";
    return false;
  }
  if (c->nrefine < 0 || c->nrefine > HY_MAX_REFINE_BOXES) {
    msg = "nrefine must be in [0, HY_MAX_REFINE_BOXES]";
    return false;
  }
  if (has_refine(c)) {
    for (int d = 0; d < 3; ++d) {
      if ((c->block[d] & 1) || c->block[d] < 2 * ng) {
        msg = "with refinement, block must be even and >= twice the ghost depth";
        return false;
      }
      for (int b = 0; b < c->nrefine; ++b) {
        if (c->refine[b][0][d] < 0 || c->refine[b][1][d] > c->n[d] / c->block[d]) {
          msg = "refined box outside the root block grid";
          return false;
        }
        if (c->refine[b][0][d] >= c->refine[b][1][d]) {
          msg = "refined box is empty";
          return false;
        }
      }
    }
  }
  const double cells = (double)c->n[0] * c->n[1] * c->n[2] * (has_refine(c) ? 8.0 : 1.0);
  if (cells * 5.0 * 8.0 * registers_of(c) > 4.0e12) { msg = "mesh too large"; return false; }
  const double blk = (double)c->block[0] * c->block[1] * c->block[2] * 5.0;
  if (blk > 2.0e9) { msg = "MeshBlock too large"; return false; }
  return true;
}

// The leaf, slab, root and coarse-face tables of a refined mesh (Sec. 2:
// MeshBlocks on two levels). Leaves: root blocks x fastest; a refined root
// stands for its 8 children, child x offset fastest. A leaf face whose
// neighbour region is at the other level gets a slab: one extra block in each
// register that holds the ghost cells there, at the leaf's level.
struct SmrLayout {
  int nr[3] = {0, 0, 0};
  int nleaf = 0, nvirt = 0, ncf = 0;
  std::vector<int32_t> binfo, vinfo, rinfo, cfinfo;
};

void build_smr(const hy_config* c, SmrLayout& L) {
  for (int d = 0; d < 3; ++d) L.nr[d] = c->n[d] / c->block[d];
  const int nroot = L.nr[0] * L.nr[1] * L.nr[2];
  L.rinfo.assign(2 * (size_t)nroot, 0);
  std::vector<std::array<int, 4>> leaf;  // level, x, y, z
  for (int rz = 0; rz < L.nr[2]; ++rz)
    for (int ry = 0; ry < L.nr[1]; ++ry)
      for (int rx = 0; rx < L.nr[0]; ++rx) {
        const int r = rx + L.nr[0] * (ry + L.nr[1] * rz);
        const bool ref = root_refined(c, rx, ry, rz);
        L.rinfo[2 * r] = ref;
        L.rinfo[2 * r + 1] = (int32_t)leaf.size();
        if (!ref) {
          leaf.push_back({0, rx, ry, rz});
        } else {
          for (int ch = 0; ch < 8; ++ch)
            leaf.push_back({1, 2 * rx + (ch & 1), 2 * ry + ((ch >> 1) & 1), 2 * rz + (ch >> 2)});
        }
      }
  L.nleaf = (int)leaf.size();
  L.binfo.assign((size_t)L.nleaf * kLeafInts, 0);
  auto refined = [&](const int r3[3]) { return L.rinfo[2 * (r3[0] + L.nr[0] * (r3[1] + L.nr[1] * r3[2]))]; };
  auto first = [&](const int r3[3]) { return L.rinfo[2 * (r3[0] + L.nr[0] * (r3[1] + L.nr[1] * r3[2])) + 1]; };
  for (int q = 0; q < L.nleaf; ++q) {
    const int lev = leaf[q][0];
    int32_t* b = &L.binfo[(size_t)q * kLeafInts];
    b[0] = lev;
    for (int d = 0; d < 3; ++d) b[7 + d] = leaf[q][1 + d];
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1;
      int l[3] = {leaf[q][1], leaf[q][2], leaf[q][3]};
      const int nl = L.nr[d] << lev;
      l[d] += (f & 1) ? 1 : -1;
      if (l[d] < 0 || l[d] >= nl) {
        if (c->bc[d][0] != HY_BC_PERIODIC) { b[1 + f] = -1; continue; }
        l[d] = (l[d] + nl) % nl;
      }
      const int r3[3] = {l[0] >> lev, l[1] >> lev, l[2] >> lev};
      const bool fine_there = refined(r3) != 0;
      if (fine_there == (lev == 1)) {  // same level
        b[1 + f] = lev == 0 ? first(r3) : first(r3) + (l[0] & 1) + 2 * (l[1] & 1) + 4 * (l[2] & 1);
      } else {                          // level change: a slab
        b[1 + f] = L.nleaf + L.nvirt++;
        L.vinfo.push_back(q);
        L.vinfo.push_back(f);
        if (lev == 0) {
          L.cfinfo.push_back(q);
          L.cfinfo.push_back(f);
          ++L.ncf;
        }
      }
    }
  }
}

// Ghost slabs packed into one block of a register: log2 of the count, and
// the cells per variable of one slab (ghost depth x largest block face).
int slab_cells(const hy_config* c) {
  return ghost_depth(c->recon) *
         std::max(c->block[1] * c->block[2], std::max(c->block[0] * c->block[2], c->block[0] * c->block[1]));
}
int slab_k2(const hy_config* c) {
  const int64_t per = (int64_t)c->block[0] * c->block[1] * c->block[2] / slab_cells(c);
  int k2 = 0;
  while ((int64_t(2) << k2) <= per) ++k2;
  return k2;
}

// Blocks per register: with refinement the leaves plus the blocks that hold
// the packed ghost slabs, else the root grid.
int64_t register_blocks(const hy_config* c) {
  if (!has_refine(c)) return (int64_t)(c->n[0] / c->block[0]) * (c->n[1] / c->block[1]) * (c->n[2] / c->block[2]);
  SmrLayout L;
  build_smr(c, L);
  const int64_t per = int64_t(1) << slab_k2(c);
  return (int64_t)L.nleaf + (L.nvirt + per - 1) / per;
}

size_t reg_bytes(const hy_config* c) {
  const size_t vs = (size_t)c->block[0] * c->block[1] * c->block[2];
  return align256((size_t)register_blocks(c) * vs * 5 * sizeof(double));
}

// Largest MeshBlock face (cells).
int max_face(const hy_config* c) {
  return std::max(c->block[1] * c->block[2], std::max(c->block[0] * c->block[2], c->block[0] * c->block[1]));
}

// Refinement tables in the workspace: leaf, slab, root and coarse-face
// tables, and with FOFC the saved step-start values of the level-0 cells on
// level faces (per coarse face, the largest block face x 5 doubles).
size_t smr_bytes(const hy_config* c, const SmrLayout* L) {
  if (!has_refine(c)) return 0;
  SmrLayout own;
  if (!L) {
    build_smr(c, own);
    L = &own;
  }
  const size_t save = c->fofc ? align256((size_t)L->ncf * max_face(c) * 5 * sizeof(double)) : 0;
  return align256(L->binfo.size() * 4) + align256(L->vinfo.size() * 4 + 4) +
         align256(L->rinfo.size() * 4) + align256(L->cfinfo.size() * 4 + 4) + save;
}

// One FOFC flag byte per leaf cell (the ghost slabs have none), then one
// byte per unit of kFixPlanes planes of a leaf (the correction pass's mask).
int64_t leaf_count(const hy_config* c) {
  if (!has_refine(c)) return register_blocks(c);
  SmrLayout L;
  build_smr(c, L);
  return L.nleaf;
}
size_t cell_flag_bytes(const hy_config* c) {
  return align256((size_t)leaf_count(c) * c->block[0] * c->block[1] * c->block[2]);
}
size_t flag_bytes(const hy_config* c) {
  if (!c->fofc) return 0;
  const size_t units = (size_t)leaf_count(c) * ((c->block[2] + kFixPlanes - 1) / kFixPlanes);
  return cell_flag_bytes(c) + align256(units);
}

// Tuned launch shapes per (block size, recon, precision).
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> g_tune;

void default_launch(const hy_problem* p, int* variant, int* kc) {
  const int bx = p->cfg.block[0], bz = p->cfg.block[2];
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(bx, p->cfg.block[1], bz, p->cfg.recon, p->cfg.precision));
    if (it != g_tune.end()) {
      *variant = it->second.first;
      *kc = it->second.second;
      return;
    }
  }
  // Preferred shapes from measurement on the 256^3 workload: FP64 does best
  // with 32x8 tiles at 3 waves per SIMD, mixed with 16x16 at 4; fall back to
  // the first variant whose width divides the block.
  const int pref[2][2] = {{3, 5}, {5, 4}};
  int v = -1;
  for (int c : pref[p->cfg.precision == HY_MIXED ? 1 : 0]) {
    int tx, ty;
    stage_variant_shape(c, &tx, &ty);
    if (c < num_stage_variants() && bx % tx == 0) { v = c; break; }
  }
  for (int i = 0; v < 0 && i < num_stage_variants(); ++i) {
    int tx, ty;
    stage_variant_shape(i, &tx, &ty);
    if (bx % tx == 0) v = i;
  }
  if (v < 0) v = 0;
  int tx, ty;
  stage_variant_shape(v, &tx, &ty);
  const int64_t cols = (int64_t)((bx + tx - 1) / tx) * ((p->cfg.block[1] + ty - 1) / ty);
  const int64_t nb = p->hp.nblocks;
  // enough tiles to fill the chip several times over; small problems march
  // through short z-chunks (down to one plane) rather than leave CUs idle
  int k = bz;
  while (k > 1 && nb * cols * ((bz + k - 1) / k) < 2048) k = (k + 1) / 2;
  *variant = v;
  *kc = k;
}

struct Plan {
  int variant, recon, prec;
  std::vector<int> idx;  // problems in this launch group
  std::vector<int> kc;   // z-chunk per problem (indexed like the batch)
};

hy_status check_batch(hy_problem* const* ps, const int32_t* nsteps, int32_t n) {
  if (n < 0 || (n > 0 && (!ps || !nsteps))) return fail(HY_ERR_ARG, "bad batch arguments");
  for (int q = 0; q < n; ++q) {
    if (!ps[q]) return fail(HY_ERR_ARG, "NULL problem in batch");
    if (nsteps[q] < 0) return fail(HY_ERR_ARG, "nsteps must be >= 0");
    for (int r = 0; r < q; ++r)
      if (ps[r] == ps[q]) return fail(HY_ERR_ARG, "a problem appears twice in the batch");
    if (ps[q]->device != ps[0]->device) return fail(HY_ERR_ARG, "problems on different devices");
  }
  return HY_OK;
}

std::vector<Plan> make_plans(hy_problem* const* ps, int32_t n) {
  std::vector<Plan> plans;
  for (int q = 0; q < n; ++q) {
    const int rc = ps[q]->cfg.recon, pr = ps[q]->cfg.precision;
    Plan* pl = nullptr;
    for (auto& x : plans)
      if (x.recon == rc && x.prec == pr) pl = &x;
    if (!pl) {
      plans.push_back(Plan{ps[q]->variant, rc, pr, {}});
      pl = &plans.back();
    }
    pl->idx.push_back(q);
  }
  // the group's tile shape: that of its largest problem
  for (auto& pl : plans) {
    int64_t best = -1;
    for (int q : pl.idx)
      if (ps[q]->ncell > best) { best = ps[q]->ncell; pl.variant = ps[q]->variant; }
  }
  // z-chunks: each problem's own (tuned or default) chunk, lengthened to a
  // common minimum K while the group still has >= 2048 tiles. A problem
  // alone marches short chunks only to fill the chip; in a batch of many
  // small problems the others fill it, and short chunks would re-load the
  // z stencil (2 NG extra planes per chunk) for nothing.
  for (auto& pl : plans) {
    int tx, ty;
    stage_variant_shape(pl.variant, &tx, &ty);
    auto kc_of = [&](int q, int K) {
      return std::max(1, std::min(std::max(ps[q]->kc, K), ps[q]->cfg.block[2]));
    };
    auto tiles = [&](int K) {
      int64_t t = 0;
      for (int q : pl.idx) {
        const hy_problem* p = ps[q];
        const int64_t cols = (int64_t)((p->cfg.block[0] + tx - 1) / tx) * ((p->cfg.block[1] + ty - 1) / ty);
        t += (int64_t)p->hp.nblocks * cols * ((p->cfg.block[2] + kc_of(q, K) - 1) / kc_of(q, K));
      }
      return t;
    };
    int K = 1;
    if (pl.idx.size() > 1)
      for (int cand = 64; cand > 1; cand /= 2)
        if (tiles(cand) >= 2048) { K = cand; break; }
    pl.kc.assign(n, 1);
    for (int q : pl.idx) pl.kc[q] = kc_of(q, K);
  }
  return plans;
}

hy_status launch_group(hy_problem* const* ps, const std::vector<int>& act, const Plan& pl,
                       int stage, int kind, const std::vector<int64_t>& step_of, int flags,
                       hipStream_t s) {
  // every problem in `act` has at least `stage` stages, and that stage is of
  // the given kernel kind (1: no step-start term, 2: with it)
  int tx, ty;
  stage_variant_shape(pl.variant, &tx, &ty);
  for (size_t c0 = 0; c0 < act.size(); c0 += kMaxBatch) {
    StageArgs a;
    std::memset(&a, 0, sizeof a);
    int64_t tiles = 0;
    int smr = 0;  // a refined problem in the launch: the stage kernel that knows ghost slabs
    const size_t c1 = std::min(act.size(), c0 + (size_t)kMaxBatch);
    for (size_t c = c0; c < c1; ++c) {
      const int q = act[c];
      const hy_problem* p = ps[q];
      smr |= p->hp.binfo != nullptr;
      BatchEntry& e = a.e[a.nprob++];
      e.p = p->dp;
      e.tile0 = (int32_t)tiles;
      e.ntx = (p->cfg.block[0] + tx - 1) / tx;
      e.nty = (p->cfg.block[1] + ty - 1) / ty;
      e.kc = pl.kc[q];
      e.ntz = (p->cfg.block[2] + e.kc - 1) / e.kc;
      e.parity = (int32_t)(step_of[q] & 1);
      e.flags = flags;
      e.seq = (uint32_t)(p->hp.nstages * step_of[q] + stage - 1);
      e.stage = stage;
      tiles += (int64_t)p->hp.nblocks * e.ntx * e.nty * e.ntz;
    }
    if (tiles > 0x7fffffff) return fail(HY_ERR_ARG, "too many tiles in one launch");
    a.ntiles = (int32_t)tiles;
    if (tiles == 0) continue;
    HY_HIP(launch_stage(pl.variant, pl.recon, pl.prec, kind, smr, a, (int)tiles, s));
  }
  return HY_OK;
}

// First-order flux correction after a stage for the problems that enable it.
hy_status launch_fix(hy_problem* const* ps, const std::vector<int>& act, const Plan& pl, int stage,
                     const std::vector<int64_t>& step_of, hipStream_t s) {
  std::vector<int> f;
  for (int q : act)
    if (ps[q]->cfg.fofc) f.push_back(q);
  for (size_t c0 = 0; c0 < f.size(); c0 += kMaxBatch) {
    FixArgs a;
    std::memset(&a, 0, sizeof a);
    int grid = 1;
    for (size_t c = c0; c < std::min(f.size(), c0 + (size_t)kMaxBatch); ++c) {
      const hy_problem* p = ps[f[c]];
      FixEntry& e = a.e[a.nprob++];
      e.p = p->dp;
      e.seq = (uint32_t)(p->hp.nstages * step_of[f[c]] + stage - 1);
      e.parity = (int32_t)(step_of[f[c]] & 1);
      e.stage = stage;
      e.last = stage == p->hp.nstages;
      a.any_last |= e.last;
      grid = std::max(grid, fofc_grid(p->hp.nblocks, p->cfg.block[2]));
    }
    HY_HIP(launch_fofc(pl.recon, pl.prec, a, std::min(grid, 65535), s));
  }
  return HY_OK;
}

// Pointwise steps between stages (RK1's copy, RK4's mix) for the problems
// that need one after this stage.
hy_status launch_combines(hy_problem* const* ps, const std::vector<int>& act, int stage,
                          const std::vector<int64_t>& step_of, hipStream_t s) {
  for (int op = 1; op <= 2; ++op) {
    std::vector<int> f;
    for (int q : act)
      if (rk_combine_after(ps[q]->hp, stage) == op) f.push_back(q);
    for (size_t c0 = 0; c0 < f.size(); c0 += kMaxBatch) {
      FixArgs a;
      std::memset(&a, 0, sizeof a);
      int64_t most = 1;
      for (size_t c = c0; c < std::min(f.size(), c0 + (size_t)kMaxBatch); ++c) {
        FixEntry& e = a.e[a.nprob++];
        e.p = ps[f[c]]->dp;
        e.parity = (int32_t)(step_of[f[c]] & 1);
        e.stage = stage;
        most = std::max(most, ps[f[c]]->ncell * 5);
      }
      HY_HIP(launch_combine(a, op, (int)std::min<int64_t>((most + 255) / 256, 4096), s));
    }
  }
  return HY_OK;
}

// Enqueue nsteps[q] steps of every problem; optional events around stages.
hy_status run_batch(hy_problem* const* ps, const int32_t* nsteps, int32_t n, hipStream_t s,
                    std::vector<hipEvent_t>* ev, int flags) {
  hy_status st = check_batch(ps, nsteps, n);
  if (st != HY_OK) return st;
  if (n == 0) return HY_OK;
  int dev;
  HY_HIP(hipGetDevice(&dev));
  if (dev != ps[0]->device) return fail(HY_ERR_ARG, "current device differs from the problems' device");
  const std::vector<Plan> plans = make_plans(ps, n);
  int32_t maxs = 0;
  int maxst = 0;
  for (int q = 0; q < n; ++q) {
    maxs = std::max(maxs, nsteps[q]);
    maxst = std::max(maxst, ps[q]->hp.nstages);
  }
  std::vector<int64_t> step_of(n);
  for (int q = 0; q < n; ++q) step_of[q] = ps[q]->steps;
  size_t evi = 0;
  if (ev) HY_HIP(hipEventRecord((*ev)[evi++], s));
  for (int32_t k = 0; k < maxs; ++k) {
    for (int stage = 1; stage <= maxst; ++stage) {
      for (const Plan& pl : plans) {
        std::vector<int> act, by_kind[2];
        for (int q : pl.idx)
          if (nsteps[q] > k && ps[q]->hp.nstages >= stage) {
            act.push_back(q);
            by_kind[rk_stage_kind(ps[q]->hp, stage) - 1].push_back(q);
          }
        for (int q : act)  // ghost slabs across level changes, from this stage's source
          if (ps[q]->hp.nvirt > 0) HY_HIP(launch_smr_ghost(ps[q]->dp, stage, ps[q]->ng, ps[q]->hp.nvirt,
                                                          ps[q]->cfg.block, s));
        for (int q : act)  // FOFC on a refined mesh, a stage that updates U in place
          if (ps[q]->hp.ncf > 0 && (flags & 1) && ps[q]->cfg.fofc && ps[q]->hp.rk[stage - 1].dst == ps[q]->hp.U)
            HY_HIP(launch_smr_save(ps[q]->dp, ps[q]->hp.ncf, ps[q]->cfg.block, s));
        for (int kind = 1; kind <= 2; ++kind) {
          st = launch_group(ps, by_kind[kind - 1], pl, stage, kind, step_of, flags, s);
          if (st != HY_OK) return st;
        }
        // FOFC belongs to counted (real) stages only. On a refined mesh with
        // FOFC, the level-0 cells on level faces are finished (and tested)
        // by k_smr_cell before the correction pass; without FOFC, the coarse
        // faces next to finer leaves take the fine fluxes after the stage.
        for (int q : act)
          if (ps[q]->hp.ncf > 0 && (flags & 1) && ps[q]->cfg.fofc) {
            const hy_problem* pq = ps[q];
            const uint32_t seq = (uint32_t)(pq->hp.nstages * step_of[q] + stage - 1);
            HY_HIP(launch_smr_cell(pl.recon, pl.prec, pq->dp, stage, (int)(step_of[q] & 1), seq, pq->hp.ncf,
                                   pq->cfg.block, s));
          }
        if (flags & 1) {
          st = launch_fix(ps, act, pl, stage, step_of, s);
          if (st != HY_OK) return st;
        }
        for (int q : act)
          if (ps[q]->hp.ncf > 0) {
            const hy_problem* pq = ps[q];
            const int last = stage == pq->hp.nstages;
            const int parity = (int)(step_of[q] & 1);
            if (!((flags & 1) && pq->cfg.fofc))
              HY_HIP(launch_smr_flux(pl.recon, pl.prec, pq->dp, stage, parity, pq->hp.ncf, pq->cfg.block, s));
            if (last) HY_HIP(launch_smr_dt(pq->dp, pq->hp.nblocks, pq->cfg.block, parity ^ 1, s));
          }
        st = launch_combines(ps, act, stage, step_of, s);
        if (st != HY_OK) return st;
      }
      if (ev) HY_HIP(hipEventRecord((*ev)[evi++], s));
    }
    for (int q = 0; q < n; ++q)
      if (nsteps[q] > k) ++step_of[q];
  }
  for (int q = 0; q < n; ++q) {
    ps[q]->steps = step_of[q];
    ps[q]->last = s;
  }
  return HY_OK;
}

// Captured step sequences, keyed by everything that is baked into them.
struct GraphKey {
  std::vector<hy_problem*> ps;
  std::vector<int32_t> nsteps;
  std::vector<int32_t> parity, variant, kc;
  bool operator==(const GraphKey& o) const {
    return ps == o.ps && nsteps == o.nsteps && parity == o.parity && variant == o.variant &&
           kc == o.kc;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;  // most recently used last
constexpr size_t kMaxGraphs = 64;

void release(GraphEntry& g) {
  (void)hipGraphExecDestroy(g.exec);
  (void)hipGraphDestroy(g.graph);
}

void drop_graphs_of(const hy_problem* p) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (size_t i = 0; i < g_graphs.size();) {
    const auto& v = g_graphs[i].key.ps;
    if (std::find(v.begin(), v.end(), p) != v.end()) {
      release(g_graphs[i]);
      g_graphs.erase(g_graphs.begin() + (long)i);
    } else {
      ++i;
    }
  }
}

hy_status read_counters(hy_problem* p, DevCounters* c) {
  HY_HIP(hipStreamSynchronize(p->last));
  HY_HIP(hipMemcpy(c, p->dc, sizeof *c, hipMemcpyDeviceToHost));
  return HY_OK;
}

}  // namespace

extern "C" {

size_t hy_workspace_bytes(const hy_config* cfg) {
  std::string msg;
  if (!validate(cfg, msg)) {
    g_err = msg;
    return 0;
  }
  return (size_t)kHeaderBytes + (size_t)registers_of(cfg) * reg_bytes(cfg) + flag_bytes(cfg) +
         smr_bytes(cfg, nullptr);
}

int32_t hy_leaves(const hy_config* cfg, int32_t* out) {
  std::string msg;
  if (!validate(cfg, msg)) {
    g_err = msg;
    return -1;
  }
  if (!has_refine(cfg)) {
    const int nr[3] = {cfg->n[0] / cfg->block[0], cfg->n[1] / cfg->block[1], cfg->n[2] / cfg->block[2]};
    int32_t q = 0;
    for (int z = 0; z < nr[2]; ++z)
      for (int y = 0; y < nr[1]; ++y)
        for (int x = 0; x < nr[0]; ++x, ++q)
          if (out) {
            out[4 * q] = 0;
            out[4 * q + 1] = x;
            out[4 * q + 2] = y;
            out[4 * q + 3] = z;
          }
    return q;
  }
  SmrLayout L;
  build_smr(cfg, L);
  if (out)
    for (int q = 0; q < L.nleaf; ++q) {
      out[4 * q] = L.binfo[(size_t)q * kLeafInts];
      for (int d = 0; d < 3; ++d) out[4 * q + 1 + d] = L.binfo[(size_t)q * kLeafInts + 7 + d];
    }
  return L.nleaf;
}

namespace {

// Fill a host problem object for a workspace at `ws` and the header bytes its
// device copy must hold (descriptor and cleared counters); with refinement,
// also the tables to upload into the workspace. No device calls.
hy_status build_problem(const hy_config* cfg, char* ws, size_t ws_bytes, int dev, hy_problem* p,
                        unsigned char hdr[kHeaderBytes], SmrLayout* L) {
  p->cfg = *cfg;
  p->ng = ghost_depth(cfg->recon);
  for (int d = 0; d < 3; ++d) p->nblk[d] = cfg->n[d] / cfg->block[d];
  p->ncell = (int64_t)cfg->n[0] * cfg->n[1] * cfg->n[2];
  p->ws = ws;
  p->ws_bytes = ws_bytes;
  p->dp = (DevProblem*)p->ws;
  p->dc = (DevCounters*)(p->ws + sizeof(DevProblem));
  p->device = dev;
  p->last = nullptr;
  p->steps = 0;

  DevProblem& h = p->hp;
  std::memset(&h, 0, sizeof h);
  h.U = (double*)(p->ws + kHeaderBytes);
  h.V = (double*)(p->ws + kHeaderBytes + reg_bytes(cfg));
  h.dtmin = p->dc->dtmin;
  h.time = &p->dc->time;
  h.floor_hits = &p->dc->floor_hits;
  h.err = &p->dc->err;
  h.bx = cfg->block[0];
  h.by = cfg->block[1];
  h.bz = cfg->block[2];
  h.nbx = p->nblk[0];
  h.nby = p->nblk[1];
  h.nbz = p->nblk[2];
  for (int d = 0; d < 3; ++d) {
    h.periodic[d] = cfg->bc[d][0] == HY_BC_PERIODIC;
    h.dx[d] = (cfg->hi[d] - cfg->lo[d]) / cfg->n[d];
  }
  h.nblocks = p->nblk[0] * p->nblk[1] * p->nblk[2];
  h.vstride = (int64_t)h.bx * h.by * h.bz;
  h.bstride = 5 * h.vstride;
  h.gamma = cfg->gamma;
  h.cfl = cfg->cfl;
  h.rho_floor = cfg->rho_floor;
  h.p_floor = cfg->p_floor;
  h.fofc = cfg->fofc;
  const int nreg = registers_of(cfg);
  h.W = nreg == 3 ? (double*)(p->ws + kHeaderBytes + 2 * reg_bytes(cfg)) : nullptr;
  h.flags = cfg->fofc ? (uint8_t*)(p->ws + kHeaderBytes + (size_t)nreg * reg_bytes(cfg)) : nullptr;
  h.fixmask = cfg->fofc ? h.flags + cell_flag_bytes(cfg) : nullptr;
  h.fofc_cnt = p->dc->fofc_cnt;
  h.fofc_total = &p->dc->fofc_total;
  h.nstages = stages_of(cfg);
  for (int st = 1; st <= h.nstages; ++st) h.rk[st - 1] = rk_stage_of(h, st);
  if (has_refine(cfg)) {
    build_smr(cfg, *L);
    if (L->nvirt > 65535 || L->ncf > 65535 || L->nleaf > 65535)
      return fail(HY_ERR_ARG, "refined mesh too large (max 65535 leaves and level-change faces)");
    char* t = p->ws + kHeaderBytes + (size_t)nreg * reg_bytes(cfg) + flag_bytes(cfg);
    h.binfo = (const int32_t*)t;
    t += align256(L->binfo.size() * 4);
    h.vinfo = (const int32_t*)t;
    t += align256(L->vinfo.size() * 4 + 4);
    h.rinfo = (const int32_t*)t;
    t += align256(L->rinfo.size() * 4);
    h.cfinfo = (const int32_t*)t;
    t += align256(L->cfinfo.size() * 4 + 4);
    h.cfarea = max_face(cfg);
    h.slab_k2 = slab_k2(cfg);
    h.slab_cells = slab_cells(cfg);
    h.cfsave = cfg->fofc ? (double*)t : nullptr;
    h.nvirt = L->nvirt;
    h.ncf = L->ncf;
    for (int d = 0; d < 3; ++d) h.nroot[d] = L->nr[d];
    h.nblocks = L->nleaf;
    p->ncell = (int64_t)L->nleaf * h.vstride;
  }
  std::memset(hdr, 0, kHeaderBytes);
  std::memcpy(hdr, &h, sizeof h);
  DevCounters c;
  std::memset(&c, 0, sizeof c);
  c.dtmin[0] = c.dtmin[1] = kInf;
  std::memcpy(hdr + sizeof(DevProblem), &c, sizeof c);
  default_launch(p, &p->variant, &p->kc);
  return HY_OK;
}

}  // namespace

hy_status hy_create(const hy_config* cfg, void* dev_ws, size_t ws_bytes, hy_problem** out) {
  std::string msg;
  if (!out) return fail(HY_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!validate(cfg, msg)) return fail(HY_ERR_ARG, msg);
  if (!dev_ws) return fail(HY_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)dev_ws) & 255) return fail(HY_ERR_ARG, "workspace must be 256-byte aligned");
  const size_t need = hy_workspace_bytes(cfg);
  if (ws_bytes < need) return fail(HY_ERR_NOMEM, "workspace smaller than hy_workspace_bytes()");
  int dev;
  HY_HIP(hipGetDevice(&dev));
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, dev_ws) != hipSuccess || attr.type != hipMemoryTypeDevice ||
      attr.device != dev) {
    (void)hipGetLastError();
    return fail(HY_ERR_ARG, "workspace is not device memory of the current device");
  }
  hy_problem* p = new (std::nothrow) hy_problem();
  if (!p) return fail(HY_ERR_NOMEM, "host allocation failed");
  unsigned char hdr[kHeaderBytes];
  SmrLayout L;
  hy_status st = build_problem(cfg, (char*)dev_ws, ws_bytes, dev, p, hdr, &L);
  if (st != HY_OK) {
    delete p;
    return st;
  }
  const DevProblem& h = p->hp;
  if (h.binfo) {
    const std::pair<const int32_t*, const std::vector<int32_t>*> tabs[4] = {
        {h.binfo, &L.binfo}, {h.vinfo, &L.vinfo}, {h.rinfo, &L.rinfo}, {h.cfinfo, &L.cfinfo}};
    for (const auto& tb : tabs)
      if (!tb.second->empty() &&
          hipMemcpy((void*)tb.first, tb.second->data(), tb.second->size() * 4, hipMemcpyHostToDevice) !=
              hipSuccess) {
        delete p;
        return fail(HY_ERR_HIP, "refinement table upload failed");
      }
  }
  if (hipMemcpy(p->ws, hdr, kHeaderBytes, hipMemcpyHostToDevice) != hipSuccess ||
      (cfg->fofc && hipMemset(h.flags, 0, flag_bytes(cfg)) != hipSuccess)) {
    delete p;
    return fail(HY_ERR_HIP, "header upload failed");
  }
  *out = p;
  return HY_OK;
}

hy_status hy_set_state(hy_problem* p, const double* U, int where, void* stream) {
  if (!p || !U) return fail(HY_ERR_ARG, "NULL argument");
  if (where != HY_HOST && where != HY_DEVICE && where != HY_HOST_PINNED)
    return fail(HY_ERR_ARG, "bad buffer location");
  hipStream_t s = (hipStream_t)stream;
  const double* src = U;
  const size_t bytes = (size_t)p->ncell * 5 * sizeof(double);
  if (p->hp.binfo) {  // refined mesh: leaf-major, the register's own layout
    HY_HIP(hipMemcpyAsync(p->hp.U, U, bytes,
                          where == HY_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  } else {
    if (where != HY_DEVICE) {
      HY_HIP(hipMemcpyAsync(p->hp.V, U, bytes, hipMemcpyHostToDevice, s));
      src = p->hp.V;
    }
    HY_HIP(launch_scatter(p->dp, src, p->hp.U, p->ncell * 5, 1, s));
  }
  const int slot = (int)(p->steps & 1);
  HY_HIP(launch_reset(p->dp, slot ^ 1, 0, s));  // the slot the next step reduces into
  HY_HIP(launch_reset(p->dp, slot, 1, s));
  HY_HIP(launch_dt(p->dp, p->ncell, slot, 1, s));
  if (where == HY_HOST) HY_HIP(hipStreamSynchronize(s));
  p->last = s;
  return HY_OK;
}

hy_status hy_get_state(hy_problem* p, double* U, int where, void* stream) {
  if (!p || !U) return fail(HY_ERR_ARG, "NULL argument");
  if (where != HY_HOST && where != HY_DEVICE && where != HY_HOST_PINNED)
    return fail(HY_ERR_ARG, "bad buffer location");
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)p->ncell * 5 * sizeof(double);
  if (p->hp.binfo) {
    HY_HIP(hipMemcpyAsync(U, p->hp.U, bytes,
                          where == HY_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  } else if (where == HY_DEVICE) {
    HY_HIP(launch_scatter(p->dp, p->hp.U, U, p->ncell * 5, 0, s));
  } else {
    HY_HIP(launch_scatter(p->dp, p->hp.U, p->hp.V, p->ncell * 5, 0, s));
    HY_HIP(hipMemcpyAsync(U, p->hp.V, bytes, hipMemcpyDeviceToHost, s));
  }
  p->last = s;
  if (where == HY_HOST_PINNED) return HY_OK;
  DevCounters c;
  hy_status st = read_counters(p, &c);
  if (st != HY_OK) return st;
  if (c.err) return fail(HY_ERR_STATE, "non-finite state or rho <= 0 seen on the device");
  return HY_OK;
}

hy_status hy_advance(hy_problem* p, int32_t nsteps, void* stream) {
  if (!p) return fail(HY_ERR_ARG, "NULL problem");
  return run_batch(&p, &nsteps, 1, (hipStream_t)stream, nullptr, 1);
}

hy_status hy_batch_advance(hy_problem* const* ps, const int32_t* nsteps, int32_t n, void* stream) {
  return run_batch(ps, nsteps, n, (hipStream_t)stream, nullptr, 1);
}

hy_status hy_batch_advance_graph(hy_problem* const* ps, const int32_t* nsteps, int32_t n,
                                 void* stream) {
  hy_status st = check_batch(ps, nsteps, n);
  if (st != HY_OK) return st;
  if (!stream) return fail(HY_ERR_ARG, "graph capture needs a non-default stream");
  if (n == 0) return HY_OK;
  hipStream_t s = (hipStream_t)stream;
  GraphKey key;
  for (int q = 0; q < n; ++q) {
    key.ps.push_back(ps[q]);
    key.nsteps.push_back(nsteps[q]);
    key.parity.push_back((int32_t)(ps[q]->steps & 1));
    key.variant.push_back(ps[q]->variant);
    key.kc.push_back(ps[q]->kc);
  }
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (size_t i = 0; i < g_graphs.size(); ++i) {
    if (g_graphs[i].key == key) {
      GraphEntry e = g_graphs[i];
      g_graphs.erase(g_graphs.begin() + (long)i);
      g_graphs.push_back(e);
      HY_HIP(hipGraphLaunch(e.exec, s));
      for (int q = 0; q < n; ++q) {
        ps[q]->steps += nsteps[q];
        ps[q]->last = s;
      }
      return HY_OK;
    }
  }
  std::vector<int64_t> before(n);
  for (int q = 0; q < n; ++q) before[q] = ps[q]->steps;
  HY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  st = run_batch(ps, nsteps, n, s, nullptr, 1);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s, &graph);
  for (int q = 0; q < n; ++q) ps[q]->steps = before[q];  // nothing ran yet
  if (st != HY_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(HY_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(HY_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  if (g_graphs.size() >= kMaxGraphs) {
    release(g_graphs.front());
    g_graphs.erase(g_graphs.begin());
  }
  g_graphs.push_back(GraphEntry{key, graph, exec});
  HY_HIP(hipGraphLaunch(exec, s));
  for (int q = 0; q < n; ++q) {
    ps[q]->steps += nsteps[q];
    ps[q]->last = s;
  }
  return HY_OK;
}

hy_status hy_query(hy_problem* p, double* t, double* dt_next, int64_t* steps, int64_t* floor_hits,
                   int64_t* fofc_cells) {
  if (!p) return fail(HY_ERR_ARG, "NULL problem");
  DevCounters c;
  hy_status st = read_counters(p, &c);
  if (st != HY_OK) return st;
  if (t) *t = c.time;
  if (dt_next) {
    double m;
    std::memcpy(&m, &c.dtmin[p->steps & 1], sizeof m);
    *dt_next = p->cfg.cfl * m;
  }
  if (steps) *steps = p->steps;
  if (floor_hits) *floor_hits = (int64_t)c.floor_hits;
  if (fofc_cells) *fofc_cells = (int64_t)(c.fofc_total + c.fofc_cnt[0] + c.fofc_cnt[1]);
  if (c.err) return fail(HY_ERR_STATE, "non-finite state or rho <= 0 seen on the device");
  return HY_OK;
}

hy_status hy_set_time(hy_problem* p, double t) {
  if (!p || !std::isfinite(t)) return fail(HY_ERR_ARG, "bad argument");
  HY_HIP(hipStreamSynchronize(p->last));
  HY_HIP(hipMemcpy(&p->dc->time, &t, sizeof t, hipMemcpyHostToDevice));
  return HY_OK;
}

hy_status hy_destroy(hy_problem* p) {
  if (!p) return HY_OK;
  hipError_t e = hipStreamSynchronize(p->last);
  drop_graphs_of(p);
  delete p;
  if (e != hipSuccess) return fail(HY_ERR_HIP, hipGetErrorString(e));
  return HY_OK;
}

const char* hy_last_error(void) { return g_err.c_str(); }

int32_t hy_num_variants(void) { return num_stage_variants(); }

hy_status hy_variant_info(int32_t v, int32_t* tx, int32_t* ty, int32_t* waves) {
  if (v < 0 || v >= num_stage_variants()) return fail(HY_ERR_ARG, "bad variant");
  int a, b;
  stage_variant_shape(v, &a, &b);
  if (tx) *tx = a;
  if (ty) *ty = b;
  if (waves) *waves = stage_variant_waves(v);
  return HY_OK;
}

hy_status hy_set_launch(hy_problem* p, int32_t variant, int32_t kc) {
  if (!p || variant < 0 || variant >= num_stage_variants() || kc < 1)
    return fail(HY_ERR_ARG, "bad launch shape");
  p->variant = variant;
  p->kc = std::min(kc, p->cfg.block[2]);
  drop_graphs_of(p);
  return HY_OK;
}

hy_status hy_get_launch(const hy_problem* p, int32_t* variant, int32_t* kc) {
  if (!p) return fail(HY_ERR_ARG, "NULL problem");
  if (variant) *variant = p->variant;
  if (kc) *kc = p->kc;
  return HY_OK;
}

hy_status hy_autotune(hy_problem* p, void* stream, int32_t full_steps, int32_t* variant,
                      int32_t* kc, double* us) {
  if (!p || full_steps < 0) return fail(HY_ERR_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  const int bz = p->cfg.block[2];
  std::vector<int> kcs;
  for (int k : {bz, bz / 2, bz / 4, 32, 16, 8, 4, 2, 1})
    if (k >= 1 && k <= bz && std::find(kcs.begin(), kcs.end(), k) == kcs.end()) kcs.push_back(k);
  if (kcs.empty()) kcs.push_back(bz);
  hipEvent_t e0, e1;
  HY_HIP(hipEventCreate(&e0));
  HY_HIP(hipEventCreate(&e1));
  const int save_v = p->variant, save_k = p->kc;
  float best = 1e30f;
  int bv = save_v, bk = save_k;
  std::vector<int64_t> step_of{p->steps};
  std::vector<int> act{0};
  hy_problem* ps[1] = {p};
  hy_status st = HY_OK;
  for (int v = 0; v < num_stage_variants() && st == HY_OK; ++v) {
    for (int k : kcs) {
      p->variant = v;
      p->kc = k;
      Plan pl{v, p->cfg.recon, p->cfg.precision, {0}};
      const int reps = full_steps > 0 ? full_steps : 3;
      // best of three timings: neighbouring candidates are often within the
      // run-to-run spread of a single one
      float cand = 1e30f;
      for (int trial = 0; trial < 3 && st == HY_OK; ++trial) {
        if (full_steps > 0) {
          int32_t one = 1;
          if (trial == 0) st = run_batch(ps, &one, 1, s, nullptr, 1);  // warm-up step
          if (st != HY_OK) break;
          if (hipEventRecord(e0, s) != hipSuccess) { st = fail(HY_ERR_HIP, "event record"); break; }
          int32_t n = full_steps;
          st = run_batch(ps, &n, 1, s, nullptr, 1);
        } else {
          if (trial == 0) st = launch_group(ps, act, pl, 1, 1, step_of, 0, s);  // warm-up
          if (st != HY_OK) break;
          if (hipEventRecord(e0, s) != hipSuccess) { st = fail(HY_ERR_HIP, "event record"); break; }
          for (int r = 0; r < reps && st == HY_OK; ++r)
            st = launch_group(ps, act, pl, 1, 1, step_of, 0, s);
        }
        if (st != HY_OK) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          st = fail(HY_ERR_HIP, "event sync");
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        cand = std::min(cand, ms);
      }
      if (st != HY_OK) break;
      if (cand < best) { best = cand; bv = v; bk = k; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != HY_OK) {
    p->variant = save_v;
    p->kc = save_k;
    return st;
  }
  p->variant = bv;
  p->kc = bk;
  p->last = s;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(p->cfg.block[0], p->cfg.block[1], p->cfg.block[2], p->cfg.recon,
                           p->cfg.precision)] = {bv, bk};
  }
  if (variant) *variant = bv;
  if (kc) *kc = bk;
  if (us) *us = best * 1000.0 / (full_steps > 0 ? (double)p->hp.nstages * full_steps : 3.0);
  return HY_OK;
}

hy_status hy_copy_probe(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || (bytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15))
    return fail(HY_ERR_ARG, "copy probe needs 16-byte aligned pointers and sizes");
  HY_HIP(launch_copy(dst, src, bytes, (hipStream_t)stream));
  return HY_OK;
}

hy_status hy_advance_timed(hy_problem* p, int32_t nsteps, void* stream, double* ms1, double* ms2) {
  if (!p || nsteps < 0) return fail(HY_ERR_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  const size_t ns = (size_t)p->hp.nstages;
  std::vector<hipEvent_t> ev(ns * (size_t)nsteps + 1);
  for (auto& e : ev) HY_HIP(hipEventCreate(&e));
  hy_status st = run_batch(&p, &nsteps, 1, s, &ev, 1);
  double a = 0, b = 0;
  if (st == HY_OK && hipEventSynchronize(ev.back()) == hipSuccess) {
    for (size_t k = 0; k < (size_t)nsteps; ++k) {
      for (size_t j = 0; j < ns; ++j) {
        float x = 0;
        (void)hipEventElapsedTime(&x, ev[ns * k + j], ev[ns * k + j + 1]);
        (j == 0 ? a : b) += x;
      }
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (ms1) *ms1 = a;
  if (ms2) *ms2 = b;
  return st;
}

}  // extern "C"

// ---------------------------------------------------- allocation-free entry
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops): the problem's whole workspace lives in a
// file-scope device array of kNoAllocBytes per GPU, held until the process
// ends. Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol): each device's address comes from
// hipGetSymbolAddress on the first call there, with that device current.
namespace {

constexpr size_t kNoAllocBytes = (size_t)HY_NOALLOC_MAX_BYTES;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hy_status scratch_of(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(HY_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr & 255)) return fail(HY_ERR_HIP, "scratch symbol address unusable");
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_scratch_ptr[dev];
  return HY_OK;
}

}  // namespace

hy_status hy_advance_noalloc(const hy_config* cfg, double* U, int32_t nsteps, double t0,
                             double* out, void* stream) {
  std::string msg;
  if (!validate(cfg, msg)) return fail(HY_ERR_ARG, msg);
  if (!U) return fail(HY_ERR_ARG, "U is NULL");
  if (nsteps < 0) return fail(HY_ERR_ARG, "nsteps must be >= 0");
  if (!std::isfinite(t0)) return fail(HY_ERR_ARG, "t0 must be finite");
  if (has_refine(cfg)) return fail(HY_ERR_ARG, "hy_advance_noalloc does not take refined meshes");
  const size_t need = hy_workspace_bytes(cfg);
  if (need > kNoAllocBytes)
    return fail(HY_ERR_NOMEM, "problem needs " + std::to_string(need) + " workspace bytes; "
                "hy_advance_noalloc holds at most " + std::to_string(kNoAllocBytes));
  int dev;
  HY_HIP(hipGetDevice(&dev));
  char* ws = nullptr;
  hy_status st = scratch_of(dev, &ws);
  if (st != HY_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hy_problem p;
  HeaderBytes hdr;
  SmrLayout L;
  st = build_problem(cfg, ws, kNoAllocBytes, dev, &p, hdr.b, &L);
  if (st != HY_OK) return st;
  {
    DevCounters c;
    std::memcpy(&c, hdr.b + sizeof(DevProblem), sizeof c);
    c.time = t0;
    std::memcpy(hdr.b + sizeof(DevProblem), &c, sizeof c);
  }
  // header (every counter starts cleared), state into the MeshBlockPack,
  // first time step, the steps, result back out; kernels only
  HY_HIP(launch_put_header(hdr, ws, s));
  HY_HIP(launch_scatter(p.dp, U, p.hp.U, p.ncell * 5, 1, s));
  HY_HIP(launch_dt(p.dp, p.ncell, 0, 1, s));
  st = run_batch(std::array<hy_problem*, 1>{&p}.data(), &nsteps, 1, s, nullptr, 1);
  if (st != HY_OK) return st;
  HY_HIP(launch_scatter(p.dp, p.hp.U, U, p.ncell * 5, 0, s));
  if (out) HY_HIP(launch_result(p.dp, (int)(p.steps & 1), out, s));
  return HY_OK;
}
