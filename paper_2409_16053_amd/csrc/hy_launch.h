// hy_launch.h -- host-side entry points of the kernels in hy_kernels.hip.
#pragma once
#include "hy_internal.h"

namespace hy {
int num_stage_variants();
void stage_variant_shape(int v, int* tx, int* ty);
int stage_variant_waves(int v);
const void* stage_kernel(int v, int recon, int prec, int stage, int smr);
hipError_t launch_stage(int v, int recon, int prec, int stage, int smr, const StageArgs& a, int grid,
                        hipStream_t s);
hipError_t launch_fofc(int recon, int prec, const FixArgs& a, int grid_x, hipStream_t s);
int fofc_grid(int nblocks, int bz);
hipError_t launch_combine(const FixArgs& a, int op, int grid_x, hipStream_t s);
hipError_t launch_reset(const DevProblem* p, int slot, int clear, hipStream_t s);
hipError_t launch_dt(const DevProblem* p, int64_t ncell, int slot, int flags, hipStream_t s);
hipError_t launch_scatter(const DevProblem* p, const double* src, double* dst, int64_t n,
                          int to_blocks, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_put_header(const HeaderBytes& h, void* dst, hipStream_t s);
hipError_t launch_result(const DevProblem* p, int slot, double* out, hipStream_t s);
hipError_t launch_smr_ghost(const DevProblem* p, int stage, int ng, int nvirt, const int32_t block[3],
                            hipStream_t s);
hipError_t launch_smr_flux(int recon, int prec, const DevProblem* p, int stage, int parity, int ncf,
                           const int32_t block[3], hipStream_t s);
hipError_t launch_smr_save(const DevProblem* p, int ncf, const int32_t block[3], hipStream_t s);
hipError_t launch_smr_cell(int recon, int prec, const DevProblem* p, int stage, int parity, unsigned seq,
                           int ncf, const int32_t block[3], hipStream_t s);
hipError_t launch_smr_dt(const DevProblem* p, int nleaf, const int32_t block[3], int slot,
                         hipStream_t s);
}  // namespace hy
