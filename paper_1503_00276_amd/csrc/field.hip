// field.hip -- Yee FDTD field solve on periodic FP32 planes (Hemker 2000,
// Ch. 3, Sec. 3.2 Eqs. 2d-field-solve-b-part1, 2d-field-solve-e,
// 2d-field-solve-b-part2; Sec. 3.3 for the x3 terms of 3D).
//
// One step of the solve is  B -= (dt/2) curl E ;  E += dt (curl B - J) ;
// B -= (dt/2) curl E  with forward differences for curl E (E -> B mesh) and
// backward differences for curl B (B -> E mesh).  The E3 update subtracts J3
// (the printed j1 of the 2D E3 equation is a typo: the B terms are the curl's
// third component).  Every kernel is one thread per cell, coalesced along x1,
// periodic neighbours by wrap; blockIdx.y selects the instance of a batch.
#include "pic_dev.h"
#include "pic_kernels.h"

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void cell_coords(const GridDesc& g, int c, int& i, int& j, int& k) {
  i = c % g.nx[0];
  int r = c / g.nx[0];
  j = r % g.nx[1];
  k = r / g.nx[1];
}

__global__ void __launch_bounds__(kBlock) zero_current(const InstDesc* __restrict__ inst) {
  const InstDesc& I = inst[blockIdx.y];
  const int n = 3 * I.g.ncell;
  if (I.g.acc_mode == 2) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) I.J64[c] = 0ull;
  } else {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) I.J[c] = 0.0f;
  }
}

// Deterministic mode: the int64 fixed-point current becomes the FP32 current.
__global__ void __launch_bounds__(kBlock) fold_current(const InstDesc* __restrict__ inst) {
  const InstDesc& I = inst[blockIdx.y];
  if (I.g.acc_mode != 2) return;
  const int n = 3 * I.g.ncell;
  const double inv = (double)I.g.jinv;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    I.J[c] = (float)((double)(long long)I.J64[c] * inv);
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) yee_b(const InstDesc* __restrict__ inst, float hfrac) {
  const InstDesc& I = inst[blockIdx.y];
  const GridDesc& g = I.g;
  const int nc = g.ncell;
  const float h = hfrac * g.dt;
  const float* E1 = I.F;
  const float* E2 = I.F + nc;
  const float* E3 = I.F + 2 * nc;
  float* B1 = I.F + 3 * nc;
  float* B2 = I.F + 4 * nc;
  float* B3 = I.F + 5 * nc;
  const int sx = 1, sy = g.nx[0], sz = g.nx[0] * g.nx[1];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    int i, j, k;
    cell_coords(g, c, i, j, k);
    int cxp = c + (i + 1 < g.nx[0] ? sx : sx - g.nx[0] * sx);
    int cyp = c + (j + 1 < g.nx[1] ? sy : sy - g.nx[1] * sy);
    float e1 = E1[c], e2 = E2[c], e3 = E3[c];
    float d2E3 = (E3[cyp] - e3) * g.rdx[1];
    float d1E3 = (E3[cxp] - e3) * g.rdx[0];
    float d1E2 = (E2[cxp] - e2) * g.rdx[0];
    float d2E1 = (E1[cyp] - e1) * g.rdx[1];
    float d3E2 = 0.0f, d3E1 = 0.0f;
    if (DIM == 3) {
      int czp = c + (k + 1 < g.nx[2] ? sz : sz - g.nx[2] * sz);
      d3E2 = (E2[czp] - e2) * g.rdx[2];
      d3E1 = (E1[czp] - e1) * g.rdx[2];
    }
    B1[c] -= h * (d2E3 - d3E2);
    B2[c] -= h * (d3E1 - d1E3);
    B3[c] -= h * (d1E2 - d2E1);
  }
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) yee_e(const InstDesc* __restrict__ inst) {
  const InstDesc& I = inst[blockIdx.y];
  const GridDesc& g = I.g;
  const int nc = g.ncell;
  const float dt = g.dt;
  float* E1 = I.F;
  float* E2 = I.F + nc;
  float* E3 = I.F + 2 * nc;
  const float* B1 = I.F + 3 * nc;
  const float* B2 = I.F + 4 * nc;
  const float* B3 = I.F + 5 * nc;
  const float* J1 = I.J;
  const float* J2 = I.J + nc;
  const float* J3 = I.J + 2 * nc;
  const int sx = 1, sy = g.nx[0], sz = g.nx[0] * g.nx[1];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    int i, j, k;
    cell_coords(g, c, i, j, k);
    int cxm = c - (i > 0 ? sx : sx - g.nx[0] * sx);
    int cym = c - (j > 0 ? sy : sy - g.nx[1] * sy);
    float b1 = B1[c], b2 = B2[c], b3 = B3[c];
    float d2B3 = (b3 - B3[cym]) * g.rdx[1];
    float d1B3 = (b3 - B3[cxm]) * g.rdx[0];
    float d1B2 = (b2 - B2[cxm]) * g.rdx[0];
    float d2B1 = (b1 - B1[cym]) * g.rdx[1];
    float d3B2 = 0.0f, d3B1 = 0.0f;
    if (DIM == 3) {
      int czm = c - (k > 0 ? sz : sz - g.nx[2] * sz);
      d3B2 = (b2 - B2[czm]) * g.rdx[2];
      d3B1 = (b1 - B1[czm]) * g.rdx[2];
    }
    E1[c] += dt * ((d2B3 - d3B2) - J1[c]);
    E2[c] += dt * ((d3B1 - d1B3) - J2[c]);
    E3[c] += dt * ((d1B2 - d2B1) - J3[c]);
  }
}

int grid_for(int max_n) {
  int b = (max_n + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  return b < 1 ? 1 : b;
}

}  // namespace

hipError_t pic_launch_zero_current(const InstDesc* d_inst, int ninst, int max_ncell, hipStream_t st) {
  hipLaunchKernelGGL(zero_current, dim3(grid_for(3 * max_ncell), ninst), dim3(kBlock), 0, st, d_inst);
  return hipGetLastError();
}

hipError_t pic_launch_fold_current(const InstDesc* d_inst, int ninst, int max_ncell, hipStream_t st) {
  hipLaunchKernelGGL(fold_current, dim3(grid_for(3 * max_ncell), ninst), dim3(kBlock), 0, st, d_inst);
  return hipGetLastError();
}

hipError_t pic_launch_yee_b(const InstDesc* d_inst, int ninst, int max_ncell, int dim, float hfrac,
                            hipStream_t st) {
  if (dim == 2)
    hipLaunchKernelGGL(yee_b<2>, dim3(grid_for(max_ncell), ninst), dim3(kBlock), 0, st, d_inst, hfrac);
  else
    hipLaunchKernelGGL(yee_b<3>, dim3(grid_for(max_ncell), ninst), dim3(kBlock), 0, st, d_inst, hfrac);
  return hipGetLastError();
}

hipError_t pic_launch_yee_e(const InstDesc* d_inst, int ninst, int max_ncell, int dim, hipStream_t st) {
  if (dim == 2)
    hipLaunchKernelGGL(yee_e<2>, dim3(grid_for(max_ncell), ninst), dim3(kBlock), 0, st, d_inst);
  else
    hipLaunchKernelGGL(yee_e<3>, dim3(grid_for(max_ncell), ninst), dim3(kBlock), 0, st, d_inst);
  return hipGetLastError();
}
