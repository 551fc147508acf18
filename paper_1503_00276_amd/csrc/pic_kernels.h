// pic_kernels.h -- host-side launchers of the HIP kernels (one translation
// unit per kernel family; the runtime calls only these).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "pic_dev.h"

// fused gather + push + deposit (gpd.hip)
size_t pic_gpd_lds_bytes(const GridDesc& g);
// LDS of step kstep of a sort cycle (at most pic_gpd_lds_bytes)
size_t pic_gpd_lds_bytes_step(const GridDesc& g, int kstep);
int pic_gpd_block();
// particles a work item of the two-phase 3D variant can hold (its chunk limit)
int pic_gpd_split_chunk();
// the two-phase periodic 2D kernel (mode 7): whether a grid takes it, and the
// particles one of its work items can hold
bool pic_gpd_two_phase2(const GridDesc& g);
int pic_gpd_two_phase2_chunk();
// padded LDS strides of the two-phase variant for g's tile and stray bound
void pic_gpd_split_strides(GridDesc& g);
int pic_gpd_max_group();
// allow the LDS size a group needs (call before launching or capturing);
// mode: the boundary logic of the group's stores (0 periodic, 1 moving window
// along x1, 2 the 2D r-z geometry, 3 r-z with a moving window, 4 periodic 3D
// in two phases, 5 the same with the compile-time LDS strides of 4x4xN
// tiles), which selects the kernel variant
hipError_t pic_gpd_prepare(int dim, int order, int mode, size_t lds);
// workgroups of the variant that are resident on one CU at once with 'lds'
// bytes of dynamic LDS (after pic_gpd_prepare)
int pic_gpd_resident(int dim, int order, int mode, size_t lds);
// kstep: steps done since the last rebin check (bounds the staged halo);
// ev0 / ev1 (may be null): events stamped at the kernel's start / end
hipError_t pic_launch_gpd(int dim, int order, int mode, const StoreDesc* d_stores, int nstores, int grid,
                          size_t lds, int parity, int kstep, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);

// Yee field solve (field.hip); instances in d_inst[0..ninst)
int pic_yee_tiles(int dim, const int nx[3]);
hipError_t pic_launch_window_advance(const InstDesc* d_inst, int ninst, hipStream_t st);
hipError_t pic_launch_smooth_pass(const InstDesc* d_inst, int ninst, int max_ncell, int axis, int lev,
                                  int parity, hipStream_t st);
// cart / cyl: the group holds Cartesian / r-z instances (each kernel skips the
// others); window: some instance has a moving window (selects the variant
// with the window terms)
// Per store: this step's fixed point of the one-phase kernels' FP32 current
// (from the store's bound on |u| and the instance's bound on |E_c|).
hipError_t pic_launch_current_units(StoreDesc* d_stores, int nstores, hipStream_t st);
hipError_t pic_launch_yee_step(const InstDesc* d_inst, int ninst, int max_tiles, int dim, bool cart, bool cyl,
                               bool window, int parity, hipStream_t st);

// tile rebin (sort.hip); stores in d_stores[0..nstores)
hipError_t pic_launch_rebin(const StoreDesc* d_stores, int nstores, int max_items, int total_tiles,
                            int total_blocks, int inject_max, hipStream_t st);

// diagnostics (diag.hip)
hipError_t pic_launch_rho64(const StoreDesc* d_store, int np_max, double* rho, hipStream_t st);
hipError_t pic_launch_fill64(double* p, double v, size_t n, hipStream_t st);
// r-z: rho = ion + folded charge / (r_j/dr) on rows j >= 1, row 0 = row 1
hipError_t pic_launch_rz_rho_finish(double* rho, int nz, int nr, double ion, hipStream_t st);
hipError_t pic_launch_gauss64(const InstDesc* d_inst, const double* rho, double* G, int ncell, int dim,
                              int fpar, hipStream_t st);
hipError_t pic_launch_charge64(const InstDesc* d_inst, const double* rho0, const double* rho1,
                               double* C, int ncell, int dim, hipStream_t st);
// compensated FP64 sums: out[0..nout) with partial scratch (>= 2*nout*pic_reduce_blocks() doubles)
int pic_reduce_blocks();
hipError_t pic_launch_field_sums(const InstDesc* d_inst, int ncell, int fpar, double* scratch, double* out,
                                 hipStream_t st);
hipError_t pic_launch_particle_sums(const StoreDesc* d_store, int np, double rqm, double* scratch,
                                    double* out, hipStream_t st);
hipError_t pic_launch_sq_sums(const double* v, int n, double* scratch, double* out, hipStream_t st);
hipError_t pic_launch_export_state(const StoreDesc* d_store, int np, double* out, int* ids, hipStream_t st);
hipError_t pic_launch_f32_to_f64(const float* in, double* out, size_t n, hipStream_t st);
hipError_t pic_launch_f64_to_f32(const double* in, float* out, size_t n, hipStream_t st);
