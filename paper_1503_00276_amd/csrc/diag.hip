// diag.hip -- FP64 diagnostics on the GPU: charge density from the stored
// particle positions, Gauss-law residual div E - rho (Hemker 2000, Ch. 3,
// Sec. 3.1, Eq. maxwell-1 in normalised units), charge-conservation residual
// (rho1 - rho0)/dt + div J (Sec. 3.2, Eq. continuity), and compensated
// (Neumaier) FP64 sums of the field and particle energies and momentum; plus
// the state export.
#include "pic_dev.h"
#include "pic_kernels.h"

namespace {

constexpr int kBlock = 256;
constexpr int kRedBlocks = 512;

// Node-centred B-spline weights of order 'order' for an offset eps in [0,1):
// nodes base..base+order relative to the particle's cell (FP64).
__device__ __forceinline__ int rho_weights(int order, double eps, double w[4]) {
  if (order == 1) {
    w[0] = 1.0 - eps;
    w[1] = eps;
    return 0;
  }
  if (order == 2) {
    int n = eps >= 0.5 ? 1 : 0;
    double t = eps - n, a = 0.5 - t, b = 0.5 + t;
    w[0] = 0.5 * a * a;
    w[1] = 0.75 - t * t;
    w[2] = 0.5 * b * b;
    return n - 1;
  }
  double f = eps, g = 1.0 - f, f2 = f * f, f3 = f2 * f;
  w[0] = g * g * g / 6.0;
  w[1] = (4.0 - 6.0 * f2 + 3.0 * f3) / 6.0;
  w[2] = (1.0 + 3.0 * f + 3.0 * f2 - 3.0 * f3) / 6.0;
  w[3] = f3 / 6.0;
  return -1;
}

__global__ void __launch_bounds__(kBlock) rho64(const StoreDesc* __restrict__ sp, double* rho) {
  const StoreDesc& S = *sp;
  const GridDesc& g = S.g;
  const int cur = pic_cur(*S.ctl);
  const int np = S.np;
  const int no = g.order + 1;
  const int wo = g.window ? S.win->origin : 0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    const int cell = S.cell[cur][p];
    if (cell < 0) continue;  // removed by a moving window
    int c[3];
    pic_unpack(g, cell, c);
    int wc = c[0] - wo;  // window column (moving window)
    if (wc < 0) wc += g.nx[0];
    double wx[4], wy[4], wz[4] = {1.0, 0.0, 0.0, 0.0};
    int bx = rho_weights(g.order, (double)S.eps[cur][0][p], wx);
    int by = rho_weights(g.order, (double)S.eps[cur][1][p], wy);
    int bz = 0;
    int nz = 1;
    if (g.dim == 3) {
      bz = rho_weights(g.order, (double)S.eps[cur][2][p], wz);
      nz = no;
    }
    double q = (double)S.w[cur][p];
    for (int k = 0; k < nz; k++) {
      int gz = g.dim == 3 ? pic_wrap(c[2] + bz + k, g.nx[2]) : 0;
      for (int j = 0; j < no; j++) {
        int gy;
        if (g.cyl) {
          // r-z: charge below the axis belongs to the mirror row, beyond the
          // wall it is dropped (rows are divided by their ring volume later)
          const int ry = c[1] + by + j;
          gy = ry <= 0 ? 1 - ry : ry;
          if (gy >= g.nx[1]) continue;
        } else {
          gy = pic_wrap(c[1] + by + j, g.nx[1]);
        }
        for (int i = 0; i < no; i++) {
          if (g.window && (unsigned)(wc + bx + i) >= (unsigned)g.nx[0]) continue;  // beyond the window
          int gx = pic_wrap(c[0] + bx + i, g.nx[0]);
          unsafeAtomicAdd(rho + gx + (size_t)g.nx[0] * (gy + (size_t)g.nx[1] * gz), q * wx[i] * wy[j] * wz[k]);
        }
      }
    }
  }
}

// r-z: rho = ion density + (folded ring charge) / (r_j / dr) on the rows
// j >= 1; row 0 holds the image of row 1.
__global__ void rz_rho_finish(double* rho, int nz, int nr, double ion) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nz * nr; c += gridDim.x * blockDim.x) {
    const int j = c / nz;
    if (j >= 1) rho[c] = ion + rho[c] / ((double)j - 0.5);
  }
}

__global__ void rz_rho_mirror(double* rho, int nz) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nz; i += gridDim.x * blockDim.x) rho[i] = rho[nz + i];
}

__global__ void fill64(double* p, double v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// Backward-difference divergence of a 3-component staggered field at node c.
template <typename T>
// wo: ring origin of a moving window (-1 without one); the x1 neighbour
// behind the window's back column is zero.  r-z: the cylindrical divergence
// dV_z/dz + (1/r) d(r V_r)/dr on the rows j >= 1 (V_r on the half rows j and
// j - 1, radii j dr and (j - 1) dr; the row radius (j - 1/2) dr); row 0
// takes the value of row 1.
__device__ __forceinline__ double div_at(const GridDesc& g, const T* V, int nc, int c, int dim, int wo = -1) {
  if (g.cyl) {
    if (c < g.nx[0]) c += g.nx[0];
    const int i = c % g.nx[0];
    const int j = c / g.nx[0];
    const int cxm = (i > 0) ? c - 1 : c + g.nx[0] - 1;
    const double vxm = (wo >= 0 && i == wo) ? 0.0 : (double)V[cxm];
    return ((double)V[c] - vxm) / g.dxd[0] +
           ((double)j * (double)V[nc + c] - (double)(j - 1) * (double)V[nc + c - g.nx[0]]) /
               (((double)j - 0.5) * g.dxd[1]);
  }
  int i = c % g.nx[0];
  int r = c / g.nx[0];
  int j = r % g.nx[1];
  int k = r / g.nx[1];
  int cxm = (i > 0) ? c - 1 : c + g.nx[0] - 1;
  int cym = (j > 0) ? c - g.nx[0] : c + (g.nx[1] - 1) * g.nx[0];
  const double vxm = (wo >= 0 && i == wo) ? 0.0 : (double)V[cxm];
  double d = ((double)V[c] - vxm) / g.dxd[0] +
             ((double)V[nc + c] - (double)V[nc + cym]) / g.dxd[1];
  if (dim == 3) {
    int sz = g.nx[0] * g.nx[1];
    int czm = (k > 0) ? c - sz : c + (g.nx[2] - 1) * sz;
    d += ((double)V[2 * nc + c] - (double)V[2 * nc + czm]) / g.dxd[2];
  }
  return d;
}

__global__ void __launch_bounds__(kBlock) gauss64(const InstDesc* __restrict__ ip, const double* rho, double* G,
                                                  int dim, int fpar) {
  const InstDesc& I = *ip;
  const int nc = I.g.ncell;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x)
    G[c] = div_at(I.g, I.F[fpar], nc, c, dim, I.g.window ? I.win->origin : -1) - rho[c];
}

__global__ void __launch_bounds__(kBlock) charge64(const InstDesc* __restrict__ ip, const double* rho0,
                                                   const double* rho1, double* C, int dim) {
  const InstDesc& I = *ip;
  const int nc = I.g.ncell;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x)
    C[c] = (rho1[c] - rho0[c]) / I.g.dtd + div_at(I.g, I.Jout, nc, c, dim, I.g.window ? I.win->origin : -1);
}

// ---------------------------------------------------------------------------
// compensated sums: each thread keeps Neumaier (sum, compensation) pairs;
// pairs are merged with an error-free two-sum; per-block pairs are combined by
// a second single-block pass.  Deterministic for a fixed launch shape.
// ---------------------------------------------------------------------------

struct Pair {
  double s, c;
};

__device__ __forceinline__ void neumaier(Pair& a, double x) {
  double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}

__device__ __forceinline__ Pair merge(Pair a, Pair b) {
  Pair r{a.s, a.c + b.c};
  neumaier(r, b.s);
  return r;
}

template <int N>
__device__ void block_reduce_store(Pair (&v)[N], double* partial) {
  __shared__ double ss[N][kBlock], sc[N][kBlock];
  for (int k = 0; k < N; k++) {
    ss[k][threadIdx.x] = v[k].s;
    sc[k][threadIdx.x] = v[k].c;
  }
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int k = 0; k < N; k++) {
        Pair a{ss[k][threadIdx.x], sc[k][threadIdx.x]};
        Pair b{ss[k][threadIdx.x + off], sc[k][threadIdx.x + off]};
        Pair r = merge(a, b);
        ss[k][threadIdx.x] = r.s;
        sc[k][threadIdx.x] = r.c;
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < N; k++) {
      partial[(size_t)k * 2 * gridDim.x + 2 * blockIdx.x] = ss[k][0];
      partial[(size_t)k * 2 * gridDim.x + 2 * blockIdx.x + 1] = sc[k][0];
    }
}

// final pass: one block folds nb partial pairs of each of nout sums
__global__ void __launch_bounds__(kBlock) reduce_final(const double* partial, int nb, int nout, double* out) {
  __shared__ double ss[kBlock], sc[kBlock];
  for (int k = 0; k < nout; k++) {
    Pair a{0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      Pair x{partial[(size_t)k * 2 * nb + 2 * b], partial[(size_t)k * 2 * nb + 2 * b + 1]};
      a = merge(a, x);
    }
    ss[threadIdx.x] = a.s;
    sc[threadIdx.x] = a.c;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        Pair r = merge(Pair{ss[threadIdx.x], sc[threadIdx.x]}, Pair{ss[threadIdx.x + off], sc[threadIdx.x + off]});
        ss[threadIdx.x] = r.s;
        sc[threadIdx.x] = r.c;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = ss[0] + sc[0];
    __syncthreads();
  }
}

// sum E^2 and B^2 over all cells (times V/2 applied on the host)
__global__ void __launch_bounds__(kBlock) field_sums(const InstDesc* __restrict__ ip, double* partial, int fpar) {
  const InstDesc& I = *ip;
  const int nc = I.g.ncell;
  Pair v[2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    // r-z: each value weighted by its ring volume in units of dz dr^2:
    // 2 pi r / dr off the axis, pi / 4 for the disc of the half rows on the
    // axis, 0 for the image row 0 of the whole-row components
    double vw = 1.0, vh = 1.0;
    if (I.g.cyl) {
      const int j = c / I.g.nx[0];
      const double two_pi = 6.283185307179586;
      vw = j == 0 ? 0.0 : two_pi * ((double)j - 0.5);
      vh = j == 0 ? 0.25 * 3.141592653589793 : two_pi * (double)j;
    }
    for (int k = 0; k < 3; k++) {
      const float* F = I.F[fpar];
      double e = F[(size_t)k * nc + c], b = F[(size_t)(3 + k) * nc + c];
      // whole rows: E_z, E_theta (k = 0, 2), B_r (k = 1); half rows the others
      neumaier(v[0], (k == 1 ? vh : vw) * e * e);
      neumaier(v[1], (k == 1 ? vw : vh) * b * b);
    }
  }
  block_reduce_store<2>(v, partial);
}

// sum w*rqm*(gamma-1) and w*rqm*u over particles (times V on the host)
__global__ void __launch_bounds__(kBlock) particle_sums(const StoreDesc* __restrict__ sp, double rqm,
                                                        double* partial) {
  const StoreDesc& S = *sp;
  const int cur = pic_cur(*S.ctl);
  Pair v[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < S.np; p += gridDim.x * blockDim.x) {
    if (S.cell[cur][p] < 0) continue;  // removed by a moving window
    double ux = S.u[cur][0][p], uy = S.u[cur][1][p], uz = S.u[cur][2][p];
    double usq = ux * ux + uy * uy + uz * uz;
    double m = (double)S.w[cur][p] * rqm;
    neumaier(v[0], m * (usq / (sqrt(1.0 + usq) + 1.0)));
    neumaier(v[1], m * ux);
    neumaier(v[2], m * uy);
    if (S.g.cyl) {
      // r-z: angular momentum about the axis, r u_theta
      const int row = (S.cell[cur][p] >> S.g.sh1) & S.g.m1;
      const double r = ((double)row + (double)S.eps[cur][1][p] - 0.5) * S.g.dxd[1];
      neumaier(v[3], m * r * uz);
    } else {
      neumaier(v[3], m * uz);
    }
  }
  block_reduce_store<4>(v, partial);
}

__global__ void __launch_bounds__(kBlock) sq_sums(const double* x, int n, double* partial) {
  Pair v[1] = {{0.0, 0.0}};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) neumaier(v[0], x[i] * x[i]);
  block_reduce_store<1>(v, partial);
}

// Export position in cell units (cell + offset), u and w of every particle
// into row id (load order); the host scales positions by the FP64 cell size.
// Rows go to their id (ids = 0..np-1), or, with ids != null (moving window:
// ids have gaps), to their storage index with the id in ids[] (-1 for a
// removed particle) for the host to sort.
__global__ void __launch_bounds__(kBlock) export_state(const StoreDesc* __restrict__ sp, double* out, int* ids) {
  const StoreDesc& S = *sp;
  const GridDesc& g = S.g;
  const int cur = pic_cur(*S.ctl);
  const int stride = g.dim + 4;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < S.np; p += gridDim.x * blockDim.x) {
    const int cell = S.cell[cur][p];
    if (ids) ids[p] = cell < 0 ? -1 : S.id[cur][p];
    if (cell < 0) continue;
    int c[3];
    pic_unpack(g, cell, c);
    double* row = out + (size_t)(ids ? p : S.id[cur][p]) * stride;
    for (int d = 0; d < g.dim; d++) row[d] = (double)c[d] + (double)S.eps[cur][d][p];
    row[g.dim + 0] = S.u[cur][0][p];
    row[g.dim + 1] = S.u[cur][1][p];
    row[g.dim + 2] = S.u[cur][2][p];
    row[g.dim + 3] = S.w[cur][p];
  }
}

__global__ void f32_to_f64(const float* in, double* out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = in[i];
}

__global__ void f64_to_f32(const double* in, float* out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

int grid_for(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  return b < 1 ? 1 : (int)b;
}

}  // namespace

int pic_reduce_blocks() { return kRedBlocks; }

hipError_t pic_launch_rho64(const StoreDesc* d_store, int np_max, double* rho, hipStream_t st) {
  hipLaunchKernelGGL(rho64, dim3(grid_for(np_max)), dim3(kBlock), 0, st, d_store, rho);
  return hipGetLastError();
}

hipError_t pic_launch_rz_rho_finish(double* rho, int nz, int nr, double ion, hipStream_t st) {
  hipLaunchKernelGGL(rz_rho_finish, dim3(grid_for((size_t)nz * nr)), dim3(kBlock), 0, st, rho, nz, nr, ion);
  hipLaunchKernelGGL(rz_rho_mirror, dim3(grid_for((size_t)nz)), dim3(kBlock), 0, st, rho, nz);
  return hipGetLastError();
}

hipError_t pic_launch_fill64(double* p, double v, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(fill64, dim3(grid_for(n)), dim3(kBlock), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t pic_launch_gauss64(const InstDesc* d_inst, const double* rho, double* G, int ncell, int dim, int fpar,
                              hipStream_t st) {
  hipLaunchKernelGGL(gauss64, dim3(grid_for(ncell)), dim3(kBlock), 0, st, d_inst, rho, G, dim, fpar);
  return hipGetLastError();
}

hipError_t pic_launch_charge64(const InstDesc* d_inst, const double* rho0, const double* rho1, double* C,
                               int ncell, int dim, hipStream_t st) {
  hipLaunchKernelGGL(charge64, dim3(grid_for(ncell)), dim3(kBlock), 0, st, d_inst, rho0, rho1, C, dim);
  return hipGetLastError();
}

hipError_t pic_launch_field_sums(const InstDesc* d_inst, int ncell, int fpar, double* scratch, double* out,
                                 hipStream_t st) {
  (void)ncell;
  hipLaunchKernelGGL(field_sums, dim3(kRedBlocks), dim3(kBlock), 0, st, d_inst, scratch, fpar);
  hipLaunchKernelGGL(reduce_final, dim3(1), dim3(kBlock), 0, st, scratch, kRedBlocks, 2, out);
  return hipGetLastError();
}

hipError_t pic_launch_particle_sums(const StoreDesc* d_store, int np, double rqm, double* scratch, double* out,
                                    hipStream_t st) {
  (void)np;
  hipLaunchKernelGGL(particle_sums, dim3(kRedBlocks), dim3(kBlock), 0, st, d_store, rqm, scratch);
  hipLaunchKernelGGL(reduce_final, dim3(1), dim3(kBlock), 0, st, scratch, kRedBlocks, 4, out);
  return hipGetLastError();
}

hipError_t pic_launch_sq_sums(const double* v, int n, double* scratch, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sq_sums, dim3(kRedBlocks), dim3(kBlock), 0, st, v, n, scratch);
  hipLaunchKernelGGL(reduce_final, dim3(1), dim3(kBlock), 0, st, scratch, kRedBlocks, 1, out);
  return hipGetLastError();
}

hipError_t pic_launch_export_state(const StoreDesc* d_store, int np, double* out, int* ids, hipStream_t st) {
  hipLaunchKernelGGL(export_state, dim3(grid_for(np)), dim3(kBlock), 0, st, d_store, out, ids);
  return hipGetLastError();
}

hipError_t pic_launch_f32_to_f64(const float* in, double* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(f32_to_f64, dim3(grid_for(n)), dim3(kBlock), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t pic_launch_f64_to_f32(const double* in, float* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(f64_to_f32, dim3(grid_for(n)), dim3(kBlock), 0, st, in, out, n);
  return hipGetLastError();
}
