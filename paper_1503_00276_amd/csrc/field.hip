// field.hip -- Yee FDTD field solve on periodic FP32 planes (Hemker 2000,
// Ch. 3, Sec. 3.2 Eqs. 2d-field-solve-b-part1, 2d-field-solve-e,
// 2d-field-solve-b-part2; Sec. 3.3 for the x3 terms of 3D).
//
// One step of the solve is  B -= (dt/2) curl E ;  E += dt (curl B - J) ;
// B -= (dt/2) curl E  with forward differences for curl E (E -> B mesh) and
// backward differences for curl B (B -> E mesh).  The E3 update subtracts J3
// (the printed j1 of the 2D E3 equation is a typo: the B terms are the curl's
// third component).  All three parts run in one kernel on LDS tiles; periodic
// neighbours by wrap; blockIdx.y selects the instance of a batch.
#include "pic_dev.h"
#include "pic_kernels.h"

namespace {

constexpr int kBlock = 256;

typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) unsigned int guint;

// Tile of cells one workgroup advances (256 cells, one per thread).
template <int DIM> struct YeeTile;
template <> struct YeeTile<2> { static constexpr int X = 32, Y = 8, Z = 1; };
template <> struct YeeTile<3> { static constexpr int X = 16, Y = 4, Z = 4; };

// One full field step on a tile, B^n, E^n -> B^{n+1}, E^{n+1}, in LDS:
//   Bh  = B^n - (dt/2) curl+ E^n     on the tile plus one node below and above
//   E'  = E^n + dt (curl- Bh - J)    on the tile plus one node above
//   B'  = Bh - (dt/2) curl+ E'       on the tile
// The halos are recomputed by every tile that needs them, with the same
// arithmetic on the same inputs, so neighbouring tiles agree bitwise.
// The current of the step is read from the accumulator the particle kernel
// filled (int64 fixed point in the deterministic mode; which of the two is
// the step's parity), copied to Jout, and the other accumulator is cleared
// for the next step.
// The fields are double-buffered: the step reads E^n, B^n from set par and
// writes E^{n+1}, B^{n+1} to the other set, so a tile never reads a halo
// node that a neighbouring workgroup has already advanced.
// Periodic wrap for an index at most one period out of range.
__device__ __forceinline__ int wrap1(int v, int n) {
  v = v < 0 ? v + n : v;
  v = v >= n ? v - n : v;
  return v >= n ? v - n : v;
}

// WIN: compiled with the moving-window terms (launched for groups that hold a
// moving window).
// The fixed point of this step's current, per store whose particles take
// the one-phase fused kernel with FP32 accumulation (Cartesian).  A
// contribution of particle p to one node is at most |w_p| |v_p| (the charge
// fraction that crosses a face in a step is at most the displacement in
// cells; the transverse weight is at most one), and the Boris step changes
// |u| by at most |q/m| dt |E| at the particle, where a gathered E_c is a
// convex combination of node values: |E| <= sqrt(3) max|E_c| + |E_0|.  The
// store keeps umax, a bound on |u| at the start of the step, and the
// instance a running bound on |E_c| (set at a field load, raised by the Yee
// step), so V = max|w| min(1, umax + kick) bounds every contribution of the
// step, and the unit 2^-e with 2^e V 1.0001 < 2^31 keeps each inside an
// int32: it follows the plasma's speed rather than c.  umax then advances
// by the kick for the next step.  The int64 mode keeps the instance's unit
// (its sums are exact in one unit), and so do r-z (whose field step keeps no
// bound) and the two-phase 3D kernel (which takes a unit per work item).
__global__ void current_units(StoreDesc* __restrict__ stores, int nstores) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nstores) return;
  StoreDesc& D = stores[k];
  const GridDesc& g = D.g;
  if (g.acc_mode == 2 || g.cyl || pic_gpd_split(g)) return;
  const float em = *(const gfloat*)D.emax;
  const float e0n = sqrtf(g.e0[0] * g.e0[0] + g.e0[1] * g.e0[1] + g.e0[2] * g.e0[2]);
  const float kick = fabsf(D.qm) * g.dt * (1.7320509f * em + e0n) * 1.0001f;
  const float um = (D.ctl->umax + kick) * 1.000001f;
  D.ctl->umax = um;
  const float V = D.wmax * fminf(1.0f, um * 1.0001f);
  int ex = 0;
  (void)frexpf(V * 1.0001f, &ex);
  const int e = V > 0.0f ? min(100, max(-100, 31 - ex)) : 100;
  D.g.jscale = ldexpf(1.0f, e);
  D.g.jinv = ldexpf(1.0f, -e);
}

template <int DIM, bool WIN>
__global__ void __launch_bounds__(kBlock) yee_step(const InstDesc* __restrict__ inst, int par) {
  using T = YeeTile<DIM>;
  constexpr int EXM = T::X + 3, EYM = T::Y + 3, EZM = DIM == 3 ? T::Z + 3 : 1;
  constexpr int BXM = T::X + 2, BYM = T::Y + 2, BZM = DIM == 3 ? T::Z + 2 : 1;
  __shared__ float sE[3][EZM * EYM * EXM];
  __shared__ float sB[3][BZM * BYM * BXM];
  const InstDesc& I = inst[blockIdx.y];
  const GridDesc& g = I.g;
  if (g.cyl) return;  // r-z instances take yee_step_rz
  const int ntx = (g.nx[0] + T::X - 1) / T::X;
  const int nty = (g.nx[1] + T::Y - 1) / T::Y;
  const int ntz = DIM == 3 ? (g.nx[2] + T::Z - 1) / T::Z : 1;
  const int tile = blockIdx.x;
  // thread layout = tile shape (T::X * T::Y * T::Z == blockDim.x)
  const int tx = threadIdx.x % T::X;
  const int ty = (threadIdx.x / T::X) % T::Y;
  const int tz = threadIdx.x / (T::X * T::Y);
  if (tile < ntx * nty * ntz) {
    const int nc = g.ncell;
    const int n0 = g.nx[0], n1 = g.nx[1], n2 = g.nx[2];
    const int o0 = (tile % ntx) * T::X;
    const int o1 = ((tile / ntx) % nty) * T::Y;
    const int o2 = DIM == 3 ? (tile / (ntx * nty)) * T::Z : 0;
    const int e0 = min(T::X, n0 - o0);
    const int e1 = min(T::Y, n1 - o1);
    const int e2 = DIM == 3 ? min(T::Z, n2 - o2) : 1;
    const int EX = e0 + 3, EY = e1 + 3, EZ = DIM == 3 ? e2 + 3 : 1;
    const int BX = e0 + 2, BY = e1 + 2, BZ = DIM == 3 ? e2 + 2 : 1;
    const int zoff = DIM == 3 ? 1 : 0;  // region origin is one node below the tile
    // moving window: the window column of region x index x (the x1 neighbour
    // beyond the window's front or back is zero), and whether the window
    // moves after this step (its back column then becomes the new, empty front)
    const bool win = WIN && g.window != 0;
    int wo = 0;
    bool wshift = false;
    if (win) {
      const WinCtl wc = *I.win;
      wo = wc.origin;
      wshift = pic_win_shifts(g.wa, wc.step + 1) > pic_win_shifts(g.wa, wc.step);
    }
    auto wcol = [&](int x) {
      int r = wrap1(o0 - 1 + x, n0) - wo;
      return r < 0 ? r + n0 : r;
    };
    auto gidx = [&](int x, int y, int z) {
      int gx = wrap1(o0 - 1 + x, n0);
      int gy = wrap1(o1 - 1 + y, n1);
      int gz = DIM == 3 ? wrap1(o2 - zoff + z, n2) : 0;
      return gx + n0 * (gy + n1 * gz);
    };
    const gfloat* F = (const gfloat*)I.F[par];
    // staging: the region's nodes in flat order, U per thread and round,
    // every load of a round issued before its first LDS write (so a thread
    // waits for memory once per round, not once per node and field)
    {
      constexpr int U = DIM == 3 ? 4 : 2;
      const int EN = EX * EY * EZ;
      for (int q0 = threadIdx.x; q0 < EN; q0 += U * kBlock) {
        float v[U][6];
        int rb[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int q = q0 + u * kBlock;
          rb[u] = -2;  // -2: no node, -1: node outside the B region
          if (q < EN) {
            const int x = q % EX, y = (q / EX) % EY, z = DIM == 3 ? q / (EX * EY) : 0;
            const int gi = gidx(x, y, z);
            v[u][0] = F[gi];
            v[u][1] = F[nc + gi];
            v[u][2] = F[2 * nc + gi];
            rb[u] = -1;
            if (x < BX && y < BY && z < BZ) {
              rb[u] = x + BX * (y + BY * z);
              v[u][3] = F[3 * nc + gi];
              v[u][4] = F[4 * nc + gi];
              v[u][5] = F[5 * nc + gi];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int q = q0 + u * kBlock;  // region index x + EX (y + EY z)
          if (rb[u] == -2) continue;
          sE[0][q] = v[u][0];
          sE[1][q] = v[u][1];
          sE[2][q] = v[u][2];
          if (rb[u] >= 0) {
            sB[0][rb[u]] = v[u][3];
            sB[1][rb[u]] = v[u][4];
            sB[2][rb[u]] = v[u][5];
          }
        }
      }
    }
    __syncthreads();
    const float h = 0.5f * g.dt;
    const float r0 = g.rdx[0], r1 = g.rdx[1], r2 = g.rdx[2];
    const int EXY = EX * EY;
    // Bh on the whole B region
    for (int z = (DIM == 3 ? tz : 0); z < BZ; z += T::Z)
      for (int y = ty; y < BY; y += T::Y)
        for (int x = tx; x < BX; x += T::X) {
          int r = x + BX * (y + BY * z);
          int c = x + EX * (y + EY * z);
          const bool front = win && wcol(x) == n0 - 1;
          float d2E3 = (sE[2][c + EX] - sE[2][c]) * r1;
          float d1E3 = ((front ? 0.0f : sE[2][c + 1]) - sE[2][c]) * r0;
          float d1E2 = ((front ? 0.0f : sE[1][c + 1]) - sE[1][c]) * r0;
          float d2E1 = (sE[0][c + EX] - sE[0][c]) * r1;
          float d3E2 = 0.0f, d3E1 = 0.0f;
          if (DIM == 3) {
            d3E2 = (sE[1][c + EXY] - sE[1][c]) * r2;
            d3E1 = (sE[0][c + EXY] - sE[0][c]) * r2;
          }
          sB[0][r] -= h * (d2E3 - d3E2);
          sB[1][r] -= h * (d3E1 - d1E3);
          sB[2][r] -= h * (d1E2 - d2E1);
        }
    __syncthreads();
    // E' on the tile plus one node above: region nodes 1 .. e+1 per axis
    const int jp = par, jn = 1 - par;
    const double jinv = (double)g.jinv;
    const int BXY = BX * BY;
    for (int z = zoff + (DIM == 3 ? tz : 0); z <= (DIM == 3 ? e2 + 1 : 0); z += T::Z)
      for (int y = 1 + ty; y <= e1 + 1; y += T::Y)
        for (int x = 1 + tx; x <= e0 + 1; x += T::X) {
          int ce = x + EX * (y + EY * z);
          int cb = x + BX * (y + BY * z);
          int gi = gidx(x, y, z);
          float J1, J2, J3;
          if (I.sm_npass > 0) {
            const gfloat* Js = (const gfloat*)I.Jsm[(I.sm_npass - 1) & 1];
            J1 = Js[gi];
            J2 = Js[nc + gi];
            J3 = Js[2 * nc + gi];
          } else if (g.acc_mode == 2) {
            J1 = (float)((double)(long long)I.J64[jp][gi] * jinv);
            J2 = (float)((double)(long long)I.J64[jp][nc + gi] * jinv);
            J3 = (float)((double)(long long)I.J64[jp][2 * nc + gi] * jinv);
          } else {
            const gfloat* Ja = (const gfloat*)I.Jacc[jp];
            J1 = Ja[gi];
            J2 = Ja[nc + gi];
            J3 = Ja[2 * nc + gi];
          }
          const bool back = win && wcol(x) == 0;
          float d2B3 = (sB[2][cb] - sB[2][cb - BX]) * r1;
          float d1B3 = (sB[2][cb] - (back ? 0.0f : sB[2][cb - 1])) * r0;
          float d1B2 = (sB[1][cb] - (back ? 0.0f : sB[1][cb - 1])) * r0;
          float d2B1 = (sB[0][cb] - sB[0][cb - BX]) * r1;
          float d3B2 = 0.0f, d3B1 = 0.0f;
          if (DIM == 3) {
            d3B2 = (sB[1][cb] - sB[1][cb - BXY]) * r2;
            d3B1 = (sB[0][cb] - sB[0][cb - BXY]) * r2;
          }
          sE[0][ce] += g.dt * ((d2B3 - d3B2) - J1);
          sE[1][ce] += g.dt * ((d3B1 - d1B3) - J2);
          sE[2][ce] += g.dt * ((d1B2 - d2B1) - J3);
          // the tile's own cells: keep the step's current and clear the other accumulator
          if (x <= e0 && y <= e1 && (DIM == 2 || z <= e2)) {
            gfloat* Jo = (gfloat*)I.Jout;
            const float keep = (back && wshift) ? 0.0f : 1.0f;  // discarded column
            Jo[gi] = J1 * keep;
            Jo[nc + gi] = J2 * keep;
            Jo[2 * nc + gi] = J3 * keep;
            if (g.acc_mode == 2) {
              I.J64[jn][gi] = 0ull;
              I.J64[jn][nc + gi] = 0ull;
              I.J64[jn][2 * nc + gi] = 0ull;
            } else {
              gfloat* Jz = (gfloat*)I.Jacc[jn];
              Jz[gi] = 0.0f;
              Jz[nc + gi] = 0.0f;
              Jz[2 * nc + gi] = 0.0f;
            }
          }
        }
    __syncthreads();
    // B' on the tile, and write E', B' back; the largest |E'_c| written
    // raises the instance's running field bound (read by the particle
    // kernel for its current unit)
    gfloat* Fw = (gfloat*)I.F[1 - par];
    float em = 0.0f;
    const float emax0 = *(const gfloat*)I.emax;
    for (int z = zoff + (DIM == 3 ? tz : 0); z <= (DIM == 3 ? e2 : 0); z += T::Z)
      for (int y = 1 + ty; y <= e1; y += T::Y)
        for (int x = 1 + tx; x <= e0; x += T::X) {
          int c = x + EX * (y + EY * z);
          int cb = x + BX * (y + BY * z);
          const int wx = win ? wcol(x) : 1;
          const bool front = win && wx == n0 - 1;
          float d2E3 = (sE[2][c + EX] - sE[2][c]) * r1;
          float d1E3 = ((front ? 0.0f : sE[2][c + 1]) - sE[2][c]) * r0;
          float d1E2 = ((front ? 0.0f : sE[1][c + 1]) - sE[1][c]) * r0;
          float d2E1 = (sE[0][c + EX] - sE[0][c]) * r1;
          float d3E2 = 0.0f, d3E1 = 0.0f;
          if (DIM == 3) {
            d3E2 = (sE[1][c + EXY] - sE[1][c]) * r2;
            d3E1 = (sE[0][c + EXY] - sE[0][c]) * r2;
          }
          int gi = gidx(x, y, z);
          // the window's back column becomes its empty front after a shift
          const float keep = (win && wshift && wx == 0) ? 0.0f : 1.0f;
          Fw[3 * nc + gi] = (sB[0][cb] - h * (d2E3 - d3E2)) * keep;
          Fw[4 * nc + gi] = (sB[1][cb] - h * (d3E1 - d1E3)) * keep;
          Fw[5 * nc + gi] = (sB[2][cb] - h * (d1E2 - d2E1)) * keep;
          Fw[gi] = sE[0][c] * keep;
          Fw[nc + gi] = sE[1][c] * keep;
          Fw[2 * nc + gi] = sE[2][c] * keep;
          em = fmaxf(em, fmaxf(fabsf(sE[0][c]), fmaxf(fabsf(sE[1][c]), fabsf(sE[2][c]))));
        }
    if (__ballot(em > emax0)) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) em = fmaxf(em, __shfl_xor(em, off));
      if ((threadIdx.x & 63) == 0)
        __hip_atomic_fetch_max((guint*)I.emax, __float_as_uint(em), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The periodic 3D field step marching along z.  A workgroup owns a 32x8
// column of cells in x-y and a run of kMarchZ planes, and keeps a rolling
// window of planes in LDS: E at z+1 and z+2, Bh at z and z+1, E' at z and
// z+1.  Each plane of E, B and J is read once per column (plus the x-y halo
// and two planes at the start of a run), instead of once per 16x4x4 tile
// with a halo on every face.  The arithmetic is that of yee_step, term by
// term, so the two agree bitwise:
//   Bh(z+1) = B(z+1) - (dt/2) curl+ E        (E at z+1, and z+2 for d/dz)
//   E'(z+1) = E(z+1) + dt (curl- Bh - J)      (Bh at z+1, and z for d/dz)
//   B'(z)   = Bh(z) - (dt/2) curl+ E'         (E' at z, and z+1 for d/dz)
// x-y indices are region-relative with the origin one node below the column
// (E region 35x11, B region 34x10); E' is formed on nodes 1..e+1, B' on the
// column's own nodes 1..e.
struct MarchTile { static constexpr int X = 32, Y = 8; };
constexpr int kMarchZ = 32;
constexpr int kMarchE = (MarchTile::X + 3) * (MarchTile::Y + 3);
constexpr int kMarchB = (MarchTile::X + 2) * (MarchTile::Y + 2);

__global__ void __launch_bounds__(kBlock) yee_march3(const InstDesc* __restrict__ inst, int par) {
  __shared__ float sE[2][3][kMarchE];
  __shared__ float sBh[2][3][kMarchB];
  __shared__ float sEp[2][3][kMarchE];
  const InstDesc& I = inst[blockIdx.y];
  const GridDesc& g = I.g;
  if (g.cyl || g.window) return;  // launched for periodic Cartesian groups only
  const int n0 = g.nx[0], n1 = g.nx[1], n2 = g.nx[2];
  const int ntx = (n0 + MarchTile::X - 1) / MarchTile::X;
  const int nty = (n1 + MarchTile::Y - 1) / MarchTile::Y;
  const int ntz = (n2 + kMarchZ - 1) / kMarchZ;
  const int tile = blockIdx.x;
  if (tile >= ntx * nty * ntz) return;
  const int tid = threadIdx.x;
  const int o0 = (tile % ntx) * MarchTile::X;
  const int o1 = ((tile / ntx) % nty) * MarchTile::Y;
  const int z0 = (tile / (ntx * nty)) * kMarchZ;
  const int z1 = min(z0 + kMarchZ, n2);
  const int e0 = min(MarchTile::X, n0 - o0), e1 = min(MarchTile::Y, n1 - o1);
  const int EX = e0 + 3, EY = e1 + 3, BX = e0 + 2, BY = e1 + 2;
  const int EN = EX * EY, BN = BX * BY, PX = e0 + 1, PN = PX * (e1 + 1);
  const size_t nc = (size_t)g.ncell;
  const size_t pl = (size_t)n0 * n1;
  const float h = 0.5f * g.dt, dt = g.dt;
  const float r0 = g.rdx[0], r1 = g.rdx[1], r2 = g.rdx[2];
  const gfloat* F = (const gfloat*)I.F[par];
  gfloat* Fw = (gfloat*)I.F[1 - par];
  const int jp = par, jn = 1 - par;
  const double jinv = (double)g.jinv;
  auto col = [&](int x, int y) {  // x-y offset of region node (x, y)
    return (size_t)wrap1(o0 - 1 + x, n0) + (size_t)n0 * wrap1(o1 - 1 + y, n1);
  };
  auto zoff = [&](int z) { return (size_t)wrap1(z, n2) * pl; };
  // A plane's global reads are issued together into registers (each thread
  // holds at most two nodes of each region), so a plane waits for one memory
  // latency rather than one per sub-update.
  // E of plane z on the E region
  auto get_e = [&](int z, float (&v)[2][3]) {
    const size_t zo = zoff(z);
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const int q = tid + k * kBlock;
      if (q < EN) {
        const size_t gi = zo + col(q % EX, q / EX);
        v[k][0] = F[gi];
        v[k][1] = F[nc + gi];
        v[k][2] = F[2 * nc + gi];
      }
    }
  };
  auto put_e = [&](int b, const float (&v)[2][3]) {
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const int q = tid + k * kBlock;
      if (q < EN) {
        sE[b][0][q] = v[k][0];
        sE[b][1][q] = v[k][1];
        sE[b][2][q] = v[k][2];
      }
    }
  };
  // B of plane z on the B region
  auto get_b = [&](int z, float (&v)[2][3]) {
    const size_t zo = zoff(z);
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const int q = tid + k * kBlock;
      if (q < BN) {
        const size_t gi = zo + col(q % BX, q / BX);
        v[k][0] = F[3 * nc + gi];
        v[k][1] = F[4 * nc + gi];
        v[k][2] = F[5 * nc + gi];
      }
    }
  };
  // J of plane z on the E' nodes 1..e+1
  auto get_j = [&](int z, float (&v)[2][3]) {
    const size_t zo = zoff(z);
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const int q = tid + k * kBlock;
      if (q < PN) {
        const size_t gi = zo + col(1 + q % PX, 1 + q / PX);
        if (I.sm_npass > 0) {
          const gfloat* Js = (const gfloat*)I.Jsm[(I.sm_npass - 1) & 1];
          v[k][0] = Js[gi];
          v[k][1] = Js[nc + gi];
          v[k][2] = Js[2 * nc + gi];
        } else if (g.acc_mode == 2) {
          v[k][0] = (float)((double)(long long)I.J64[jp][gi] * jinv);
          v[k][1] = (float)((double)(long long)I.J64[jp][nc + gi] * jinv);
          v[k][2] = (float)((double)(long long)I.J64[jp][2 * nc + gi] * jinv);
        } else {
          const gfloat* Ja = (const gfloat*)I.Jacc[jp];
          v[k][0] = Ja[gi];
          v[k][1] = Ja[nc + gi];
          v[k][2] = Ja[2 * nc + gi];
        }
      }
    }
  };
  // Bh of plane z on the B region into buffer z & 1: E of z in buffer a, of
  // z+1 in c, B of z in v
  auto make_bh = [&](int z, int a, int c, const float (&v)[2][3]) {
    const int hb = z & 1;
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const int q = tid + k * kBlock;
      if (q >= BN) continue;
      const int x = q % BX, y = q / BX;
      const int ce = x + EX * y;
      const float d2E3 = (sE[a][2][ce + EX] - sE[a][2][ce]) * r1;
      const float d1E3 = (sE[a][2][ce + 1] - sE[a][2][ce]) * r0;
      const float d1E2 = (sE[a][1][ce + 1] - sE[a][1][ce]) * r0;
      const float d2E1 = (sE[a][0][ce + EX] - sE[a][0][ce]) * r1;
      const float d3E2 = (sE[c][1][ce] - sE[a][1][ce]) * r2;
      const float d3E1 = (sE[c][0][ce] - sE[a][0][ce]) * r2;
      float b1 = v[k][0], b2 = v[k][1], b3 = v[k][2];
      b1 -= h * (d2E3 - d3E2);
      b2 -= h * (d3E1 - d1E3);
      b3 -= h * (d1E2 - d2E1);
      sBh[hb][0][q] = b1;
      sBh[hb][1][q] = b2;
      sBh[hb][2][q] = b3;
    }
  };
  // E' of plane z on nodes 1..e+1 into buffer z & 1 (E of z in buffer a, J
  // of z in v); on the column's own cells of a plane of this run, Jout and
  // the clear of the other accumulator
  auto make_ep = [&](int z, int a, const float (&v)[2][3]) {
    const size_t zo = zoff(z);
    const int hb = z & 1, hm = (z - 1) & 1, eb = z & 1;
    const bool own = z >= z0 && z < z1;
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const int q = tid + k * kBlock;
      if (q >= PN) continue;
      const int x = 1 + q % PX, y = 1 + q / PX;
      const int ce = x + EX * y, cb = x + BX * y;
      const float J1 = v[k][0], J2 = v[k][1], J3 = v[k][2];
      const float d2B3 = (sBh[hb][2][cb] - sBh[hb][2][cb - BX]) * r1;
      const float d1B3 = (sBh[hb][2][cb] - sBh[hb][2][cb - 1]) * r0;
      const float d1B2 = (sBh[hb][1][cb] - sBh[hb][1][cb - 1]) * r0;
      const float d2B1 = (sBh[hb][0][cb] - sBh[hb][0][cb - BX]) * r1;
      const float d3B2 = (sBh[hb][1][cb] - sBh[hm][1][cb]) * r2;
      const float d3B1 = (sBh[hb][0][cb] - sBh[hm][0][cb]) * r2;
      float v1 = sE[a][0][ce], v2 = sE[a][1][ce], v3 = sE[a][2][ce];
      v1 += dt * ((d2B3 - d3B2) - J1);
      v2 += dt * ((d3B1 - d1B3) - J2);
      v3 += dt * ((d1B2 - d2B1) - J3);
      sEp[eb][0][ce] = v1;
      sEp[eb][1][ce] = v2;
      sEp[eb][2][ce] = v3;
      if (own && x <= e0 && y <= e1) {
        const size_t gi = zo + col(x, y);
        gfloat* Jo = (gfloat*)I.Jout;
        Jo[gi] = J1;
        Jo[nc + gi] = J2;
        Jo[2 * nc + gi] = J3;
        if (g.acc_mode == 2) {
          I.J64[jn][gi] = 0ull;
          I.J64[jn][nc + gi] = 0ull;
          I.J64[jn][2 * nc + gi] = 0ull;
        } else {
          gfloat* Jz = (gfloat*)I.Jacc[jn];
          Jz[gi] = 0.0f;
          Jz[nc + gi] = 0.0f;
          Jz[2 * nc + gi] = 0.0f;
        }
      }
    }
  };

  // prologue: Bh(z0-1), Bh(z0), E'(z0)
  float ev[2][3], bv[2][3], jv[2][3];
  {
    float ew[2][3], bw[2][3];
    get_e(z0 - 1, ev);
    get_e(z0, ew);
    get_b(z0 - 1, bv);
    get_b(z0, bw);
    get_j(z0, jv);
    put_e((z0 - 1) & 1, ev);
    put_e(z0 & 1, ew);
    get_e(z0 + 1, ev);
    __syncthreads();
    make_bh(z0 - 1, (z0 - 1) & 1, z0 & 1, bv);
    __syncthreads();
    put_e((z0 + 1) & 1, ev);  // over E(z0-1)
    __syncthreads();
    make_bh(z0, z0 & 1, (z0 + 1) & 1, bw);
    __syncthreads();
    make_ep(z0, z0 & 1, jv);
    __syncthreads();
  }
  float em = 0.0f;
  const int tx = tid % MarchTile::X, ty = tid / MarchTile::X;
  // the reads of a plane are issued one plane ahead, so they are in flight
  // while the previous plane is computed
  get_e(z0 + 2, ev);
  get_b(z0 + 1, bv);
  get_j(z0 + 1, jv);
  for (int z = z0; z < z1; z++) {
    // E(z+2) over E(z), which E'(z) no longer needs
    put_e(z & 1, ev);
    float bc[2][3], jc[2][3];
#pragma unroll
    for (int k = 0; k < 2; k++)
#pragma unroll
      for (int c = 0; c < 3; c++) {
        bc[k][c] = bv[k][c];
        jc[k][c] = jv[k][c];
      }
    if (z + 1 < z1) {
      get_e(z + 3, ev);
      get_b(z + 2, bv);
      get_j(z + 2, jv);
    }
    __syncthreads();
    make_bh(z + 1, (z + 1) & 1, z & 1, bc);
    __syncthreads();
    make_ep(z + 1, (z + 1) & 1, jc);
    __syncthreads();
    // B'(z) on the column's cells, and E'(z), B'(z) written out
    if (tx < e0 && ty < e1) {
      const int x = 1 + tx, y = 1 + ty;
      const int c = x + EX * y, cb = x + BX * y;
      const int a = z & 1, b = (z + 1) & 1;
      const float d2E3 = (sEp[a][2][c + EX] - sEp[a][2][c]) * r1;
      const float d1E3 = (sEp[a][2][c + 1] - sEp[a][2][c]) * r0;
      const float d1E2 = (sEp[a][1][c + 1] - sEp[a][1][c]) * r0;
      const float d2E1 = (sEp[a][0][c + EX] - sEp[a][0][c]) * r1;
      const float d3E2 = (sEp[b][1][c] - sEp[a][1][c]) * r2;
      const float d3E1 = (sEp[b][0][c] - sEp[a][0][c]) * r2;
      const size_t gi = zoff(z) + col(x, y);
      Fw[3 * nc + gi] = sBh[a][0][cb] - h * (d2E3 - d3E2);
      Fw[4 * nc + gi] = sBh[a][1][cb] - h * (d3E1 - d1E3);
      Fw[5 * nc + gi] = sBh[a][2][cb] - h * (d1E2 - d2E1);
      Fw[gi] = sEp[a][0][c];
      Fw[nc + gi] = sEp[a][1][c];
      Fw[2 * nc + gi] = sEp[a][2][c];
      em = fmaxf(em, fmaxf(fabsf(sEp[a][0][c]), fmaxf(fabsf(sEp[a][1][c]), fabsf(sEp[a][2][c]))));
    }
  }
  // the largest |E'_c| written raises the instance's running field bound
  const float emax0 = *(const gfloat*)I.emax;
  if (__ballot(em > emax0)) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) em = fmaxf(em, __shfl_xor(em, off));
    if ((tid & 63) == 0)
      __hip_atomic_fetch_max((guint*)I.emax, __float_as_uint(em), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The r-z field step (Sec. 3.3, Eqs. 2d-field-solve-cyl and
// 2d-field-solve-cyl-b1-axis) on the 2D tiles, in the three parts of
// yee_step.  E_z, E_theta, B_r (components 0, 2, 4) sit on whole rows at
// r = (j - 1/2) dr, E_r, B_z, B_theta (1, 3, 5) on half rows at r = j dr.
// Staged values below the axis are mirror images (z components keep the
// sign, r and theta components change it), at and beyond the wall zero;
// row 0 of the whole-row components is never read and is stored as zero;
// E_r and B_theta stay zero on the axis, and B_z there follows Faraday's
// law over the disc of radius dr/2, dB_z/dt = -4 E_theta(row 1) / dr.  The
// accumulators hold the folded ring currents: each row is divided by its
// ring volume (in units of 2 pi dr^2 dz) as it is read, and Jout keeps the
// current density.
__global__ void __launch_bounds__(kBlock) yee_step_rz(const InstDesc* __restrict__ inst, int par) {
  using T = YeeTile<2>;
  constexpr int EXM = T::X + 3, EYM = T::Y + 3;
  constexpr int BXM = T::X + 2, BYM = T::Y + 2;
  __shared__ float sE[3][EYM * EXM];
  __shared__ float sB[3][BYM * BXM];
  const InstDesc& I = inst[blockIdx.y];
  const GridDesc& g = I.g;
  if (!g.cyl) return;
  const int ntx = (g.nx[0] + T::X - 1) / T::X;
  const int nty = (g.nx[1] + T::Y - 1) / T::Y;
  const int tile = blockIdx.x;
  if (tile >= ntx * nty) return;
  const int tx = threadIdx.x % T::X;
  const int ty = threadIdx.x / T::X;
  const int nc = g.ncell;
  const int n0 = g.nx[0], n1 = g.nx[1];
  const int o0 = (tile % ntx) * T::X;
  const int o1 = (tile / ntx) * T::Y;
  const int e0 = min(T::X, n0 - o0);
  const int e1 = min(T::Y, n1 - o1);
  const int EX = e0 + 3, EY = e1 + 3;
  const int BX = e0 + 2, BY = e1 + 2;
  // moving window along z: the window column of region column x; the z
  // neighbours beyond the window's front and back are zero, and the back
  // column is discarded (becomes the empty front) after a shift
  const bool win = g.window != 0;
  int wo = 0;
  bool wshift = false;
  if (win) {
    const WinCtl wc = *I.win;
    wo = wc.origin;
    wshift = pic_win_shifts(g.wa, wc.step + 1) > pic_win_shifts(g.wa, wc.step);
  }
  auto wcol = [&](int x) {
    int r = wrap1(o0 - 1 + x, n0) - wo;
    return r < 0 ? r + n0 : r;
  };
  // region node (x, y) is column o0 - 1 + x (periodic) and row o1 - 1 + y
  const gfloat* F = (const gfloat*)I.F[par];
  for (int y = ty; y < EY; y += T::Y)
    for (int x = tx; x < EX; x += T::X) {
      const int gx = wrap1(o0 - 1 + x, n0);
      const int ry = o1 - 1 + y;
      const int rw = ry <= 0 ? 1 - ry : ry;
      const int rh = ry < 0 ? -ry : ry;
      const float sw = ry <= 0 ? -1.0f : 1.0f, sh = ry < 0 ? -1.0f : 1.0f;
      const bool iw = rw < n1, ih = rh < n1;
      const int gw = gx + n0 * rw, gh = gx + n0 * rh;
      const int r = x + EX * y;
      sE[0][r] = iw ? F[gw] : 0.0f;
      sE[1][r] = ih ? sh * F[nc + gh] : 0.0f;
      sE[2][r] = iw ? sw * F[2 * nc + gw] : 0.0f;
      if (x < BX && y < BY) {
        const int rb = x + BX * y;
        sB[0][rb] = ih ? F[3 * nc + gh] : 0.0f;
        sB[1][rb] = iw ? sw * F[4 * nc + gw] : 0.0f;
        sB[2][rb] = ih ? sh * F[5 * nc + gh] : 0.0f;
      }
    }
  __syncthreads();
  const float h = 0.5f * g.dt;
  const float rz = g.rdx[0], rr = g.rdx[1];
  // Bh on the B region (B_z, B_theta on half rows, B_r on whole rows); the
  // general r weights also give the mirror rows below the axis their images
  for (int y = ty; y < BY; y += T::Y)
    for (int x = tx; x < BX; x += T::X) {
      const int r = x + BX * y;
      const int c = x + EX * y;
      const int j = o1 - 1 + y;
      const bool front = win && wcol(x) == n0 - 1;
      sB[1][r] -= h * (-((front ? 0.0f : sE[2][c + 1]) - sE[2][c]) * rz);
      sB[2][r] -= h * (((front ? 0.0f : sE[1][c + 1]) - sE[1][c]) * rz - (sE[0][c + EX] - sE[0][c]) * rr);
      const float cz = j == 0 ? 4.0f * sE[2][c + EX] * rr
                              : ((j + 0.5f) * sE[2][c + EX] - (j - 0.5f) * sE[2][c]) * rr / (float)j;
      sB[0][r] -= h * cz;
    }
  __syncthreads();
  // E' on the tile plus one node above (zero at and beyond the wall)
  const int jp = par, jn = 1 - par;
  const double jinv = (double)g.jinv;
  for (int y = 1 + ty; y <= e1 + 1; y += T::Y)
    for (int x = 1 + tx; x <= e0 + 1; x += T::X) {
      const int ce = x + EX * y;
      const int cb = x + BX * y;
      const int j = o1 - 1 + y;
      if (j >= n1) {
        sE[0][ce] = 0.0f;
        sE[1][ce] = 0.0f;
        sE[2][ce] = 0.0f;
        continue;
      }
      const int gi = wrap1(o0 - 1 + x, n0) + n0 * j;
      float J1, J2, J3;
      // ring volumes of the row: whole rows (j - 1/2), half rows j
      const float vw = j >= 1 ? 1.0f / ((float)j - 0.5f) : 0.0f;
      const float vh = j >= 1 ? 1.0f / (float)j : 0.0f;
      if (I.sm_npass > 0) {  // the smoothed current is a density already
        const gfloat* Js = (const gfloat*)I.Jsm[(I.sm_npass - 1) & 1];
        const float on = j >= 1 ? 1.0f : 0.0f;
        J1 = on * Js[gi];
        J2 = on * Js[nc + gi];
        J3 = on * Js[2 * nc + gi];
      } else {
        if (g.acc_mode == 2) {
          J1 = (float)((double)(long long)I.J64[jp][gi] * jinv);
          J2 = (float)((double)(long long)I.J64[jp][nc + gi] * jinv);
          J3 = (float)((double)(long long)I.J64[jp][2 * nc + gi] * jinv);
        } else {
          const gfloat* Ja = (const gfloat*)I.Jacc[jp];
          J1 = Ja[gi];
          J2 = Ja[nc + gi];
          J3 = Ja[2 * nc + gi];
        }
        J1 *= vw;
        J2 *= vh;
        J3 *= vw;
      }
      const bool back = win && wcol(x) == 0;
      const float bt_m = back ? 0.0f : sB[2][cb - 1], br_m = back ? 0.0f : sB[1][cb - 1];
      sE[1][ce] = j == 0 ? 0.0f : sE[1][ce] + g.dt * (-(sB[2][cb] - bt_m) * rz - J2);
      sE[2][ce] += g.dt * ((sB[1][cb] - br_m) * rz - (sB[0][cb] - sB[0][cb - BX]) * rr - J3);
      sE[0][ce] += g.dt * (((float)j * sB[2][cb] - (float)(j - 1) * sB[2][cb - BX]) * rr * vw - J1);
      if (x <= e0 && y <= e1) {
        gfloat* Jo = (gfloat*)I.Jout;
        const float keep = (back && wshift) ? 0.0f : 1.0f;  // discarded column
        Jo[gi] = J1 * keep;
        Jo[nc + gi] = J2 * keep;
        Jo[2 * nc + gi] = J3 * keep;
        if (g.acc_mode == 2) {
          I.J64[jn][gi] = 0ull;
          I.J64[jn][nc + gi] = 0ull;
          I.J64[jn][2 * nc + gi] = 0ull;
        } else {
          gfloat* Jz = (gfloat*)I.Jacc[jn];
          Jz[gi] = 0.0f;
          Jz[nc + gi] = 0.0f;
          Jz[2 * nc + gi] = 0.0f;
        }
      }
    }
  __syncthreads();
  // B' on the tile, and write E', B' back
  gfloat* Fw = (gfloat*)I.F[1 - par];
  for (int y = 1 + ty; y <= e1; y += T::Y)
    for (int x = 1 + tx; x <= e0; x += T::X) {
      const int c = x + EX * y;
      const int cb = x + BX * y;
      const int j = o1 - 1 + y;
      const int gi = wrap1(o0 - 1 + x, n0) + n0 * j;
      const float cz = j == 0 ? 4.0f * sE[2][c + EX] * rr
                              : ((j + 0.5f) * sE[2][c + EX] - (j - 0.5f) * sE[2][c]) * rr / (float)j;
      const int wx = win ? wcol(x) : 1;
      const bool front = win && wx == n0 - 1;
      const float br = sB[1][cb] - h * (-((front ? 0.0f : sE[2][c + 1]) - sE[2][c]) * rz);
      const float bt = sB[2][cb] - h * (((front ? 0.0f : sE[1][c + 1]) - sE[1][c]) * rz - (sE[0][c + EX] - sE[0][c]) * rr);
      const bool in = j >= 1;
      // the window's back column becomes its empty front after a shift
      const float keep = (win && wshift && wx == 0) ? 0.0f : 1.0f;
      Fw[gi] = in ? sE[0][c] * keep : 0.0f;
      Fw[nc + gi] = sE[1][c] * keep;
      Fw[2 * nc + gi] = in ? sE[2][c] * keep : 0.0f;
      Fw[3 * nc + gi] = (sB[0][cb] - h * cz) * keep;
      Fw[4 * nc + gi] = in ? br * keep : 0.0f;
      Fw[5 * nc + gi] = in ? bt * keep : 0.0f;
    }
}

// One smoothing pass of the current along 'axis' (pass 'lev' of that axis)
// for every instance that has it: J <- a J[i-1] + b J[i] + c J[i+1] with the
// normalised weights, periodic.  The instance's first pass reads the
// accumulator of the step's parity; later passes read the other buffer.
// One smoothing pass of an r-z instance.  The filtered quantity is the
// current density (the deposit divided by the ring volume of its row: radius
// (j - 1/2) dr for the whole rows of J_z, J_theta, j dr for the half rows of
// J_r).  Neighbours below the axis are the mirror images (J_z even, J_r and
// J_theta odd), those at and beyond the wall zero.  Row 0 keeps the axis
// value of J_r (zero) and the image of row 1 for J_z, J_theta, so the row-0
// entries of the passes are never read as sources.
__device__ __forceinline__ void smooth_pass_rz(const InstDesc& I, int axis, float a, float b, float c,
                                               gfloat* dst, const gfloat* src, bool first, bool fixed,
                                               double jinv, int par) {
  const GridDesc& g = I.g;
  const int nc = g.ncell;
  const int n0 = g.nx[0], n1 = g.nx[1];
  // the density of component comp at (row, column): mirror and wall rules,
  // raw deposit divided by the ring volume on the first pass
  auto load = [&](int comp, int row, int col) -> float {
    const bool half = comp == 1;
    float sg = 1.0f;
    if (half ? row < 0 : row <= 0) {
      row = half ? -row : 1 - row;
      if (comp != 0) sg = -1.0f;
    }
    if (row >= n1) return 0.0f;
    const int q = comp * nc + col + n0 * row;
    if (!first) return sg * src[q];
    const float rv = half ? (float)row : (float)row - 0.5f;
    if (rv <= 0.0f) return 0.0f;  // J_r on the axis
    float v;
    if (fixed)
      v = (float)((double)(long long)I.J64[par][q] * jinv);
    else
      v = ((const gfloat*)I.Jacc[par])[q];
    return sg * v / rv;
  };
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 3 * nc; e += gridDim.x * blockDim.x) {
    const int comp = e / nc;
    const int q = e - comp * nc;
    const int i = q % n0;
    int j = q / n0;
    float out;
    if (axis == 0) {
      // along z: periodic, or zero beyond the ends of a moving window
      float am = a, cp = c;
      if (g.window) {
        int wr = i - I.win->origin;
        if (wr < 0) wr += n0;
        if (wr == 0) am = 0.0f;
        if (wr == n0 - 1) cp = 0.0f;
      }
      const int im = i == 0 ? n0 - 1 : i - 1;
      const int ip = i == n0 - 1 ? 0 : i + 1;
      out = am * load(comp, j, im) + b * load(comp, j, i) + cp * load(comp, j, ip);
    } else {
      float sg = 1.0f;
      if (j == 0) {  // axis row: J_r zero, J_z and J_theta the image of row 1
        if (comp == 1) {
          dst[e] = 0.0f;
          continue;
        }
        j = 1;
        sg = comp == 0 ? 1.0f : -1.0f;
      }
      out = sg * (a * load(comp, j - 1, i) + b * load(comp, j, i) + c * load(comp, j + 1, i));
    }
    dst[e] = out;
  }
}

__global__ void __launch_bounds__(kBlock) smooth_pass(const InstDesc* __restrict__ inst, int axis, int lev,
                                                      int par) {
  const InstDesc& I = inst[blockIdx.y];
  if (lev >= I.sm_level[axis]) return;
  const GridDesc& g = I.g;
  const int k = I.sm_first[axis] + lev;
  const int nc = g.ncell;
  const int n = g.nx[axis];
  const int stride = axis == 0 ? 1 : (axis == 1 ? g.nx[0] : g.nx[0] * g.nx[1]);
  const float a = I.sm_w[axis][lev][0], b = I.sm_w[axis][lev][1], c = I.sm_w[axis][lev][2];
  gfloat* dst = (gfloat*)I.Jsm[k & 1];
  const gfloat* src = (const gfloat*)I.Jsm[(k - 1) & 1];
  const bool first = k == 0;
  const bool fixed = g.acc_mode == 2;
  const double jinv = (double)g.jinv;
  if (g.cyl) {
    smooth_pass_rz(I, axis, a, b, c, dst, src, first, fixed, jinv, par);
    return;
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 3 * nc; e += gridDim.x * blockDim.x) {
    const int comp = e / nc;
    const int q = e - comp * nc;
    const int i = (q / stride) % n;
    const int qm = i == 0 ? q + (n - 1) * stride : q - stride;
    const int qp = i == n - 1 ? q - (n - 1) * stride : q + stride;
    // moving window: beyond the x1 ends the current is zero
    float am = a, cp = c;
    if (g.window && axis == 0) {
      int wr = i - I.win->origin;
      if (wr < 0) wr += n;
      if (wr == 0) am = 0.0f;
      if (wr == n - 1) cp = 0.0f;
    }
    const int o = comp * nc;
    float vm, v0, vp;
    if (!first) {
      vm = src[o + qm];
      v0 = src[o + q];
      vp = src[o + qp];
    } else if (fixed) {
      vm = (float)((double)(long long)I.J64[par][o + qm] * jinv);
      v0 = (float)((double)(long long)I.J64[par][o + q] * jinv);
      vp = (float)((double)(long long)I.J64[par][o + qp] * jinv);
    } else {
      const gfloat* Ja = (const gfloat*)I.Jacc[par];
      vm = Ja[o + qm];
      v0 = Ja[o + q];
      vp = Ja[o + qp];
    }
    dst[e] = am * vm + b * v0 + cp * vp;
  }
}

// End of a step of a moving window: count the step and, when c t has passed
// the next whole cell, move the window (advance the ring origin, count the
// injected particles' ids).  One thread per instance.
__global__ void window_advance(const InstDesc* __restrict__ inst, int ninst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ninst) return;
  const InstDesc& I = inst[k];
  if (!I.g.window) return;
  WinCtl w = *I.win;
  const bool sh = pic_win_shifts(I.g.wa, w.step + 1) > pic_win_shifts(I.g.wa, w.step);
  w.step += 1;
  if (sh) {
    w.shifts += 1;
    w.origin = w.origin + 1 == I.g.nx[0] ? 0 : w.origin + 1;
    w.next_id += I.win_inject;
  }
  *I.win = w;
}

}  // namespace

hipError_t pic_launch_window_advance(const InstDesc* d_inst, int ninst, hipStream_t st) {
  hipLaunchKernelGGL(window_advance, dim3((ninst + 63) / 64), dim3(64), 0, st, d_inst, ninst);
  return hipGetLastError();
}

hipError_t pic_launch_smooth_pass(const InstDesc* d_inst, int ninst, int max_ncell, int axis, int lev,
                                  int parity, hipStream_t st) {
  long b = ((long)3 * max_ncell + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(smooth_pass, dim3((int)b, ninst), dim3(kBlock), 0, st, d_inst, axis, lev, parity);
  return hipGetLastError();
}

int pic_yee_tiles(int dim, const int nx[3]) {
  if (dim == 2)
    return ((nx[0] + YeeTile<2>::X - 1) / YeeTile<2>::X) * ((nx[1] + YeeTile<2>::Y - 1) / YeeTile<2>::Y);
  // the larger of the tile counts of yee_step (moving windows) and yee_march3
  const int t = ((nx[0] + YeeTile<3>::X - 1) / YeeTile<3>::X) * ((nx[1] + YeeTile<3>::Y - 1) / YeeTile<3>::Y) *
                ((nx[2] + YeeTile<3>::Z - 1) / YeeTile<3>::Z);
  const int m = ((nx[0] + MarchTile::X - 1) / MarchTile::X) * ((nx[1] + MarchTile::Y - 1) / MarchTile::Y) *
                ((nx[2] + kMarchZ - 1) / kMarchZ);
  return t > m ? t : m;
}

hipError_t pic_launch_current_units(StoreDesc* d_stores, int nstores, hipStream_t st) {
  hipLaunchKernelGGL(current_units, dim3((nstores + 63) / 64), dim3(64), 0, st, d_stores, nstores);
  return hipGetLastError();
}

hipError_t pic_launch_yee_step(const InstDesc* d_inst, int ninst, int max_tiles, int dim, bool cart, bool cyl,
                               bool window, int parity, hipStream_t st) {
  const dim3 grid(max_tiles, ninst);
  if (dim == 2) {
    if (cart && window) hipLaunchKernelGGL((yee_step<2, true>), grid, dim3(kBlock), 0, st, d_inst, parity);
    if (cart && !window) hipLaunchKernelGGL((yee_step<2, false>), grid, dim3(kBlock), 0, st, d_inst, parity);
    if (cyl) hipLaunchKernelGGL(yee_step_rz, grid, dim3(kBlock), 0, st, d_inst, parity);
  } else if (window) {
    hipLaunchKernelGGL((yee_step<3, true>), grid, dim3(kBlock), 0, st, d_inst, parity);
  } else {
    hipLaunchKernelGGL(yee_march3, grid, dim3(kBlock), 0, st, d_inst, parity);
  }
  return hipGetLastError();
}
