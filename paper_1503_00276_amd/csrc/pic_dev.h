// pic_dev.h -- device-side data layout shared by the HIP kernels and the host
// runtime of libpic.so.  Plain structs, copied to device memory once and read
// by the kernels through a pointer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PIC_MAX_SPECIES 8
#define PIC_NSLOT 27  // neighbour slots (-1,0,+1)^3 for the rebin
#define PIC_REBIN_TILES 256  // destination tiles per workgroup of the rebin planner

// One periodic box: grid, time step, shape order and tiling.
struct GridDesc {
  int dim;            // 2 or 3
  int order;          // 1, 2, 3
  int nx[3];          // cells per axis (1 on unused axes)
  int tile[3];        // tile extent (cells)
  int ntile[3];       // tiles per axis
  int ntiles;         // product of ntile
  int sh1, sh2;       // bit shifts of the packed cell index (c0 | c1<<sh1 | c2<<sh2)
  int m0, m1;         // masks of c0 and c1
  int slack;          // cells a particle may stray outside its tile at a step start (max of slk)
  int slk[3];         // per axis: the stray bound of the last step of a sort cycle
  float vstep[3];     // per axis: cells a particle can move in one step (c dt / dx, rounded up)
  int flag_slack;     // stray distance (cells) beyond which a rebin is requested
  int ncell;          // product of nx
  float dx[3];        // cell size
  float rdx[3];       // 1 / dx
  float cdt[3];       // dx / dt (current per unit charge density per cell moved)
  float dt;
  float e0[3], b0[3]; // uniform external fields
  double dxd[3];      // cell size in FP64 (diagnostics)
  double dtd;         // time step in FP64 (diagnostics)
  // current accumulation: contributions are rounded to integers in units of
  // jinv = 1/jscale (a power of two) and summed exactly in int64
  float jscale, jinv;
  int acc_mode;       // 0/1: FP32 fold of the tile sums, 2: int64 fold (deterministic)
  int deposit;        // 0: ISIS ordering average, 1: TRISTAN path cut at faces (linear shape)
  int window;         // 1: moving window along x1 (x1 open; grid stored as a ring, see WinCtl)
  double wa;          // moving window: c dt / dx1 (shifts after n steps: floor(n wa))
  int cyl;            // 1: 2D r-z geometry (x1 = z, x2 = r; axis mid first cell, wall at the top)
  // LDS region geometry (nodes relative to the tile origin):
  // field region [-(slack+fa), e+slack+fb), current region [-(slack+ja), e+slack+jb)
  int fa, fb, ja, jb;
  // two-phase 3D kernel: LDS strides (nodes) of a field-region row and plane
  // and of a current-region row and plane, padded so that the lanes of a
  // wavefront, one particle per cell of the tile, spread over the LDS banks
  int fs0, fs01, js0, js01;
  // 1: the two-phase periodic 2D kernel runs this grid (set by the host)
  int tp2;
};

// Control words of one particle store.  The buffer set holding the particles
// is cur ^ pending: the rebin's fold kernel (one workgroup per store, so no
// atomics are needed) folds pending into cur when it next runs, and sets
// pending when it plans a rebin whose scatter fills the other set.
struct StoreCtl {
  int cur;          // buffer set, before the pending flip
  int pending;      // 1: the other set is current (a scatter filled it)
  int flag;         // a particle strayed beyond flag_slack: rebin at the next check
  int active;       // the planned rebin of this check (read by the scatter)
  int n_items[2];   // work items of each buffer set
  int bad;          // a particle was found outside its staged region (skipped)
  int nsorts;       // rebins performed
  int nchecks;      // rebin checks performed
  int force;        // set by the host for autotuner trials: k > 0 rebins at
                    // every k-th check (nchecks % k == 0), flagged or not
  int np;           // particles in the current set after the last rebin (moving window)
  int sorted;       // 1: every particle sits in its own tile (loaded, or re-sorted at the last check)
  float umax;       // bound on |u| of the store's particles at the start of the step: set at
                    // a load (with the largest thermal momentum a moving window can inject),
                    // raised at every step by the largest kick it can give (see gpd_body)
};

__host__ __device__ inline int pic_cur(const StoreCtl& c) { return c.cur ^ c.pending; }

// Moving-window state of one instance.  The grid and the particles' cell
// indices are kept in ring coordinates along x1: ring column r holds window
// column (r - origin) mod nx1, so a shift only advances the origin, zeroes
// the old back column (the new front) and refills it.  Kernels read the
// state at launch; the step's last kernel advances it.
struct WinCtl {
  long long step;     // steps done
  int shifts;         // cell shifts done
  int origin;         // ring column of window column 0
  long long next_id;  // id of the next injected particle
  int pad[2];
};

// The periodic 3D ISIS variant of the fused kernel runs each work item in two
// phases whose field and current tiles share one LDS region (fused-kernel
// MODE 4); every other box takes the one-phase kernel.
__host__ __device__ inline bool pic_gpd_split(const GridDesc& g) {
  return g.dim == 3 && !g.window && !g.cyl && g.deposit == 0;
}

// Shifts after n steps of a window moving at c.
__host__ __device__ inline int pic_win_shifts(double wa, long long n) { return (int)floor((double)n * wa); }

// Work item: a contiguous run of particles that all belong to one tile.
struct Item {
  int tile, begin, end, pad;
};

// One particle species of one instance: SoA particles in two ping-pong sets.
struct StoreDesc {
  GridDesc g;
  float qm;                  // charge-to-mass ratio q/m = 1/rqm
  float wmax;                // max |w| over the store's particles (rounded up)
  int np;                    // particles stored
  int chunk;                 // maximum particles per work item
  int max_items;
  float* F[2];               // instance fields E1 E2 E3 B1 B2 B3 (planes of ncell floats), double-
                             // buffered: step n reads set n&1, the Yee step writes the other
  float* Jacc[2];            // FP32 current accumulators (J1 J2 J3 planes), double-buffered
  unsigned long long* J64[2];// int64 fixed-point accumulators (deterministic mode only)
  int* cell[2];              // packed cell index
  float* eps[2][3];          // in-cell offset in [0,1)
  float* u[2][3];            // u = gamma v
  float* w[2];               // charge weight
  int* id[2];                // load order
  int* toff[2];              // tile offsets [ntiles+1]
  int* ioff[2];              // first item of each tile [ntiles+1]
  Item* items[2];
  int* cnt;                  // [max_items][27] slot counts of the current items
  int* pre;                  // [max_items][27] prefix of cnt over earlier items of the tile
  int* tot;                  // [ntiles][27]
  int* dbase;                // [ntiles][27] slot base inside the destination tile
  int* dcount;               // [ntiles]
  int* bsum;                 // [nblk][2] particles and items of each block of kRebinTiles tiles
  int* bpre;                 // [nblk][2] their exclusive prefix
  int tile0, blk0;           // first tile and tile block of this store within its launch group
  int cap;                   // particles the buffer sets hold
  WinCtl* win;               // moving window state of the instance (null without a window)
  int inj_ppc[3];            // moving window: injected particles per cell per axis
  float inj_w;               // moving window: weight of an injected particle
  double inj_uth;            // moving window: thermal spread of the injected momenta (0: at rest)
  unsigned long long inj_seed;  // moving window: seed of their generator
  const int* nsrc;           // [ntiles][27] tile - delta_s (periodic), per instance
  const int* ndst;           // [ntiles][27] tile + delta_s (periodic), per instance
  StoreCtl* ctl;
  const float* emax;         // the instance's running bound on |E_c| (see InstDesc)
};

// One instance (for the field kernels).
struct InstDesc {
  GridDesc g;
  float* F[2];
  float* Jacc[2];
  unsigned long long* J64[2];
  float* Jout;               // the current of the last step (FP32, used by the E update)
  // current smoothing: passes per axis, normalised 3-point weights, the
  // instance's pass number of each axis' first pass, and two FP32 buffers
  // the passes alternate between (the last one feeds the E update)
  int sm_level[3];
  int sm_first[3];
  int sm_npass;
  float sm_w[3][8][3];
  float* Jsm[2];
  WinCtl* win;               // moving window state (null without a window)
  int win_inject;            // moving window: particles injected per shift
  float* emax;               // running bound on |E_c| over the grid (Cartesian): set at a field
                             // load, raised by the Yee step, never lowered
};

// ---------------------------------------------------------------------------
// small helpers used by several kernels
// ---------------------------------------------------------------------------

__host__ __device__ inline int pic_wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Position of cell coordinate c relative to a tile starting at o with extent
// e on a periodic axis of n cells.  Cells inside the tile map to [0, e);
// outside, the nearer side wins (ties go above), giving a value in (-n, n).
__host__ __device__ inline int pic_local(int c, int o, int e, int n) {
  int r = c - o;
  if (r < 0) r += n;
  if (r < e) return r;
  int dh = r - e + 1;
  int dl = n - r;
  return (dh <= dl) ? r : r - n;
}

__host__ __device__ inline void pic_unpack(const GridDesc& g, int cell, int c[3]) {
  c[0] = cell & g.m0;
  c[1] = (cell >> g.sh1) & g.m1;
  c[2] = cell >> g.sh2;
}

__host__ __device__ inline int pic_pack(const GridDesc& g, int c0, int c1, int c2) {
  return c0 | (c1 << g.sh1) | (c2 << g.sh2);
}

__host__ __device__ inline void pic_tile_coords(const GridDesc& g, int t, int tc[3]) {
  tc[0] = t % g.ntile[0];
  int r = t / g.ntile[0];
  tc[1] = r % g.ntile[1];
  tc[2] = r / g.ntile[1];
}

__host__ __device__ inline int pic_tile_index(const GridDesc& g, int t0, int t1, int t2) {
  return t0 + g.ntile[0] * (t1 + g.ntile[1] * t2);
}

// Slot (0..26) of a displacement d in {-1,0,1}^3.
__host__ __device__ inline int pic_slot(int d0, int d1, int d2) {
  return (d0 + 1) + 3 * (d1 + 1) + 9 * (d2 + 1);
}
