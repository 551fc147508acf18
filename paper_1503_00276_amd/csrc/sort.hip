// sort.hip -- periodic tile rebin of the particle storage (counting sort by
// tile).  Not part of the dissertation's CPU code, which keeps particles in
// plain arrays; here it keeps every tile's particles contiguous so the fused
// kernel can stage the tile's fields in LDS.
//
// Between rebins a particle strays at most 'slack' cells outside its tile,
// so at a rebin every particle moves to its own tile or to one of the 3^d - 1
// neighbours.  The rebin is a stable counting sort over those 27 neighbour
// slots: the particles of destination tile d are, in order, those of source
// tile d - delta_s with slot s, for s = 0..26, each in its old order.  The
// per-item slot counts come from the fused particle kernel of the last step.
//
// A check is five launches over every store of a launch group:
//   count   (per source tile)       slot prefix over the tile's items, slot totals
//   dest    (per destination tile)  slot bases, particles, items; block sums
//   fold    (per store)             scan of the block sums; control words
//   offsets (per destination tile)  tile offsets, item offsets, item list
//   scatter (per source item)       stable scatter into the other buffer set
// Only stores whose fused kernel raised the flag (or whose check the host
// forces, in autotuner trials) do any work; for the others every launch
// returns at once.
#include "pic_dev.h"
#include "pic_kernels.h"

namespace {

constexpr int kBlock = 256;
constexpr int kScanBlock = 1024;
constexpr int kMaxGroup = 256;
constexpr int kTB = PIC_REBIN_TILES;

static_assert(kTB == kBlock, "one destination tile per thread of the planner");

// Store of a flat index over the stores of a group, given per-store starts
// (pref[0..n-1], increasing) in LDS.
// Whether the host forces this check to rebin (autotuner trials: every
// force-th check).  nchecks only changes at the end of a check (in the fold),
// so every kernel of one check takes the same decision.
__device__ __forceinline__ bool forced_check(const StoreCtl* c) {
  const int k = c->force;
  return k > 0 && c->nchecks % k == 0;
}

__device__ __forceinline__ int store_of(const int* pref, int n, int x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pref[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Moving window: whether the window moves after the current step.
__device__ __forceinline__ bool win_shift_now(const StoreDesc& S) {
  if (!S.g.window) return false;
  const long long n = S.win->step;
  return pic_win_shifts(S.g.wa, n + 1) > pic_win_shifts(S.g.wa, n);
}

// Particles a moving window injects into destination tile d at this check
// (the tile's cells in the new front column, which is the ring column of the
// old origin, times the particles per cell).
__device__ __forceinline__ int win_inject_count(const StoreDesc& S, int d) {
  if (!S.g.window || !win_shift_now(S)) return 0;
  const GridDesc& g = S.g;
  int tc[3];
  pic_tile_coords(g, d, tc);
  const int o = S.win->origin;
  const int org0 = tc[0] * g.tile[0];
  if (o < org0 || o >= org0 + min(g.tile[0], g.nx[0] - org0)) return 0;
  int cells = 1;
  for (int k = 1; k < g.dim; k++) cells *= min(g.tile[k], g.nx[k] - tc[k] * g.tile[k]);
  int n = cells * S.inj_ppc[0] * S.inj_ppc[1] * S.inj_ppc[2];
  // r-z: the lattice points of the axis row below the axis are not injected
  if (g.cyl && tc[1] == 0) n -= S.inj_ppc[0] * (S.inj_ppc[1] / 2);
  return n;
}

// Slot of a particle with packed cell 'cell' that is stored in tile t
// (-1 for a particle a moving window removed).
__device__ __forceinline__ int particle_slot(const GridDesc& g, int t, int cell) {
  if (cell < 0) return -1;
  int tc[3], c[3];
  pic_tile_coords(g, t, tc);
  pic_unpack(g, cell, c);
  int dd[3] = {0, 0, 0};
  for (int d = 0; d < g.dim; d++) {
    int o = tc[d] * g.tile[d];
    int e = min(g.tile[d], g.nx[d] - o);
    int l = pic_local(c[d], o, e, g.nx[d]);
    dd[d] = l < 0 ? -1 : (l >= e ? 1 : 0);
  }
  return pic_slot(dd[0], dd[1], dd[2]);
}

// Exclusive scan of two ints over a 256-thread block; returns the totals.
__device__ __forceinline__ void block_scan2(int a, int b, int& ea, int& eb, int& ta, int& tb) {
  __shared__ int wa[kBlock / 64], wb[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int ia = a, ib = b;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int va = __shfl_up(ia, off);
    int vb = __shfl_up(ib, off);
    if (lane >= off) {
      ia += va;
      ib += vb;
    }
  }
  if (lane == 63) {
    wa[wave] = ia;
    wb[wave] = ib;
  }
  __syncthreads();
  int ca = 0, cb = 0;
  ta = 0;
  tb = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; w++) {
    if (w < wave) {
      ca += wa[w];
      cb += wb[w];
    }
    ta += wa[w];
    tb += wb[w];
  }
  ea = ca + ia - a;
  eb = cb + ib - b;
  __syncthreads();
}

// --- 1. per source tile and slot: running counts over the tile's items ------
// One thread per (tile, slot): consecutive threads read and write
// consecutive words of the slot-major count rows.
__global__ void __launch_bounds__(kBlock) rebin_count(const StoreDesc* __restrict__ stores, int nstores,
                                                      int total_tiles) {
  __shared__ int t0[kMaxGroup];
  for (int i = threadIdx.x; i < nstores; i += blockDim.x) t0[i] = stores[i].tile0;
  __syncthreads();
  const int total = total_tiles * PIC_NSLOT;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const int gt = q / PIC_NSLOT, sl = q - gt * PIC_NSLOT;
    const StoreDesc& S = stores[store_of(t0, nstores, gt)];
    if (!(S.ctl->flag || forced_check(S.ctl)) && !win_shift_now(S)) continue;
    const int cur = pic_cur(*S.ctl);
    const int t = gt - S.tile0;
    const int i0 = S.ioff[cur][t], i1 = S.ioff[cur][t + 1];
    int run = 0;
    for (int i = i0; i < i1; i++) {
      const int c = S.cnt[i * PIC_NSLOT + sl];
      S.pre[i * PIC_NSLOT + sl] = run;
      run += c;
    }
    S.tot[t * PIC_NSLOT + sl] = run;
  }
}

// --- 2. per destination tile: incoming particles in slot order; block sums ---
__global__ void __launch_bounds__(kBlock) rebin_dest(const StoreDesc* __restrict__ stores, int nstores) {
  __shared__ int b0[kMaxGroup];
  for (int i = threadIdx.x; i < nstores; i += blockDim.x) b0[i] = stores[i].blk0;
  __syncthreads();
  const StoreDesc& S = stores[store_of(b0, nstores, blockIdx.x)];
  if (!(S.ctl->flag || forced_check(S.ctl)) && !win_shift_now(S)) return;
  const int blk = blockIdx.x - S.blk0;
  const int d = blk * kTB + threadIdx.x;
  int acc = 0, ni = 0;
  if (d < S.g.ntiles) {
    int src[PIC_NSLOT], v[PIC_NSLOT];
#pragma unroll
    for (int sl = 0; sl < PIC_NSLOT; sl++) src[sl] = S.nsrc[d * PIC_NSLOT + sl];
#pragma unroll
    for (int sl = 0; sl < PIC_NSLOT; sl++) v[sl] = S.tot[src[sl] * PIC_NSLOT + sl];
#pragma unroll
    for (int sl = 0; sl < PIC_NSLOT; sl++) {
      S.dbase[d * PIC_NSLOT + sl] = acc;
      acc += v[sl];
    }
    acc += win_inject_count(S, d);  // injected particles follow the incoming ones
    S.dcount[d] = acc;
    ni = (acc + S.chunk - 1) / S.chunk;
  }
  int ea, eb, ta, tb;
  block_scan2(acc, ni, ea, eb, ta, tb);
  if (threadIdx.x == 0) {
    S.bsum[2 * blk] = ta;
    S.bsum[2 * blk + 1] = tb;
  }
}

// --- 3. per store: scan of the block sums, totals, control words ---------------
__global__ void __launch_bounds__(kScanBlock) rebin_fold(const StoreDesc* __restrict__ stores) {
  const StoreDesc& S = stores[blockIdx.x];
  __shared__ int sa[kScanBlock], sb[kScanBlock];
  __shared__ int s_cur, s_act;
  if (threadIdx.x == 0) {
    const StoreCtl c = *S.ctl;
    s_cur = c.cur ^ c.pending;
    s_act = (c.flag || forced_check(&c) || win_shift_now(S)) ? 1 : 0;
  }
  __syncthreads();
  const int cur = s_cur;
  const int act = s_act;
  if (act) {
    const int nblk = (S.g.ntiles + kTB - 1) / kTB;
    int carry_a = 0, carry_b = 0;
    for (int base = 0; base < nblk; base += kScanBlock) {
      const int k = base + threadIdx.x;
      const int a = k < nblk ? S.bsum[2 * k] : 0;
      const int b = k < nblk ? S.bsum[2 * k + 1] : 0;
      sa[threadIdx.x] = a;
      sb[threadIdx.x] = b;
      __syncthreads();
      for (int off = 1; off < kScanBlock; off <<= 1) {
        int va = threadIdx.x >= off ? sa[threadIdx.x - off] : 0;
        int vb = threadIdx.x >= off ? sb[threadIdx.x - off] : 0;
        __syncthreads();
        sa[threadIdx.x] += va;
        sb[threadIdx.x] += vb;
        __syncthreads();
      }
      if (k < nblk) {
        S.bpre[2 * k] = carry_a + sa[threadIdx.x] - a;
        S.bpre[2 * k + 1] = carry_b + sb[threadIdx.x] - b;
      }
      carry_a += sa[kScanBlock - 1];
      carry_b += sb[kScanBlock - 1];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const int nxt = 1 - cur;
      S.toff[nxt][S.g.ntiles] = carry_a;
      S.ioff[nxt][S.g.ntiles] = carry_b;
      S.ctl->n_items[nxt] = min(carry_b, S.max_items);
      S.ctl->np = carry_a;
      // in a periodic box the count is fixed; a moving window (removal,
      // injection) or the r-z wall (removal) change it within the capacity
      if (carry_b > S.max_items || ((S.g.window || S.g.cyl) ? carry_a > S.cap : carry_a != S.np)) S.ctl->bad |= 4;
    }
  }
  if (threadIdx.x == 0) {
    // this workgroup is the only writer of the control words during a check
    StoreCtl* c = S.ctl;
    c->cur = cur;
    c->pending = act ? 1 : 0;  // the scatter of this check fills set 1 - cur
    c->active = act;
    c->flag = 0;
    c->nchecks += 1;
    c->nsorts += act;
    // after this check every particle sits in its own tile (re-sorted), or
    // within flag_slack cells of it (no particle strayed further)
    c->sorted = act;
  }
}

// --- 4. per destination tile: tile offsets, item offsets, item list -----------
__global__ void __launch_bounds__(kBlock) rebin_offsets(const StoreDesc* __restrict__ stores, int nstores) {
  __shared__ int b0[kMaxGroup];
  for (int i = threadIdx.x; i < nstores; i += blockDim.x) b0[i] = stores[i].blk0;
  __syncthreads();
  const StoreDesc& S = stores[store_of(b0, nstores, blockIdx.x)];
  if (!S.ctl->active) return;
  const int nxt = 1 - S.ctl->cur;
  const int blk = blockIdx.x - S.blk0;
  const int t = blk * kTB + threadIdx.x;
  const int chunk = S.chunk;
  const int c = t < S.g.ntiles ? S.dcount[t] : 0;
  const int ni = (c + chunk - 1) / chunk;
  int ea, eb, ta, tb;
  block_scan2(c, ni, ea, eb, ta, tb);
  if (t < S.g.ntiles) {
    const int ra = S.bpre[2 * blk] + ea;
    const int rb = S.bpre[2 * blk + 1] + eb;
    S.toff[nxt][t] = ra;
    S.ioff[nxt][t] = rb;
    Item* items = S.items[nxt];
    for (int k = 0; k < ni && rb + k < S.max_items; k++) {
      Item it;
      it.tile = t;
      it.begin = ra + k * chunk;
      it.end = min(ra + (k + 1) * chunk, ra + c);
      it.pad = 0;
      items[rb + k] = it;
    }
  }
}

// Block-shared prefix over stores of a per-store count (0 for idle stores).
template <typename F>
__device__ void group_prefix(const StoreDesc* stores, int nstores, int* pref, F count) {
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int s = 0; s < nstores; s++) {
      pref[s] = acc;
      acc += stores[s].ctl->active ? count(stores[s]) : 0;
    }
    pref[nstores] = acc;
  }
  __syncthreads();
}

// --- 5. per old item: stable scatter into the other buffer set ---------------
__global__ void __launch_bounds__(kBlock) rebin_scatter(const StoreDesc* __restrict__ stores, int nstores) {
  __shared__ int pref[kMaxGroup + 1];
  __shared__ int run[PIC_NSLOT];
  __shared__ int wcnt[kBlock / 64][PIC_NSLOT];
  // the source set is cur (the fold set pending for the destination)
  group_prefix(stores, nstores, pref, [](const StoreDesc& S) { return S.ctl->n_items[S.ctl->cur]; });
  const int total = pref[nstores];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int s = 0;
  for (int gi = blockIdx.x; gi < total; gi += gridDim.x) {
    while (gi >= pref[s + 1]) s++;
    const StoreDesc& S = stores[s];
    const GridDesc& g = S.g;
    const int cur = S.ctl->cur, nxt = 1 - cur;
    const int ii = gi - pref[s];
    const Item it = S.items[cur][ii];
    if (threadIdx.x < PIC_NSLOT) {
      int sl = threadIdx.x;
      int d = S.ndst[it.tile * PIC_NSLOT + sl];
      run[sl] = S.toff[nxt][d] + S.dbase[d * PIC_NSLOT + sl] + S.pre[ii * PIC_NSLOT + sl];
    }
    for (int base = it.begin; base < it.end; base += blockDim.x) {
      __syncthreads();
      if (threadIdx.x < (kBlock / 64) * PIC_NSLOT) (&wcnt[0][0])[threadIdx.x] = 0;
      __syncthreads();
      int p = base + threadIdx.x;
      // every load of the particle is issued here, before the rank
      // computation, so the round waits for one memory latency, not two
      const bool have = p < it.end;
      int cell = 0, pid = 0;
      float ev[3] = {0.0f, 0.0f, 0.0f}, uv[3] = {0.0f, 0.0f, 0.0f}, wv = 0.0f;
      if (have) {
        cell = S.cell[cur][p];
        for (int d = 0; d < g.dim; d++) ev[d] = S.eps[cur][d][p];
        uv[0] = S.u[cur][0][p];
        uv[1] = S.u[cur][1][p];
        uv[2] = S.u[cur][2][p];
        wv = S.w[cur][p];
        pid = S.id[cur][p];
      }
      int sl = have ? particle_slot(g, it.tile, cell) : -1;
      int rank = 0;
      unsigned long long todo = __ballot(sl >= 0);
      while (todo) {
        int leader = __ffsll((long long)todo) - 1;
        int ls = __shfl(sl, leader);
        unsigned long long m = __ballot(sl == ls);
        if (sl == ls) rank = (int)__popcll(m & lt);
        if (lane == leader) wcnt[wave][ls] = (int)__popcll(m);
        todo &= ~m;
      }
      __syncthreads();
      int pos = -1;
      if (sl >= 0) {
        pos = run[sl] + rank;
        for (int w = 0; w < wave; w++) pos += wcnt[w][sl];
        if (pos < 0 || pos >= S.cap) {  // inconsistent counts: never write out of bounds
          atomicOr(&S.ctl->bad, 2);
          pos = -1;
        }
      }
      if (pos >= 0) {
        S.cell[nxt][pos] = cell;
        for (int d = 0; d < g.dim; d++) S.eps[nxt][d][pos] = ev[d];
        S.u[nxt][0][pos] = uv[0];
        S.u[nxt][1][pos] = uv[1];
        S.u[nxt][2][pos] = uv[2];
        S.w[nxt][pos] = wv;
        S.id[nxt][pos] = pid;
      }
      __syncthreads();
      if (threadIdx.x < PIC_NSLOT) {
        int add = 0;
        for (int w = 0; w < kBlock / 64; w++) add += wcnt[w][threadIdx.x];
        run[threadIdx.x] += add;
      }
    }
    __syncthreads();
  }
}

// --- 6. moving window: a cold plasma in the new front column ------------------
// Particle k of the column (cells in increasing linear index, lattice points
// of a cell with axis 1 fastest) goes to its tile's range after the incoming
// particles, at its rank among the tile's injected particles; ids continue
// from the window's counter.
// Output n >= 1 of the SplitMix64 generator seeded with s (Steele, Lea and
// Flood, "Fast splittable pseudorandom number generators", 2014): the state
// advances by the golden-ratio increment, the output mixes it.
__device__ unsigned long long splitmix64_output(unsigned long long s, unsigned long long n) {
  unsigned long long z = s + n * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Standard normal deviate of component c of the particle with id 'id':
// Box-Muller (1958) on U1 in (0, 1] and U2 in [0, 1), 53 bits each.
__device__ double thermal_normal(unsigned long long seed, long long id, int c) {
  const unsigned long long n = 8ull * (unsigned long long)id + 2ull * (unsigned long long)c;
  const double u1 = (double)((splitmix64_output(seed, n + 1) >> 11) + 1) * 0x1.0p-53;
  const double u2 = (double)(splitmix64_output(seed, n + 2) >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__global__ void __launch_bounds__(kBlock) rebin_inject(const StoreDesc* __restrict__ stores, int nstores) {
  const StoreDesc& S = stores[blockIdx.y];
  if (!S.g.window || !S.ctl->active || !win_shift_now(S)) return;
  const GridDesc& g = S.g;
  const int nxt = 1 - S.ctl->cur;
  const int p0 = S.inj_ppc[0], p1 = S.inj_ppc[1], p2 = g.dim == 3 ? S.inj_ppc[2] : 1;
  const int ppc = p0 * p1 * p2;
  const int ny = g.nx[1], nz = g.dim == 3 ? g.nx[2] : 1;
  const int total = ppc * ny * nz;
  const int o = S.win->origin;
  const long long id0 = S.win->next_id;
  // r-z: lattice points below the axis (axis-row offsets under 1/2) are
  // skipped; the others of the tile holding the axis row move up in rank
  const int nex = g.cyl ? p1 / 2 : 0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
    const int cidx = k / ppc, li = k - cidx * ppc;
    const int cy = cidx % ny, cz = cidx / ny;
    const int l0 = li % p0, l1 = (li / p0) % p1, l2 = li / (p0 * p1);
    if (cy == 0 && l1 < nex) continue;
    const int ty = cy / g.tile[1], tz = g.dim == 3 ? cz / g.tile[2] : 0;
    const int t = pic_tile_index(g, o / g.tile[0], ty, tz);
    const int oy = ty * g.tile[1], oz = tz * g.tile[2];
    const int ey = min(g.tile[1], ny - oy);
    const int rank = ((cy - oy) + ey * (cz - oz)) * ppc + li - (oy == 0 ? p0 * nex : 0);
    const int pos = S.toff[nxt][t] + S.dcount[t] - win_inject_count(S, t) + rank;
    if (pos < 0 || pos >= S.cap) {
      atomicOr(&S.ctl->bad, 2);
      continue;
    }
    S.cell[nxt][pos] = pic_pack(g, o, cy, cz);
    S.eps[nxt][0][pos] = ((float)l0 + 0.5f) / (float)p0;
    S.eps[nxt][1][pos] = ((float)l1 + 0.5f) / (float)p1;
    if (g.dim == 3) S.eps[nxt][2][pos] = ((float)l2 + 0.5f) / (float)p2;
    // at rest, or thermal: a Box-Muller normal deviate per component from
    // the SplitMix64 outputs 8 id + 2c + 1 and 8 id + 2c + 2 (FP64)
    const long long id = id0 + k;
#pragma unroll
    for (int c = 0; c < 3; c++)
      S.u[nxt][c][pos] = S.inj_uth > 0.0 ? (float)(S.inj_uth * thermal_normal(S.inj_seed, id, c)) : 0.0f;
    // r-z: a uniform density takes a weight proportional to the radius
    S.w[nxt][pos] = g.cyl ? S.inj_w * ((float)cy + ((float)l1 + 0.5f) / (float)p1 - 0.5f) : S.inj_w;
    S.id[nxt][pos] = (int)(id0 + k);
  }
}

int cap_grid(long n, int per) {
  long b = (n + per - 1) / per;
  if (b > 8192) b = 8192;
  return b < 1 ? 1 : (int)b;
}

}  // namespace

hipError_t pic_launch_rebin(const StoreDesc* d_stores, int nstores, int max_items, int total_tiles,
                            int total_blocks, int inject_max, hipStream_t st) {
  if (nstores > kMaxGroup || nstores < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rebin_count, dim3(cap_grid((long)total_tiles * PIC_NSLOT, kBlock)), dim3(kBlock), 0, st,
                     d_stores, nstores, total_tiles);
  hipLaunchKernelGGL(rebin_dest, dim3(total_blocks), dim3(kBlock), 0, st, d_stores, nstores);
  hipLaunchKernelGGL(rebin_fold, dim3(nstores), dim3(kScanBlock), 0, st, d_stores);
  hipLaunchKernelGGL(rebin_offsets, dim3(total_blocks), dim3(kBlock), 0, st, d_stores, nstores);
  hipLaunchKernelGGL(rebin_scatter, dim3(cap_grid(max_items, 1)), dim3(kBlock), 0, st, d_stores, nstores);
  if (inject_max > 0)
    hipLaunchKernelGGL(rebin_inject, dim3(cap_grid(inject_max, kBlock), nstores), dim3(kBlock), 0, st, d_stores,
                       nstores);
  return hipGetLastError();
}
