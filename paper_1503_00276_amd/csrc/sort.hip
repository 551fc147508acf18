// sort.hip -- periodic tile rebin of the particle storage (counting sort by
// tile).  Not part of the dissertation's CPU code, which keeps particles in
// plain arrays; here it keeps every tile's particles contiguous so the fused
// kernel can stage the tile's fields in LDS.
//
// Between rebins a particle strays at most 'slack' cells outside its tile,
// so at a rebin every particle moves to its own tile or to one of the 3^d - 1
// neighbours.  The rebin is a stable counting sort over those 27 neighbour
// slots: the particles of destination tile d are, in order, those of source
// tile d - delta_s with slot s, for s = 0..26, each in its old order.
//
// The rebin runs only when the fused kernel raised the store's flag (some
// particle strayed beyond flag_slack); every kernel returns at once otherwise,
// so the check costs a few empty launches.  The sorted particles go to the
// other buffer set and the final kernel flips the current set.
#include "pic_dev.h"
#include "pic_kernels.h"

namespace {

constexpr int kBlock = 256;
constexpr int kScanBlock = 1024;
constexpr int kMaxGroup = 256;

// The scatter of this check runs for stores whose planner found the flag set.
__device__ __forceinline__ bool active(const StoreDesc& S) { return S.ctl->active != 0; }

// Slot of a particle with packed cell 'cell' that is stored in tile t.
__device__ __forceinline__ int particle_slot(const GridDesc& g, int t, int cell) {
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

// Block-shared prefix over stores of a per-store count (0 for idle stores).
template <typename F>
__device__ void group_prefix(const StoreDesc* stores, int nstores, int* pref, F count) {
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int s = 0; s < nstores; s++) {
      pref[s] = acc;
      acc += active(stores[s]) ? count(stores[s]) : 0;
    }
    pref[nstores] = acc;
  }
  __syncthreads();
}

// --- 1. per store, one workgroup: slot totals per tile, slot bases per
// destination tile, tile offsets, item offsets and the new item list.  The
// per-item slot counts come from the fused particle kernel of the last step.
__global__ void __launch_bounds__(kScanBlock) rebin_plan(const StoreDesc* __restrict__ stores) {
  const StoreDesc& S = stores[blockIdx.x];
  __shared__ int sa[kScanBlock], sb[kScanBlock];
  __shared__ int s_cur, s_act;
  if (threadIdx.x == 0) {
    // fold the flip of the previous rebin and turn the flag into this
    // check's decision; this workgroup is the only writer of these words
    StoreCtl* c = S.ctl;
    const int cur = c->cur ^ c->pending;
    const int act = c->flag;
    c->cur = cur;
    c->pending = 0;
    c->active = act;
    c->flag = 0;
    c->nchecks += 1;
    c->nsorts += act;
    s_cur = cur;
    s_act = act;
  }
  __syncthreads();
  if (!s_act) return;
  const int nt = S.g.ntiles;
  const int cur = s_cur;
  const int nxt = 1 - cur;
  // running slot counts over the items of each source tile (27 independent
  // loads per item, issued together)
  for (int t = threadIdx.x; t < nt; t += blockDim.x) {
    const int i0 = S.ioff[cur][t], i1 = S.ioff[cur][t + 1];
    int run[PIC_NSLOT];
#pragma unroll
    for (int sl = 0; sl < PIC_NSLOT; sl++) run[sl] = 0;
    for (int i = i0; i < i1; i++) {
      int c[PIC_NSLOT];
#pragma unroll
      for (int sl = 0; sl < PIC_NSLOT; sl++) c[sl] = S.cnt[i * PIC_NSLOT + sl];
#pragma unroll
      for (int sl = 0; sl < PIC_NSLOT; sl++) {
        S.pre[i * PIC_NSLOT + sl] = run[sl];
        run[sl] += c[sl];
      }
    }
#pragma unroll
    for (int sl = 0; sl < PIC_NSLOT; sl++) S.tot[t * PIC_NSLOT + sl] = run[sl];
  }
  __syncthreads();
  // incoming particles of each destination tile, in slot order
  for (int d = threadIdx.x; d < nt; d += blockDim.x) {
    int src[PIC_NSLOT], v[PIC_NSLOT];
#pragma unroll
    for (int sl = 0; sl < PIC_NSLOT; sl++) src[sl] = S.nsrc[d * PIC_NSLOT + sl];
#pragma unroll
    for (int sl = 0; sl < PIC_NSLOT; sl++) v[sl] = S.tot[src[sl] * PIC_NSLOT + sl];
    int acc = 0;
#pragma unroll
    for (int sl = 0; sl < PIC_NSLOT; sl++) {
      S.dbase[d * PIC_NSLOT + sl] = acc;
      acc += v[sl];
    }
    S.dcount[d] = acc;
  }
  __syncthreads();
  const int chunk = S.chunk;
  const int seg = (nt + kScanBlock - 1) / kScanBlock;
  const int t0 = threadIdx.x * seg;
  const int t1 = min(nt, t0 + seg);
  int a = 0, b = 0;
  for (int t = t0; t < t1; t++) {
    int c = S.dcount[t];
    a += c;
    b += (c + chunk - 1) / chunk;
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  // inclusive scan (Hillis-Steele) over the block
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int va = threadIdx.x >= off ? sa[threadIdx.x - off] : 0;
    int vb = threadIdx.x >= off ? sb[threadIdx.x - off] : 0;
    __syncthreads();
    sa[threadIdx.x] += va;
    sb[threadIdx.x] += vb;
    __syncthreads();
  }
  int ra = sa[threadIdx.x] - a, rb = sb[threadIdx.x] - b;  // exclusive
  int* toff = S.toff[nxt];
  int* ioff = S.ioff[nxt];
  Item* items = S.items[nxt];
  for (int t = t0; t < t1; t++) {
    int c = S.dcount[t];
    int ni = (c + chunk - 1) / chunk;
    toff[t] = ra;
    ioff[t] = rb;
    for (int k = 0; k < ni; k++) {
      if (rb + k >= S.max_items) {
        atomicOr(&S.ctl->bad, 4);
        break;
      }
      Item it;
      it.tile = t;
      it.begin = ra + k * chunk;
      it.end = min(ra + (k + 1) * chunk, ra + c);
      it.pad = 0;
      items[rb + k] = it;
    }
    ra += c;
    rb += ni;
  }
  if (threadIdx.x == kScanBlock - 1) {
    toff[nt] = sa[kScanBlock - 1];
    ioff[nt] = sb[kScanBlock - 1];
    S.ctl->n_items[nxt] = min(sb[kScanBlock - 1], S.max_items);
    S.ctl->pending = 1;  // the scatter of this check fills set nxt
  }
}

// --- 2. per old item: stable scatter into the other buffer set -----------------
__global__ void __launch_bounds__(kBlock) rebin_scatter(const StoreDesc* __restrict__ stores, int nstores) {
  __shared__ int pref[kMaxGroup + 1];
  __shared__ int run[PIC_NSLOT];
  __shared__ int wcnt[kBlock / 64][PIC_NSLOT];
  // the source set is cur (the planner set pending for the destination)
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
      int sl = p < it.end ? particle_slot(g, it.tile, S.cell[cur][p]) : -1;
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
        if (pos < 0 || pos >= S.np) {  // inconsistent counts: never write out of bounds
          atomicOr(&S.ctl->bad, 2);
          pos = -1;
        }
      }
      if (pos >= 0) {
        S.cell[nxt][pos] = S.cell[cur][p];
        for (int d = 0; d < g.dim; d++) S.eps[nxt][d][pos] = S.eps[cur][d][p];
        S.u[nxt][0][pos] = S.u[cur][0][p];
        S.u[nxt][1][pos] = S.u[cur][1][p];
        S.u[nxt][2][pos] = S.u[cur][2][p];
        S.w[nxt][pos] = S.w[cur][p];
        S.id[nxt][pos] = S.id[cur][p];
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

int cap_grid(long n, int per) {
  long b = (n + per - 1) / per;
  if (b > 8192) b = 8192;
  return b < 1 ? 1 : (int)b;
}

}  // namespace

hipError_t pic_launch_rebin(const StoreDesc* d_stores, int nstores, int max_items, int max_tiles,
                            hipStream_t st) {
  (void)max_tiles;
  if (nstores > kMaxGroup) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rebin_plan, dim3(nstores), dim3(kScanBlock), 0, st, d_stores);
  hipLaunchKernelGGL(rebin_scatter, dim3(cap_grid(max_items, 1)), dim3(kBlock), 0, st, d_stores, nstores);
  return hipGetLastError();
}
