// gpd.hip -- the fused particle kernel: field gather, relativistic Boris push,
// position advance and charge-conserving current deposit, one tile of particles
// per work item (Hemker 2000, Ch. 3, Sec. 3.1 loop; Sec. 3.2 equations).
//
// Per work item (a run of particles that belong to one tile):
//  1. stage E and B of the tile plus guard nodes from HBM into LDS
//     (periodic wrap applied here, so the global planes carry no guards);
//  2. clear an LDS current tile (tile plus deposit guards);
//  3. for each particle: shape weights at the six staggered offsets, gather,
//     Boris push, advance, re-cell, and the ISIS current in Esirkepov's closed
//     form added to the LDS tile with LDS atomics;
//  4. add the LDS current tile into the global current with atomics
//     (overlapping guards of neighbouring tiles fold in here).
//
// Positions are stored as a packed integer cell plus an FP32 offset in [0,1)
// per axis; all arithmetic is FP32.
#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

#include "pic_dev.h"
#include "pic_kernels.h"

namespace {

// Global-address-space views: pointers read from the descriptor are generic;
// casting them lets the compiler emit global (not flat) memory instructions.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) int gint;

constexpr int kBlock = 256;
constexpr int kMaxGroup = 256;

// ---------------------------------------------------------------------------
// shape weights
// ---------------------------------------------------------------------------

// Weights of a B-spline of order ORDER for the staggered component whose
// nodes sit at offset 0 (half=false) or 1/2 (half=true) from the cell's node
// along one axis; eps is the particle's in-cell offset.  base is the first
// node, relative to the particle's cell.
template <int ORDER>
__device__ __forceinline__ void gather_weights(float eps, bool half, int& base, float w[ORDER + 1]) {
  if constexpr (ORDER == 1) {
    float f;
    if (!half) {
      base = 0;
      f = eps;
    } else {
      bool hi = eps >= 0.5f;
      base = hi ? 0 : -1;
      f = hi ? eps - 0.5f : eps + 0.5f;
    }
    w[0] = 1.0f - f;
    w[1] = f;
  } else if constexpr (ORDER == 2) {
    float t;
    if (!half) {
      int n = eps >= 0.5f ? 1 : 0;
      t = eps - (float)n;
      base = n - 1;
    } else {
      t = eps - 0.5f;
      base = -1;
    }
    float a = 0.5f - t, b = 0.5f + t;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - t * t;
    w[2] = 0.5f * b * b;
  } else {
    float f;
    if (!half) {
      base = -1;
      f = eps;
    } else {
      bool hi = eps >= 0.5f;
      base = hi ? -1 : -2;
      f = hi ? eps - 0.5f : eps + 0.5f;
    }
    float g = 1.0f - f, f2 = f * f, f3 = f2 * f;
    const float s6 = 1.0f / 6.0f;
    w[0] = g * g * g * s6;
    w[1] = (4.0f - 6.0f * f2 + 3.0f * f3) * s6;
    w[2] = (1.0f + 3.0f * f + 3.0f * f2 - 3.0f * f3) * s6;
    w[3] = f3 * s6;
  }
}

// Old shape S0 on a window of ORDER+2 nodes starting at node 'base' (relative
// to the particle's old cell) and the change D = S1 - S0 on that window, for
// a move from offset e0 in the old cell to offset e1 in the cell c (-1,0,1)
// cells away.  D is formed from factored differences (proportional to the
// displacement, or, for a move across a knot of the shape, to the distances
// on either side of the knot), keeping full FP32 relative accuracy for short
// moves.
// p0 (0 or 1) is the window position of the old shape's first node and wide
// is true when the new shape's support is shifted by one node (the union
// then fills all ORDER+2 window positions; otherwise D vanishes outside the
// ORDER+1 positions p0 .. p0+ORDER).
template <int ORDER>
__device__ __forceinline__ void deposit_shape(float e0, float e1, int c, int& base, int& p0, bool& wide,
                                              float S0[ORDER + 2], float D[ORDER + 2]) {
  constexpr int W = ORDER + 2;
#pragma unroll
  for (int k = 0; k < W; k++) {
    S0[k] = 0.0f;
    D[k] = 0.0f;
  }
  if constexpr (ORDER == 1) {
    // old nodes 0,1; new nodes c, c+1
    base = c < 0 ? -1 : 0;
    p0 = -base;  // window position of old node 0
    wide = c != 0;
    float a0 = 1.0f - e0;
    if (p0 == 0) {
      S0[0] = a0;
      S0[1] = e0;
    } else {
      S0[1] = a0;
      S0[2] = e0;
    }
    if (c == 0) {
      float d = e1 - e0;
      D[0] = -d;
      D[1] = d;
    } else if (c > 0) {
      D[0] = -a0;
      D[1] = a0 - e1;
      D[2] = e1;
    } else {
      float a1 = 1.0f - e1;
      D[0] = a1;
      D[1] = e0 - a1;
      D[2] = -e0;
    }
  } else if constexpr (ORDER == 2) {
    int h0 = e0 >= 0.5f ? 1 : 0;
    int h1 = e1 >= 0.5f ? 1 : 0;
    int n0 = h0, n1 = c + h1;           // nearest nodes, relative to the old cell
    float t0 = e0 - (float)h0, t1 = e1 - (float)h1;
    int nlo = n0 < n1 ? n0 : n1;
    base = nlo - 1;
    p0 = n0 - 1 - base;  // 0 or 1
    wide = n1 != n0;
    float a = 0.5f - t0, b = 0.5f + t0;
    float w0 = 0.5f * a * a, w1 = 0.75f - t0 * t0, w2 = 0.5f * b * b;
    if (p0 == 0) {
      S0[0] = w0; S0[1] = w1; S0[2] = w2;
    } else {
      S0[1] = w0; S0[2] = w1; S0[3] = w2;
    }
    if (n1 == n0) {
      float d = t1 - t0, s = t0 + t1;
      float v0 = 0.5f * d * (s - 1.0f), v1 = -d * s, v2 = 0.5f * d * (1.0f + s);
      if (p0 == 0) {
        D[0] = v0; D[1] = v1; D[2] = v2;
      } else {
        D[1] = v0; D[2] = v1; D[3] = v2;
      }
    } else if (n1 > n0) {
      // the move crosses the half-node x_k = n0 + 1/2, a knot of every node's
      // spline in the window: each difference is taken on the two pieces on
      // either side of x_k, factored by the distances a = x_k - x0 and
      // b = x1 - x_k (exact near the crossing), so a short move keeps its
      // relative precision
      const float a = 0.5f - t0, b = t1 + 0.5f;
      D[0] = -0.5f * a * a;
      D[1] = -a * (0.5f + t0) - 0.5f * b * (2.0f - b);
      D[2] = 0.5f * a * (1.5f + t0) + b * (1.0f - b);
      D[3] = 0.5f * b * b;
    } else {
      // mirror image: crossing x_k = n0 - 1/2 to the left
      const float a = t0 + 0.5f, b = 0.5f - t1;
      D[0] = 0.5f * b * b;
      D[1] = 0.5f * a * (1.5f - t0) + b * (1.0f - b);
      D[2] = -a * (0.5f - t0) - 0.5f * b * (2.0f - b);
      D[3] = -0.5f * a * a;
    }
  } else {
    // old nodes -1..2 (floor = 0), new nodes c-1..c+2
    base = (c < 0 ? c : 0) - 1;
    p0 = -1 - base;  // 0 or 1
    wide = c != 0;
    const float s6 = 1.0f / 6.0f;
    float g0 = 1.0f - e0, f2 = e0 * e0, f3 = f2 * e0;
    float w0 = g0 * g0 * g0 * s6, w1 = (4.0f - 6.0f * f2 + 3.0f * f3) * s6;
    float w2 = (1.0f + 3.0f * e0 + 3.0f * f2 - 3.0f * f3) * s6, w3 = f3 * s6;
    if (p0 == 0) {
      S0[0] = w0; S0[1] = w1; S0[2] = w2; S0[3] = w3;
    } else {
      S0[1] = w0; S0[2] = w1; S0[3] = w2; S0[4] = w3;
    }
    if (c == 0) {
      float d = e1 - e0;
      float s = e1 + e0, q = e1 * e1 + e1 * e0 + e0 * e0;
      float g1 = 1.0f - e1;
      float a = g1 * g1 + g1 * g0 + g0 * g0;
      D[0] = -(d * s6) * a;
      D[1] = d * (0.5f * q - s);
      D[2] = (0.5f * d) * (1.0f + s - q);
      D[3] = (d * s6) * q;
    } else if (c > 0) {
      // the move crosses the cell face x_k = 1, a knot of every node's spline
      // in the window: each difference is taken on the pieces on either side
      // of it, factored by a = 1 - e0 and b = e1 (exact near the crossing)
      const float a = 1.0f - e0, b = e1;
      D[0] = -(a * a * a) * s6;
      D[1] = -0.5f * a * (1.0f + a - a * a) - b * (3.0f - 3.0f * b + b * b) * s6;
      D[2] = 0.5f * a * a * (2.0f - a) - 0.5f * b * b * (2.0f - b);
      D[3] = a * (3.0f - 3.0f * a + a * a) * s6 + 0.5f * b * (1.0f + b - b * b);
      D[4] = b * b * b * s6;
    } else {
      // mirror image: crossing the face x_k = 0 to the left, a = e0, b = 1 - e1
      const float a = e0, b = 1.0f - e1;
      D[0] = b * b * b * s6;
      D[1] = a * (3.0f - 3.0f * a + a * a) * s6 + 0.5f * b * (1.0f + b - b * b);
      D[2] = 0.5f * a * a * (2.0f - a) - 0.5f * b * b * (2.0f - b);
      D[3] = -0.5f * a * (1.0f + a - a * a) - b * (3.0f - 3.0f * b + b * b) * s6;
      D[4] = -(a * a * a) * s6;
    }
  }
}

// LDS current accumulator.  FP32 atomic adds to LDS are slow on gfx950
// (about 0.3 lane-ops per cycle per CU against 5-10 for integer adds), so each
// FP32 contribution v, bounded by |w| max(dx/dt, 1), is rounded to an integer
// in units of 1/scale (|v*scale| < 2^30) and summed exactly in int64.
typedef unsigned long long acc_t;

// floor(x + 1/2) as an int32 in one instruction (round half up)
__device__ __forceinline__ int cvt_rpi(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// v is already in units of the fixed point (the instance's, or the work
// item's in the two-phase 3D kernel; the scale is folded into the
// per-particle prefactors); it is rounded to the nearest unit.
__device__ __forceinline__ void lds_add(acc_t* p, float v) {
  const int q = cvt_rpi(v);
  if (q != 0)
    __hip_atomic_fetch_add(p, (acc_t)(long long)q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Unconditional add (for nodes whose contribution is rarely zero).
__device__ __forceinline__ void lds_add_any(acc_t* p, float v) {
  __hip_atomic_fetch_add(p, (acc_t)(long long)cvt_rpi(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The same on a 32-bit tile (two's complement sums in an unsigned word).
__device__ __forceinline__ void lds_add_any(unsigned* p, float v) {
  __hip_atomic_fetch_add(p, (unsigned)cvt_rpi(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Fixed point of one work item's int64 current tile: Q = 2^e with Q b < 2^29
// for a bound b on any single contribution (a factor 2 to spare for the FP32
// rounding of the shape differences), so that every contribution converts
// to an int32; e = 0 when nothing can be deposited.
__device__ __forceinline__ int item_exponent(float b) {
  int ex = 0;
  (void)frexpf(b, &ex);
  return b > 0.0f ? min(100, max(-100, 29 - ex)) : 0;
}

// The same for a 32-bit tile summing at most n contributions per node:
// Q = 2^e with Q n b (1 + 2^-16) < 2^31.  FP32 rounding lets a contribution
// exceed its bound b by a few tens of ulps (under 2^-19 relative), and the
// rounding to the unit adds at most 1/2, so a node's sum of n of them stays
// below 2^31 - 2^14 in magnitude.
__device__ __forceinline__ int item_exponent32(float b, int n) {
  int ex = 0;
  (void)frexpf((float)n * b * 1.0000153f, &ex);  // n b (1 + 2^-16) < 2^ex
  return b > 0.0f ? min(100, max(-100, 31 - ex)) : 0;
}

// An int64 node sum times its unit, as FP32.  The low word is taken signed
// (q = hi 2^32 + lo, lo in [-2^31, 2^31)), so a sum below 2^31 in magnitude
// converts with a single FP32 rounding (an unsigned low word of a small
// negative sum would sit near 2^32 and cancel against hi = -1).
__device__ __forceinline__ float item_sum_f32(long long q, float unit) {
  const int lo = (int)(unsigned)(q & 0xffffffffll);
  const long long hi = (q - (long long)lo) >> 32;
  return fmaf((float)hi, 4294967296.0f, (float)lo) * unit;
}

// TRISTAN (Villasenor-Buneman) current of one particle for the linear shape
// (Sec. 3.2): the straight move from offset e in the old cell by dl cells
// (|dl| < 1 per axis) is cut where it crosses cell faces; each piece lies in
// one cell and adds that cell's in-cell current, the average over the
// orderings of its orthogonal moves:
//   2D  J1 on the two x edges: a1 dx (1 - ym | ym), J2 likewise, and J3 at
//       the four nodes the piece's share of w v3 times the time average of
//       the product of the two linear shapes;
//   3D  J1 on the four x edges: a1 dx (Wy Wz + s dy dz / 12), s = +1 on the
//       (0,0), (1,1) edges and -1 on the others; J2, J3 likewise.
// b0..b2 are the LDS current-region coordinates of the old cell; a_d are
// w (dx_d/dt) in fixed-point units, v3s = w v3 in fixed-point units (2D).
template <int DIM>
// With a moving window (wcol >= 0, the particle's window column) the adds to
// x1 nodes beyond the window's ends are dropped.
__device__ __forceinline__ void deposit_tristan(acc_t* sJ, int jn, const int JR[3], int b0, int b1, int b2,
                                                const float e[3], const float dl[3], const int mv[3], float a1,
                                                float a2, float a3, float v3s, int wcol, int nx0) {
  // crossing parameter of each axis (2 when the axis stays in its cell)
  float tc[3] = {2.0f, 2.0f, 2.0f};
#pragma unroll
  for (int d = 0; d < DIM; d++)
    if (mv[d] != 0) {
      float t = (mv[d] > 0 ? 1.0f - e[d] : -e[d]) / dl[d];
      tc[d] = fminf(fmaxf(t, 0.0f), 1.0f);
    }
  // the cut parameters in increasing order
  float c0 = tc[0], c1 = tc[1], c2 = tc[2];
  if (c1 < c0) { float x = c0; c0 = c1; c1 = x; }
  if (DIM == 3) {
    if (c2 < c1) { float x = c1; c1 = c2; c2 = x; }
    if (c1 < c0) { float x = c0; c0 = c1; c1 = x; }
  }
  const float cut[4] = {c0, c1, c2, 2.0f};
  acc_t* J1 = sJ;
  acc_t* J2 = sJ + jn;
  acc_t* J3 = sJ + 2 * jn;
  const int R0 = JR[0], R01 = JR[0] * JR[1];
  float ta = 0.0f;
#pragma unroll
  for (int s = 0; s <= DIM; s++) {
    const float tb = fminf(cut[s], 1.0f);
    if (tb > ta) {
      float pa[3], pb[3];
      int o[3] = {0, 0, 0};
#pragma unroll
      for (int d = 0; d < DIM; d++) {
        o[d] = (mv[d] != 0 && tc[d] <= ta) ? mv[d] : 0;  // faces crossed before this piece
        pa[d] = fminf(fmaxf(e[d] + ta * dl[d] - (float)o[d], 0.0f), 1.0f);
        pb[d] = fminf(fmaxf(e[d] + tb * dl[d] - (float)o[d], 0.0f), 1.0f);
      }
      const float dx = pb[0] - pa[0], dy = pb[1] - pa[1];
      const float xm = 0.5f * (pa[0] + pb[0]), ym = 0.5f * (pa[1] + pb[1]);
      // x1 nodes of the piece's cell: inside the window or not
      const float in0 = (wcol < 0 || (unsigned)(wcol + o[0]) < (unsigned)nx0) ? 1.0f : 0.0f;
      const float in1 = (wcol < 0 || (unsigned)(wcol + o[0] + 1) < (unsigned)nx0) ? 1.0f : 0.0f;
      if constexpr (DIM == 2) {
        const int c = (b1 + o[1]) * R0 + b0 + o[0];
        const float f1 = a1 * dx * in0, f2 = a2 * dy;
        lds_add(J1 + c, f1 * (1.0f - ym));
        lds_add(J1 + c + R0, f1 * ym);
        lds_add(J2 + c, f2 * (1.0f - xm) * in0);
        lds_add(J2 + c + 1, f2 * xm * in1);
        const float f3 = v3s * (tb - ta);
        const float sxa[2] = {(1.0f - pa[0]) * in0, pa[0] * in1}, sxb[2] = {(1.0f - pb[0]) * in0, pb[0] * in1};
        const float sya[2] = {1.0f - pa[1], pa[1]}, syb[2] = {1.0f - pb[1], pb[1]};
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
          for (int i = 0; i < 2; i++)
            lds_add(J3 + c + j * R0 + i,
                    f3 * ((sxa[i] * sya[j] + sxb[i] * syb[j]) * (1.0f / 3.0f) +
                          (sxa[i] * syb[j] + sxb[i] * sya[j]) * (1.0f / 6.0f)));
      } else {
        const float dz = pb[2] - pa[2], zm = 0.5f * (pa[2] + pb[2]);
        const int c = ((b2 + o[2]) * JR[1] + b1 + o[1]) * R0 + b0 + o[0];
        const float Wx[2] = {1.0f - xm, xm}, Wy[2] = {1.0f - ym, ym}, Wz[2] = {1.0f - zm, zm};
        const float s[2] = {-1.0f, 1.0f};
        const float inx[2] = {in0, in1};
        const float yz = dy * dz * (1.0f / 12.0f), xz = dx * dz * (1.0f / 12.0f), xy = dx * dy * (1.0f / 12.0f);
        const float f1 = a1 * dx * in0, f2 = a2 * dy, f3 = a3 * dz;
#pragma unroll
        for (int k = 0; k < 2; k++)
#pragma unroll
          for (int j = 0; j < 2; j++) {
            lds_add(J1 + c + k * R01 + j * R0, f1 * (Wy[j] * Wz[k] + s[j] * s[k] * yz));
            lds_add(J2 + c + k * R01 + j, f2 * inx[j] * (Wx[j] * Wz[k] + s[j] * s[k] * xz));
            lds_add(J3 + c + k * R0 + j, f3 * inx[j] * (Wx[j] * Wy[k] + s[j] * s[k] * xy));
          }
      }
    }
    ta = fmaxf(ta, tb);
  }
}

// Coordinates of a flat index over a box of extents R[3] that advances by a
// fixed step: kept up to date by additions, so the staging and flush loops
// divide only once per workgroup.
// n / d for 0 <= n < 2^20 and d >= 1 through the FP32 reciprocal: the
// quotient (n + 1/2) / d sits at least 1/(2d) from an integer, farther than
// the reciprocal's error of a few 2^-24 relative reaches below 2^20.
__device__ __forceinline__ int small_div(int n, int d) {
  return (int)(((float)n + 0.5f) * __builtin_amdgcn_rcpf((float)d));
}

struct BoxWalk {
  int x, y, z, sx, sy, sz;
  __device__ BoxWalk(int start, int step, const int R[3]) {
    int r = small_div(start, R[0]);
    x = start - r * R[0];
    z = small_div(r, R[1]);
    y = r - z * R[1];
    r = small_div(step, R[0]);
    sx = step - r * R[0];
    sz = small_div(r, R[1]);
    sy = r - sz * R[1];
  }
  __device__ void advance(const int R[3]) {
    x += sx;
    const int cy = x >= R[0] ? 1 : 0;
    x -= cy ? R[0] : 0;
    y += sy + cy;
    const int cz = y >= R[1] ? 1 : 0;
    y -= cz ? R[1] : 0;
    z += sz + cz;
  }
};

// Periodic wrap, cheap when the index is already inside.
__device__ __forceinline__ int wrap_fast(int v, int n) { return (unsigned)v < (unsigned)n ? v : pic_wrap(v, n); }

// ---------------------------------------------------------------------------
// one work item
// ---------------------------------------------------------------------------

// One axis of the 3D current in Esirkepov's closed form, split into the core
// of the old support (K = ORDER+1 nodes from window position p0) and the one
// node (S-type: old shape S, change D) or face (P-type: the prefix current P
// along the axis) outside it, which is nonzero only when the support widened.
// The transverse factor S_B S_C + (D_B S_C + S_B D_C)/2 + D_B D_C/3 of the
// closed form equals H_B H_C + G_B G_C with H = S + D/2 and G = D/sqrt(12),
// so each axis carries H and G instead of S and D.
template <int K>
struct DepAxis {
  float H[K], G[K];
  float P[K - 1];
  float He, Ge, Pe;
  int oS, oP;  // node offsets of the extras from the core origin
  bool wide;
};

// Component A of the current (flow along axis A; B, C the other axes) on one
// block of nodes: core or extra along each axis (EA, EB, EC).  The value is
// P_A * (H_B H_C + G_B G_C).
template <int K, int A, bool EA, bool EB, bool EC, typename Acc>
__device__ __forceinline__ void dep3_part(Acc* J, int cb, const int st[3], const DepAxis<K> (&ax)[3]) {
  constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
  constexpr int NA = EA ? 1 : K - 1, NB = EB ? 1 : K, NC = EC ? 1 : K;
#pragma unroll
  for (int kc = 0; kc < NC; kc++) {
    const float hc = EC ? ax[C].He : ax[C].H[kc], gc = EC ? ax[C].Ge : ax[C].G[kc];
    const int oc = (EC ? ax[C].oS : kc) * st[C];
#pragma unroll
    for (int kb = 0; kb < NB; kb++) {
      const float hb = EB ? ax[B].He : ax[B].H[kb], gb = EB ? ax[B].Ge : ax[B].G[kb];
      const float T = fmaf(hb, hc, gb * gc);
      const int ob = cb + oc + (EB ? ax[B].oS : kb) * st[B];
#pragma unroll
      for (int ka = 0; ka < NA; ka++) {
        const float pa = EA ? ax[A].Pe : ax[A].P[ka];
        lds_add_any(J + ob + (EA ? ax[A].oP : ka) * st[A], pa * T);
      }
    }
  }
}

template <int K, int A, typename Acc>
__device__ __forceinline__ void dep3_comp(Acc* J, int cb, const int st[3], const DepAxis<K> (&ax)[3]) {
  constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
  const bool wa = ax[A].wide, wb = ax[B].wide, wc = ax[C].wide;
  dep3_part<K, A, false, false, false>(J, cb, st, ax);
  if (wa) dep3_part<K, A, true, false, false>(J, cb, st, ax);
  if (wb) dep3_part<K, A, false, true, false>(J, cb, st, ax);
  if (wc) dep3_part<K, A, false, false, true>(J, cb, st, ax);
  if (wa && wb) dep3_part<K, A, true, true, false>(J, cb, st, ax);
  if (wa && wc) dep3_part<K, A, true, false, true>(J, cb, st, ax);
  if (wb && wc) dep3_part<K, A, false, true, true>(J, cb, st, ax);
  if (wa && wb && wc) dep3_part<K, A, true, true, true>(J, cb, st, ax);
}

// MODE selects the boundary logic compiled into the kernel: 0 periodic,
// 1 moving window along x1 (a launch whose stores include a moving window),
// 2 the 2D r-z geometry (x1 = z, x2 = r), 3 both.  Without it the code is
// absent.  Modes 4-6 are the two-phase periodic 3D kernel (process_item3):
// 4 with an int64 current tile (the deterministic int64 accumulation), 5 and
// 6 with a 32-bit tile, 5 for the LDS strides of 4x4xN tiles as constants,
// 6 for strides read at run time.  Mode 7 is the two-phase periodic 2D
// kernel (process_item2) for FP32 accumulation with Esirkepov's deposit.
// kstep: steps done since the last rebin check (0 for the first step of a
// sort cycle).
template <int DIM, int ORDER, int MODE>
__device__ void process_item(const StoreDesc& S, int cur, const Item it, int ii, int jp, int kstep, float* smem,
                             int* scnt) {
  constexpr int NG = ORDER + 1;  // gather taps per axis
  constexpr int W = ORDER + 2;   // deposit window per axis
  constexpr bool WIN = MODE == 1 || MODE == 3;
  constexpr bool RZ = DIM == 2 && (MODE == 2 || MODE == 3);
  const GridDesc& g = S.g;
  const int tid = threadIdx.x;

  const int set = cur;
  gint* __restrict__ cellp = (gint*)S.cell[set];
  gfloat* __restrict__ ep0 = (gfloat*)S.eps[set][0];
  gfloat* __restrict__ ep1 = (gfloat*)S.eps[set][1];
  gfloat* __restrict__ ep2 = (gfloat*)S.eps[set][2];
  gfloat* __restrict__ up0 = (gfloat*)S.u[set][0];
  gfloat* __restrict__ up1 = (gfloat*)S.u[set][1];
  gfloat* __restrict__ up2 = (gfloat*)S.u[set][2];
  const gfloat* __restrict__ wp = (const gfloat*)S.w[set];

  int tc[3];
  pic_tile_coords(g, it.tile, tc);
  // How far a particle can be outside its tile at the start of this step:
  // 0 after a check that re-sorted (or a load), flag_slack after one that
  // did not, plus what kstep steps can cover along each axis; never more
  // than the last step of a cycle, for which the LDS is sized.  Only that
  // much halo is staged and flushed.
  // (the values are uniform: kept in scalar registers, so the per-particle
  // code keeps its vector registers)
  const int s0 = __builtin_amdgcn_readfirstlane(S.ctl->sorted) ? 0 : g.flag_slack;
  int sl[3];
#pragma unroll
  for (int d = 0; d < 3; d++)
    sl[d] = d < DIM ? __builtin_amdgcn_readfirstlane(min(s0 + (int)ceilf((float)kstep * g.vstep[d]), g.slk[d])) : 0;
  int org[3], ext[3], FR[3], JR[3], flo[3], jlo[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    if (d < DIM) {
      org[d] = tc[d] * g.tile[d];
      ext[d] = min(g.tile[d], g.nx[d] - org[d]);
      flo[d] = sl[d] + g.fa;  // region-relative index of tile node 0
      jlo[d] = sl[d] + g.ja;
      FR[d] = ext[d] + 2 * sl[d] + g.fa + g.fb;
      JR[d] = ext[d] + 2 * sl[d] + g.ja + g.jb;
    } else {
      org[d] = 0; ext[d] = 1; flo[d] = 0; jlo[d] = 0; FR[d] = 1; JR[d] = 1;
    }
  }
  const int fn = FR[0] * FR[1] * FR[2];
  const int jn = JR[0] * JR[1] * JR[2];
  float* sF = smem;                                     // [6][fn]
  acc_t* sJ = (acc_t*)(smem + ((6 * fn + 1) & ~1));     // [3][jn], 8-byte aligned

  // the state of each thread's first particle is requested here, after the
  // control word above has arrived and before the fields are staged, so its
  // latency overlaps the staging
  int n_cell = 0;
  float n_e0 = 0.0f, n_e1 = 0.0f, n_e2 = 0.0f, n_ux = 0.0f, n_uy = 0.0f, n_uz = 0.0f, n_w = 0.0f;
  if (it.begin + tid < it.end) {
    const int p = it.begin + tid;
    n_cell = cellp[p];
    n_e0 = ep0[p];
    n_e1 = ep1[p];
    if (DIM == 3) n_e2 = ep2[p];
    n_ux = up0[p];
    n_uy = up1[p];
    n_uz = up2[p];
    n_w = wp[p];
  }
  // 1. stage E, B with periodic wrap
  const int ncell = g.ncell;
  {
    BoxWalk bw(tid, blockDim.x, FR);
    const gfloat* Fg = (const gfloat*)S.F[jp];
    for (int idx = tid; idx < fn; idx += blockDim.x, bw.advance(FR)) {
      int gx = wrap_fast(org[0] - flo[0] + bw.x, g.nx[0]);
      if constexpr (RZ) {
        // r-z: rows below the axis are mirror images (z components keep the
        // sign, r and theta components change it); rows at and beyond the
        // wall hold zero.  E_z, E_theta, B_r sit on whole rows, E_r, B_z,
        // B_theta on half rows (the axis is half row 0).
        const int ry = org[1] - flo[1] + bw.y;
        const int rw = ry <= 0 ? 1 - ry : ry;
        const int rh = ry < 0 ? -ry : ry;
        const float sw = ry <= 0 ? -1.0f : 1.0f, sh = ry < 0 ? -1.0f : 1.0f;
        const bool iw = rw < g.nx[1], ih = rh < g.nx[1];
        const int gw = gx + g.nx[0] * rw, gh = gx + g.nx[0] * rh;
        const float ez = iw ? Fg[gw] : 0.0f;
        const float er = ih ? sh * Fg[(size_t)ncell + gh] : 0.0f;
        const float et = iw ? sw * Fg[(size_t)2 * ncell + gw] : 0.0f;
        sF[idx] = ez;
        sF[fn + idx] = er;
        sF[2 * fn + idx] = et;
        sF[3 * fn + idx] = ih ? Fg[(size_t)3 * ncell + gh] : 0.0f;
        sF[4 * fn + idx] = iw ? sw * Fg[(size_t)4 * ncell + gw] : 0.0f;
        sF[5 * fn + idx] = ih ? sh * Fg[(size_t)5 * ncell + gh] : 0.0f;
        continue;
      }
      // two nodes per round: the loads of both are in flight together
      const int idx2 = idx + blockDim.x;
      int gy = wrap_fast(org[1] - flo[1] + bw.y, g.nx[1]);
      int gz = DIM == 3 ? wrap_fast(org[2] - flo[2] + bw.z, g.nx[2]) : 0;
      const int gi = gx + g.nx[0] * (gy + g.nx[1] * gz);
      bw.advance(FR);
      const bool two = idx2 < fn;
      int gi2 = gi;
      if (two) {
        const int gx2 = wrap_fast(org[0] - flo[0] + bw.x, g.nx[0]);
        const int gy2 = wrap_fast(org[1] - flo[1] + bw.y, g.nx[1]);
        const int gz2 = DIM == 3 ? wrap_fast(org[2] - flo[2] + bw.z, g.nx[2]) : 0;
        gi2 = gx2 + g.nx[0] * (gy2 + g.nx[1] * gz2);
      }
      float v1[6], v2[6];
#pragma unroll
      for (int c = 0; c < 6; c++) v1[c] = Fg[(size_t)c * ncell + gi];
      if (two) {
#pragma unroll
        for (int c = 0; c < 6; c++) v2[c] = Fg[(size_t)c * ncell + gi2];
      }
#pragma unroll
      for (int c = 0; c < 6; c++) sF[c * fn + idx] = v1[c];
      if (two) {
#pragma unroll
        for (int c = 0; c < 6; c++) sF[c * fn + idx2] = v2[c];
      }
      idx = idx2;  // the loop step takes it (and the walker) one node further
    }
  }
  // 2. clear the current tile and the rebin slot counters
  for (int idx = tid; idx < 3 * jn; idx += blockDim.x) sJ[idx] = 0ull;
  if (tid < PIC_NSLOT) scnt[tid] = 0;
  __syncthreads();
  // the instance's fixed point (see the host's current scale); the two-phase
  // 3D kernel below chooses one per work item instead
  const float Qi = g.jscale;

  const float h = 0.5f * S.qm * g.dt;
  bool strayed = false, bad = false, died = false;
  // moving window: ring origin of the x1 columns and whether the window
  // moves after this step (its back column is then discarded)
  const bool win = WIN && g.window != 0;
  int wo = 0;
  bool wshift = false;
  if (win) {
    const WinCtl wc = *S.win;
    wo = wc.origin;
    wshift = pic_win_shifts(g.wa, wc.step + 1) > pic_win_shifts(g.wa, wc.step);
  }

  // 3. particles; the next particle's state is loaded while this one is
  // processed (hides the global-load latency at the top of the loop)
  for (int p = it.begin + tid; p < it.end; p += blockDim.x) {
    int cell = n_cell;
    float e[3];
    e[0] = n_e0;
    e[1] = n_e1;
    e[2] = DIM == 3 ? n_e2 : 0.0f;
    float ux = n_ux, uy = n_uy, uz = n_uz;
    float wq = n_w;
    {
      const int pn = p + blockDim.x;
      if (pn < it.end) {
        n_cell = cellp[pn];
        n_e0 = ep0[pn];
        n_e1 = ep1[pn];
        if (DIM == 3) n_e2 = ep2[pn];
        n_ux = up0[pn];
        n_uy = up1[pn];
        n_uz = up2[pn];
        n_w = wp[pn];
      }
    }
    if ((win || RZ) && cell < 0) continue;  // removed, awaiting the rebin
    int cc[3];
    pic_unpack(g, cell, cc);
    int l[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; d++) {
      l[d] = pic_local(cc[d], org[d], ext[d], g.nx[d]);
      ok = ok && (l[d] >= -sl[d]) && (l[d] < ext[d] + sl[d]);
    }
    if (!ok) {
      bad = true;
      if constexpr (WIN || RZ) continue;
      // periodic: the step is reported as failed; the lane still runs,
      // clamped into the staged region, so that every path through the loop
      // body ends in the stores and the wait for the next particle's loads
      // at the loop's end does not wait for this particle's stores too
#pragma unroll
      for (int d = 0; d < DIM; d++) l[d] = min(max(l[d], -sl[d]), ext[d] + sl[d] - 1);
    }

    // ---- gather: weights at offset 0 and 1/2 per axis
    int b0[3], bh[3];
    float w0[3][NG], wh[3][NG];
#pragma unroll
    for (int d = 0; d < DIM; d++) {
      gather_weights<ORDER>(e[d], false, b0[d], w0[d]);
      gather_weights<ORDER>(e[d], true, bh[d], wh[d]);
    }
    // moving window: x1 nodes beyond the window's ends hold zero fields
    int wcol = 0;
    if (win) {
      wcol = cc[0] - wo;
      if (wcol < 0) wcol += g.nx[0];
#pragma unroll
      for (int i = 0; i < NG; i++) {
        if ((unsigned)(wcol + b0[0] + i) >= (unsigned)g.nx[0]) w0[0][i] = 0.0f;
        if ((unsigned)(wcol + bh[0] + i) >= (unsigned)g.nx[0]) wh[0][i] = 0.0f;
      }
    }
    float Fp[6];
    // LDS offsets of the first tap: one multiply per particle; the offsets of
    // the half-staggered nodes differ from the node ones by 0 or -1 per axis
    const int FR0 = FR[0];
    const int gb0 = (flo[1] + l[1] + b0[1]) * FR0 + flo[0] + l[0] + b0[0];
    const int dgx = bh[0] - b0[0];
    const int dgy = bh[1] == b0[1] ? 0 : (bh[1] < b0[1] ? -FR0 : FR0);
#pragma unroll
    for (int c = 0; c < 6; c++) {
      // component c: E_c staggered half along axis c, B_c half along the others
      bool hx = (c < 3) ? (c == 0) : (c != 3);
      bool hy = (c < 3) ? (c == 1) : (c != 4);
      bool hz = (c < 3) ? (c == 2) : (c != 5);
      const float* wx = hx ? wh[0] : w0[0];
      const float* wy = hy ? wh[1] : w0[1];
      int sx = flo[0] + l[0] + (hx ? bh[0] : b0[0]);
      int sy = flo[1] + l[1] + (hy ? bh[1] : b0[1]);
      const float* Fc = sF + c * fn;
      float acc = 0.0f;
      if constexpr (DIM == 2) {
        const float* row = Fc + gb0 + (hx ? dgx : 0) + (hy ? dgy : 0);
#pragma unroll
        for (int j = 0; j < NG; j++) {
          float r = 0.0f;
#pragma unroll
          for (int i = 0; i < NG; i++) r += wx[i] * row[i];
          acc += wy[j] * r;
          row += FR0;
        }
      } else {
        const float* wz = hz ? wh[2] : w0[2];
        int sz = flo[2] + l[2] + (hz ? bh[2] : b0[2]);
#pragma unroll
        for (int k = 0; k < NG; k++) {
          float pl = 0.0f;
#pragma unroll
          for (int j = 0; j < NG; j++) {
            const float* row = Fc + ((sz + k) * FR[1] + (sy + j)) * FR[0] + sx;
            float r = 0.0f;
#pragma unroll
            for (int i = 0; i < NG; i++) r += wx[i] * row[i];
            pl += wy[j] * r;
          }
          acc += wz[k] * pl;
        }
      }
      Fp[c] = acc;
    }
    float Ex = Fp[0] + g.e0[0], Ey = Fp[1] + g.e0[1], Ez = Fp[2] + g.e0[2];
    float Bx = Fp[3] + g.b0[0], By = Fp[4] + g.b0[1], Bz = Fp[5] + g.b0[2];

    // ---- Boris push (Sec. 3.2, Eq. momentum-update)
    float mx = ux + h * Ex, my = uy + h * Ey, mz = uz + h * Ez;
    float gim = rsqrtf(1.0f + mx * mx + my * my + mz * mz);
    float tx = h * Bx * gim, ty = h * By * gim, tz = h * Bz * gim;
    float sfac = 2.0f * __builtin_amdgcn_rcpf(1.0f + tx * tx + ty * ty + tz * tz);
    float px = mx + (my * tz - mz * ty);
    float py = my + (mz * tx - mx * tz);
    float pz = mz + (mx * ty - my * tx);
    float sx_ = sfac * tx, sy_ = sfac * ty, sz_ = sfac * tz;
    ux = mx + (py * sz_ - pz * sy_) + h * Ex;
    uy = my + (pz * sx_ - px * sz_) + h * Ey;
    uz = mz + (px * sy_ - py * sx_) + h * Ez;

    // ---- advance (Eq. 2d-position-update; in-plane only in 2D)
    float gi = rsqrtf(1.0f + ux * ux + uy * uy + uz * uz);
    float uu[3] = {ux, uy, uz};
    float en[3];
    int mv[3] = {0, 0, 0};
    float urn = uy, utn = uz;  // r-z: momenta in the frame of the new position
#pragma unroll
    for (int d = 0; d < DIM; d++) {
      float x;
      if (RZ && d == 1) {
        // r-z (Eqs. 2d-cyl-position-update-1..3): the straight 3D move from
        // radius r by (dt v_r, dt v_theta), in cells; the new radius rn and
        // the change rn - r written without cancellation; momenta rotated
        // into the new r-z plane (u_theta from the angular momentum)
        const float r = (float)cc[1] + e[1] - 0.5f;
        const float mr = g.dt * g.rdx[1] * (uy * gi);
        const float mt = g.dt * g.rdx[1] * (uz * gi);
        const float yr = r + mr;
        const float rn = sqrtf(yr * yr + mt * mt);
        const float den = rn + r;
        x = e[1] + (den > 0.0f ? (mr * (r + yr) + mt * mt) / den : 0.0f);
        if (rn > 0.0f) {
          urn = (uy * yr + uz * mt) / rn;
          utn = uz * r / rn;
        } else {
          urn = -uy;  // on the axis: moving out on the other side
          utn = 0.0f;
        }
      } else {
        x = e[d] + g.dt * g.rdx[d] * (uu[d] * gi);
      }
      float f = floorf(x);
      int c = (int)f;
      float r = x - f;
      if (r >= 1.0f) {  // rounding edge: keep the offset in [0,1)
        r = 0.0f;
        c += 1;
      }
      // the Courant condition keeps |move| below one cell; clamp so a
      // rounding of a move at the limit never leaves the deposit window
      if (c > 1) {
        c = 1;
        r = 0.99999994f;
      } else if (c < -1) {
        c = -1;
        r = 0.0f;
      }
      en[d] = r;
      mv[d] = c;
    }

    // ---- deposit
    if (ORDER == 1 && g.deposit == 1) {
      // TRISTAN: the straight move cut at the faces it crosses
      const float js = Qi;
      float dl[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int d = 0; d < DIM; d++) dl[d] = (float)mv[d] + en[d] - e[d];
      const int b0 = jlo[0] + l[0], b1 = jlo[1] + l[1], b2 = DIM == 3 ? jlo[2] + l[2] : 0;
      deposit_tristan<DIM>(sJ, jn, JR, b0, b1, b2, e, dl, mv, wq * g.cdt[0] * js, wq * g.cdt[1] * js,
                           wq * g.cdt[2] * js, wq * uz * gi * js, win ? wcol : -1, g.nx[0]);
    } else {
      // ISIS ordering average in Esirkepov's closed form
      int wb[3], p0[3];
      bool wide[3];
      float S0[3][W], D[3][W];
  #pragma unroll
      for (int d = 0; d < DIM; d++) deposit_shape<ORDER>(e[d], en[d], mv[d], wb[d], p0[d], wide[d], S0[d], D[d]);
      int jx = jlo[0] + l[0] + wb[0];
      int jy = jlo[1] + l[1] + wb[1];
      acc_t* J1 = sJ;
      acc_t* J2 = sJ + jn;
      acc_t* J3 = sJ + 2 * jn;
      const float js = Qi;
      float q1 = -wq * g.cdt[0] * js, q2 = -wq * g.cdt[1] * js;
      float P1[W - 1], P2[W - 1];
      {
        float a = 0.0f, b = 0.0f;
  #pragma unroll
        for (int k = 0; k < W - 1; k++) {
          a += D[0][k];
          b += D[1][k];
          P1[k] = q1 * a;
          P2[k] = q2 * b;
        }
      }
      if (win) {
        // moving window: currents at x1 nodes beyond the window are dropped
        // (the prefix above still counts the charge change there)
#pragma unroll
        for (int k = 0; k < W; k++)
          if ((unsigned)(wcol + wb[0] + k) >= (unsigned)g.nx[0]) {
            S0[0][k] = 0.0f;
            D[0][k] = 0.0f;
            if (k < W - 1) P1[k] = 0.0f;
          }
      }
      if constexpr (DIM == 2) {
        // The window of ORDER+2 nodes per axis splits into a core of K = ORDER+1
        // nodes starting at p0 (the old shape's support, never all zero) and one
        // extra node (p0 = 1: the node below the core; p0 = 0: the node above),
        // which is nonzero only when the support is wide along that axis.  Core
        // adds are unconditional; the extra row, column and corner are added
        // only by the lanes that need them, one branch per group instead of one
        // per add.  J3 is skipped by lanes without out-of-plane motion (an
        // in-plane laser drives none).
        constexpr int K = ORDER + 1;
        const float v3 = wq * uz * gi * js;
        const bool px = p0[0] != 0, py = p0[1] != 0;
        // core and extra of the S0, D windows (S-type: K core values) and of the
        // prefix currents P (K-1 core values)
        float Sx[K], Dx[K], Sy[K], Dy[K], Px[K - 1], Py[K - 1];
  #pragma unroll
        for (int k = 0; k < K; k++) {
          Sx[k] = px ? S0[0][k + 1] : S0[0][k];
          Dx[k] = px ? D[0][k + 1] : D[0][k];
          Sy[k] = py ? S0[1][k + 1] : S0[1][k];
          Dy[k] = py ? D[1][k + 1] : D[1][k];
        }
  #pragma unroll
        for (int k = 0; k < K - 1; k++) {
          Px[k] = px ? P1[k + 1] : P1[k];
          Py[k] = py ? P2[k + 1] : P2[k];
        }
        const float Sxe = px ? S0[0][0] : S0[0][K], Dxe = px ? D[0][0] : D[0][K];
        const float Sye = py ? S0[1][0] : S0[1][K], Dye = py ? D[1][0] : D[1][K];
        const float Pxe = wide[0] ? (px ? P1[0] : P1[K - 1]) : 0.0f;
        const float Pye = wide[1] ? (py ? P2[0] : P2[K - 1]) : 0.0f;
        // node offsets of the extras relative to the core base, per array type
        const int exS = px ? -1 : K, exP = px ? -1 : K - 1;
        const int cx = jx + p0[0], cy = jy + p0[1];
        const int R = JR[0];
        const int cb = cy * R + cx;  // core base: the only multiply of the deposit
        const int ey = py ? -R : K * R;  // row offset of the extra row (S-type)
        const int eyp = py ? -R : (K - 1) * R;  // (P-type)
        // y-direction factors of J1 and J3 (T1 = S0 + D/2, U2 = S0/2 + D/3) and
        // x-direction factor of J2 (S0 + D/2)
        float T1[K], U2[K], X2[K];
  #pragma unroll
        for (int k = 0; k < K; k++) {
          T1[k] = Sy[k] + 0.5f * Dy[k];
          U2[k] = 0.5f * Sy[k] + (1.0f / 3.0f) * Dy[k];
          X2[k] = Sx[k] + 0.5f * Dx[k];
        }
        const float T1e = Sye + 0.5f * Dye, U2e = 0.5f * Sye + (1.0f / 3.0f) * Dye;
        const float X2e = Sxe + 0.5f * Dxe;
        // core
  #pragma unroll
        for (int j = 0; j < K; j++) {
          acc_t* r1 = J1 + cb + j * R;
          acc_t* r3 = J3 + cb + j * R;
  #pragma unroll
          for (int i = 0; i < K - 1; i++) lds_add_any(r1 + i, Px[i] * T1[j]);
          if (v3 != 0.0f) {
  #pragma unroll
            for (int i = 0; i < K; i++) lds_add_any(r3 + i, v3 * (Sx[i] * T1[j] + Dx[i] * U2[j]));
          }
        }
  #pragma unroll
        for (int j = 0; j < K - 1; j++) {
          acc_t* r2 = J2 + cb + j * R;
  #pragma unroll
          for (int i = 0; i < K; i++) lds_add_any(r2 + i, Py[j] * X2[i]);
        }
        // extra column (x)
        if (wide[0]) {
  #pragma unroll
          for (int j = 0; j < K; j++) {
            lds_add_any(J1 + cb + j * R + exP, Pxe * T1[j]);
            if (v3 != 0.0f) lds_add_any(J3 + cb + j * R + exS, v3 * (Sxe * T1[j] + Dxe * U2[j]));
          }
  #pragma unroll
          for (int j = 0; j < K - 1; j++) lds_add_any(J2 + cb + j * R + exS, Py[j] * X2e);
        }
        // extra row (y)
        if (wide[1]) {
  #pragma unroll
          for (int i = 0; i < K - 1; i++) lds_add_any(J1 + cb + ey + i, Px[i] * T1e);
  #pragma unroll
          for (int i = 0; i < K; i++) {
            if (v3 != 0.0f) lds_add_any(J3 + cb + ey + i, v3 * (Sx[i] * T1e + Dx[i] * U2e));
            lds_add_any(J2 + cb + eyp + i, Pye * X2[i]);
          }
        }
        // extra corner
        if (wide[0] && wide[1]) {
          lds_add_any(J1 + cb + ey + exP, Pxe * T1e);
          if (v3 != 0.0f) lds_add_any(J3 + cb + ey + exS, v3 * (Sxe * T1e + Dxe * U2e));
          lds_add_any(J2 + cb + eyp + exS, Pye * X2e);
        }
      } else {
        // 3D: per axis the core of ORDER+1 nodes of the old support plus one
        // extra node (or face) that only a widened support reaches, as in 2D;
        // core adds are unconditional, each extra block is one branch.  A
        // particle that did not move deposits nothing.
        const bool moved = mv[0] != 0 || mv[1] != 0 || mv[2] != 0 || en[0] != e[0] || en[1] != e[1] ||
                           en[2] != e[2];
        if (moved) {
          int jz = jlo[2] + l[2] + wb[2];
          float q3 = -wq * g.cdt[2] * js;
          float P3[W - 1];
          {
            float a = 0.0f;
  #pragma unroll
            for (int k = 0; k < W - 1; k++) {
              a += D[2][k];
              P3[k] = q3 * a;
            }
          }
          constexpr int K = ORDER + 1;
          DepAxis<K> ax[3];
          const float* Pw[3] = {P1, P2, P3};
  #pragma unroll
          for (int d = 0; d < 3; d++) {
            const bool pd = p0[d] != 0;
  #pragma unroll
            for (int k = 0; k < K; k++) {
              const float sk = pd ? S0[d][k + 1] : S0[d][k], dk = pd ? D[d][k + 1] : D[d][k];
              ax[d].H[k] = fmaf(0.5f, dk, sk);
              ax[d].G[k] = 0.28867513f * dk;  // 1/sqrt(12)
            }
  #pragma unroll
            for (int k = 0; k < K - 1; k++) ax[d].P[k] = pd ? Pw[d][k + 1] : Pw[d][k];
            {
              const float se = pd ? S0[d][0] : S0[d][K], de = pd ? D[d][0] : D[d][K];
              ax[d].He = fmaf(0.5f, de, se);
              ax[d].Ge = 0.28867513f * de;
            }
            ax[d].Pe = wide[d] ? (pd ? Pw[d][0] : Pw[d][K - 1]) : 0.0f;
            ax[d].oS = pd ? -1 : K;
            ax[d].oP = pd ? -1 : K - 1;
            ax[d].wide = wide[d];
          }
          const int st[3] = {1, JR[0], JR[0] * JR[1]};
          const int cb = ((jz + p0[2]) * JR[1] + (jy + p0[1])) * JR[0] + jx + p0[0];
          dep3_comp<K, 0>(J1, cb, st, ax);
          dep3_comp<K, 1>(J2, cb, st, ax);
          dep3_comp<K, 2>(J3, cb, st, ax);
        }
      }

    }

    // ---- store the new state; count the particle's rebin slot
    if constexpr (RZ) {
      uy = urn;  // the deposit above used the push's u_theta
      uz = utn;
    }
    int nc[3] = {0, 0, 0};
    int dd[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; d++) {
      nc[d] = cc[d] + mv[d];
      if (nc[d] < 0) nc[d] += g.nx[d];
      if (nc[d] >= g.nx[d]) nc[d] -= g.nx[d];
      int ln = pic_local(nc[d], org[d], ext[d], g.nx[d]);
      strayed = strayed || ln < -g.flag_slack || ln >= ext[d] + g.flag_slack;
      dd[d] = ln < 0 ? -1 : (ln >= ext[d] ? 1 : 0);
    }
    // moving window: a particle that left through an x1 face, or sits in the
    // back column when the window moves after this step, is removed (its
    // current of this step is already deposited)
    bool dead = false;
    if (win) {
      const int wn = wcol + mv[0];
      dead = wn < 0 || wn >= g.nx[0] || (wshift && wn == 0);
      died = died || dead;
    }
    if constexpr (RZ) {
      // r-z: a particle that reached the wall is removed
      dead = dead || cc[1] + mv[1] >= g.nx[1];
      died = died || dead;
    }
    {
      // wave-aggregated count per slot (almost every particle is in slot 13)
      const int sl = dead ? -1 : pic_slot(dd[0], dd[1], dd[2]);
      unsigned long long todo = __ballot(sl >= 0);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int ls = __shfl(sl, leader);
        const unsigned long long m = __ballot(sl == ls);
        if ((int)(threadIdx.x & 63) == leader) atomicAdd(&scnt[ls], (int)__popcll(m));
        todo &= ~m;
      }
    }
    cellp[p] = dead ? -1 : pic_pack(g, nc[0], nc[1], DIM == 3 ? nc[2] : 0);
    ep0[p] = en[0];
    ep1[p] = en[1];
    if (DIM == 3) ep2[p] = en[2];
    up0[p] = ux;
    up1[p] = uy;
    up2[p] = uz;
  }
  // one plain store per workgroup (all writers store the same value)
  const int any_strayed = __syncthreads_or((strayed || died) ? 1 : 0);
  const int any_bad = __syncthreads_or(bad ? 1 : 0);
  if (tid == 0) {
    if (any_strayed) S.ctl->flag = 1;
    if (any_bad) S.ctl->bad = 1;
  }
  if (tid < PIC_NSLOT) S.cnt[ii * PIC_NSLOT + tid] = scnt[tid];

  // 4. fold the LDS current into the global current (periodic wrap): FP32
  // atomics of the sums times the unit, or int64 atomics of the sums
  const float qinv = g.jinv;
  BoxWalk bj(tid, blockDim.x, JR);
  for (int idx = tid; idx < jn; idx += blockDim.x, bj.advance(JR)) {
    int gx = wrap_fast(org[0] - jlo[0] + bj.x, g.nx[0]);
    if constexpr (RZ) {
      // r-z: current below the axis goes to the mirror row with the mirror
      // sign (J_z keeps it, J_r and J_theta change it; J_r on the axis
      // cancels itself), current at and beyond the wall is dropped
      const int ry = org[1] - jlo[1] + bj.y;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        long long q = (long long)sJ[c * jn + idx];
        const int row = c == 1 ? (ry < 0 ? -ry : ry) : (ry <= 0 ? 1 - ry : ry);
        if (q == 0 || row >= g.nx[1] || (c == 1 && ry == 0)) continue;
        if ((c == 1 && ry < 0) || (c == 2 && ry <= 0)) q = -q;
        const size_t gi = (size_t)c * ncell + gx + g.nx[0] * row;
        if (g.acc_mode == 2)
          atomicAdd(S.J64[jp] + gi, (acc_t)q);
        else
          __builtin_amdgcn_global_atomic_fadd_f32((gfloat*)S.Jacc[jp] + gi, item_sum_f32(q, qinv));
      }
      continue;
    }
    int gy = wrap_fast(org[1] - jlo[1] + bj.y, g.nx[1]);
    int gz = DIM == 3 ? wrap_fast(org[2] - jlo[2] + bj.z, g.nx[2]) : 0;
    int gi = gx + g.nx[0] * (gy + g.nx[1] * gz);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      long long q = (long long)sJ[c * jn + idx];
      if (q != 0) {
        if (g.acc_mode == 2)
          atomicAdd(S.J64[jp] + (size_t)c * ncell + gi, (acc_t)q);
        else
          __builtin_amdgcn_global_atomic_fadd_f32((gfloat*)S.Jacc[jp] + (size_t)c * ncell + gi,
                                                  item_sum_f32(q, qinv));
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// periodic 3D work item in two phases
// ---------------------------------------------------------------------------
//
// Phase A stages E and B of the tile and pushes every particle of the item
// (up to kSplitR per thread), keeping what the deposit needs in registers.
// Phase B clears the integer current tile in the same LDS and deposits into it.
// Field tile and current tile never coexist, so a workgroup needs the larger
// of the two instead of their sum, and more workgroups share a CU.  The
// regions carry only the guards the shapes reach (see the host's region
// guards of this variant).
//
// The fixed point of the tile is chosen per work item from the particles
// just pushed.  A contribution of particle p to one node is at most
// |w_p| |v_p|: the charge fraction that crosses a face in one step is at most
// the displacement in cells (the prefix of the shape change along the axis
// is 1-Lipschitz), and the transverse weight (a time average of products of
// shape values) is at most one.  With Q = 2^e and Q max_p |w_p| |v_p| < 2^29
// every contribution converts to an int32 (with a factor 2 to spare for the
// FP32 rounding of the shape differences) and the int64 sums are exact; the
// rounding unit follows the item's fastest particle instead of the speed of
// light, so a slow or cold plasma keeps its relative precision.
//
// The tile is 32-bit (Acc = unsigned) unless the instance sums its current
// deterministically in int64.  A node gets at most one contribution per
// particle of the item, so Q max_p |w_p| |v_p| n < 2^31 (with a small margin
// for rounding) for an item of n particles keeps the int32 sums exact
// (item_exponent32): the unit is about 2^-31 n of the largest contribution,
// 2^-23 for the 256 particles of a 4x4x4 tile at four per cell, the FP32
// rounding of one such contribution.  A 32-bit tile halves the LDS lane
// traffic of the adds and drops the sign extension of each one.

constexpr int kSplitR = 3;  // particles per thread per work item

// LDS the re-interleave below needs: class counts, and one occupancy mask
// and one start per level (at most one level per particle of the item)
constexpr size_t kInterleaveLds = 64 * sizeof(int) + (size_t)kSplitR * kBlock * (sizeof(unsigned long long) + sizeof(int));

// The particles of a work item are stored after the step inside the item's
// range in cell-interleaved order: the cells of the tile fall into 64
// classes (local linear index mod 64, x fastest), and the order is the first
// particle of every class in class order, then the second of every class,
// and so on.  The lanes of a wavefront then hold particles of (nearly) 64
// different cells, so the next step's LDS gathers and current adds spread
// over the banks and rarely hit one address together; without it the loaded
// order decays as particles change cells, and the kernel slows by about a
// third.  Among particles of one class the order is that of the LDS atomics
// (not reproducible), which only permutes storage: every particle's own
// arithmetic, the item's membership and its fixed-point unit are unchanged,
// and the integer current sums are order-free.
//
// interleave_slots: key[r] is the class of the thread's r-th particle (-1:
// none); on return pos[r] is its slot in the item.  smem is free LDS of at
// least kInterleaveLds bytes; every thread of the workgroup calls it.
__device__ __forceinline__ void interleave_slots(const int (&key)[kSplitR], int (&pos)[kSplitR], float* smem) {
  constexpr int R = kSplitR;
  const int tid = threadIdx.x;
  int* s_n = (int*)smem;                                      // [64]
  unsigned long long* s_m = (unsigned long long*)(smem + 64); // [R * kBlock]
  int* s_l = (int*)(s_m + R * kBlock);                        // [R * kBlock]
  if (tid < 64) s_n[tid] = 0;
  __syncthreads();
  int lev[R];
#pragma unroll
  for (int r = 0; r < R; r++) lev[r] = key[r] >= 0 ? atomicAdd(&s_n[key[r]], 1) : 0;
  __syncthreads();
  if (tid < 64) {
    // level k holds the classes with more than k particles: its occupancy
    // mask and its start in the item
    const int n = s_n[tid];
    int top = n;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) top = max(top, __shfl_xor(top, off));
    int acc = 0;
    for (int k = 0; k < top; k++) {
      const unsigned long long m = __ballot(n > k);
      if (tid == 0) {
        s_m[k] = m;
        s_l[k] = acc;
      }
      acc += (int)__popcll(m);
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; r++)
    pos[r] = key[r] >= 0 ? s_l[lev[r]] + (int)__popcll(s_m[lev[r]] & ((1ull << key[r]) - 1ull)) : -1;
  __syncthreads();  // the tables are read before the LDS is reused
}

// FIXED: the LDS strides are the 12-node rows and 144-node planes that 4x4xN
// tiles take (every shape order, stray bound 1), as compile-time constants,
// so that the taps and adds address LDS through instruction offsets.
template <int ORDER, bool FIXED, typename Acc>
__device__ void process_item3(const StoreDesc& S, int cur, const Item it, int ii, int jp, int kstep, float* smem,
                              int* scnt, float* sred) {
  constexpr bool kWide = sizeof(Acc) == 8;
  constexpr int NG = ORDER + 1;  // gather taps per axis
  constexpr int K = ORDER + 1;   // deposit core per axis
  constexpr int W = ORDER + 2;   // deposit window per axis
  constexpr int R = kSplitR;
  const GridDesc& g = S.g;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;

  const int set = cur;
  gint* __restrict__ cellp = (gint*)S.cell[set];
  gfloat* __restrict__ ep0 = (gfloat*)S.eps[set][0];
  gfloat* __restrict__ ep1 = (gfloat*)S.eps[set][1];
  gfloat* __restrict__ ep2 = (gfloat*)S.eps[set][2];
  gfloat* __restrict__ up0 = (gfloat*)S.u[set][0];
  gfloat* __restrict__ up1 = (gfloat*)S.u[set][1];
  gfloat* __restrict__ up2 = (gfloat*)S.u[set][2];
  gfloat* __restrict__ wp = (gfloat*)S.w[set];
  gint* __restrict__ idp = (gint*)S.id[set];

  int tc[3];
  pic_tile_coords(g, it.tile, tc);
  // stray bound of this step (as in the one-phase kernel)
  const int s0 = __builtin_amdgcn_readfirstlane(S.ctl->sorted) ? 0 : g.flag_slack;
  int sl[3], org[3], ext[3], FR[3], JR[3], flo[3], jlo[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    sl[d] = __builtin_amdgcn_readfirstlane(min(s0 + (int)ceilf((float)kstep * g.vstep[d]), g.slk[d]));
    org[d] = tc[d] * g.tile[d];
    ext[d] = min(g.tile[d], g.nx[d] - org[d]);
    flo[d] = sl[d] + g.fa;
    jlo[d] = sl[d] + g.ja;
    FR[d] = ext[d] + 2 * sl[d] + g.fa + g.fb;
    JR[d] = ext[d] + 2 * sl[d] + g.ja + g.jb;
  }
  // LDS layout: padded row and plane strides (fixed for the box, sized for
  // the largest region of a sort cycle); fn / jn count the region's nodes
  const int fn = FR[0] * FR[1] * FR[2];
  const int jn = JR[0] * JR[1] * JR[2];
  const int fs0 = FIXED ? 12 : g.fs0, fs01 = FIXED ? 144 : g.fs01;
  const int js0 = FIXED ? 12 : g.js0, js01 = FIXED ? 144 : g.js01;
  const int fpl = fs01 * FR[2];  // one field component
  const int jpl = js01 * JR[2];  // one current component
  float* sF = smem;            // phase A: [6][fpl]
  Acc* sJ = (Acc*)smem;        // phase B: [3][jpl]

  // this thread's particles: requested before the fields are staged
  int pc[R], pid[R];
  float pe[R][3], pu[R][3], pw[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int p = it.begin + tid + r * nthr;
    pc[r] = -1;
    pid[r] = 0;
    pe[r][0] = pe[r][1] = pe[r][2] = 0.0f;
    pu[r][0] = pu[r][1] = pu[r][2] = 0.0f;
    pw[r] = 0.0f;
    if (p < it.end) {
      pc[r] = cellp[p];
      pe[r][0] = ep0[p];
      pe[r][1] = ep1[p];
      pe[r][2] = ep2[p];
      pu[r][0] = up0[p];
      pu[r][1] = up1[p];
      pu[r][2] = up2[p];
      pw[r] = wp[p];
      pid[r] = idp[p];
    }
  }

  // 1. stage E, B with periodic wrap: four nodes per thread per batch, every
  // load of a batch in flight before its LDS writes
  const int ncell = g.ncell;
  {
    const gfloat* Fg = (const gfloat*)S.F[jp];
    BoxWalk bw(tid, nthr, FR);
    for (int base = 0; base < fn; base += 4 * nthr) {
      float v[4][6];
      int gi[4];
      int li[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int gx = wrap_fast(org[0] - flo[0] + bw.x, g.nx[0]);
        const int gy = wrap_fast(org[1] - flo[1] + bw.y, g.nx[1]);
        const int gz = wrap_fast(org[2] - flo[2] + bw.z, g.nx[2]);
        gi[q] = gx + g.nx[0] * (gy + g.nx[1] * gz);
        li[q] = bw.x + bw.y * fs0 + bw.z * fs01;
        bw.advance(FR);
      }
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (base + q * nthr + tid < fn) {
#pragma unroll
          for (int c = 0; c < 6; c++) v[q][c] = Fg[(size_t)c * ncell + gi[q]];
        }
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if (base + q * nthr + tid < fn) {
#pragma unroll
          for (int c = 0; c < 6; c++) sF[c * fpl + li[q]] = v[q][c];
        }
      }
    }
  }
  if (tid < PIC_NSLOT) scnt[tid] = 0;
  __syncthreads();

  // 2. phase A: gather, Boris push, advance; store the new state
  const float h = 0.5f * S.qm * g.dt;
  bool strayed = false, bad = false;
  float bmax = 0.0f;
  // kept for the deposit: old and new offsets, the move, the weight and the
  // old cell in current-region coordinates (-1: nothing to deposit); kept
  // for the interleaved store: the new cell, its class (-1: no particle) and
  // the new momentum
  float se0[R][3], sen[R][3], swq[R], snu[R][3];
  int smv[R], sjc[R], sncell[R], skey[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int p = it.begin + tid + r * nthr;
    smv[r] = 0;
    sjc[r] = -1;
    skey[r] = -1;
    sncell[r] = 0;
    swq[r] = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; d++) se0[r][d] = sen[r][d] = snu[r][d] = 0.0f;
    int dd[3] = {0, 0, 0};
    bool live = p < it.end;
    if (live) {
      int cc[3];
      pic_unpack(g, pc[r], cc);
      int l[3];
      bool ok = true;
#pragma unroll
      for (int d = 0; d < 3; d++) {
        l[d] = pic_local(cc[d], org[d], ext[d], g.nx[d]);
        ok = ok && (l[d] >= -sl[d]) && (l[d] < ext[d] + sl[d]);
      }
      if (!ok) {
        // reported as a failed step; the particle is clamped into the
        // staged region so that every access stays inside it
        bad = true;
#pragma unroll
        for (int d = 0; d < 3; d++) l[d] = min(max(l[d], -sl[d]), ext[d] + sl[d] - 1);
      }
      const float e[3] = {pe[r][0], pe[r][1], pe[r][2]};
      // ---- gather: weights at offset 0 and 1/2 per axis
      int b0[3], bh[3];
      float w0[3][NG], wh[3][NG];
#pragma unroll
      for (int d = 0; d < 3; d++) {
        gather_weights<ORDER>(e[d], false, b0[d], w0[d]);
        gather_weights<ORDER>(e[d], true, bh[d], wh[d]);
      }
      float Fp[6];
#pragma unroll
      for (int c = 0; c < 6; c++) {
        // component c: E_c staggered half along axis c, B_c half along the others
        const bool hx = (c < 3) ? (c == 0) : (c != 3);
        const bool hy = (c < 3) ? (c == 1) : (c != 4);
        const bool hz = (c < 3) ? (c == 2) : (c != 5);
        const float* wx = hx ? wh[0] : w0[0];
        const float* wy = hy ? wh[1] : w0[1];
        const float* wz = hz ? wh[2] : w0[2];
        const int sx = flo[0] + l[0] + (hx ? bh[0] : b0[0]);
        const int sy = flo[1] + l[1] + (hy ? bh[1] : b0[1]);
        const int sz = flo[2] + l[2] + (hz ? bh[2] : b0[2]);
        const float* Fc = sF + c * fpl + sz * fs01 + sy * fs0 + sx;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < NG; k++) {
          float pl = 0.0f;
#pragma unroll
          for (int j = 0; j < NG; j++) {
            const float* row = Fc + k * fs01 + j * fs0;
            float rr = 0.0f;
#pragma unroll
            for (int i = 0; i < NG; i++) rr += wx[i] * row[i];
            pl += wy[j] * rr;
          }
          acc += wz[k] * pl;
        }
        Fp[c] = acc;
      }
      const float Ex = Fp[0] + g.e0[0], Ey = Fp[1] + g.e0[1], Ez = Fp[2] + g.e0[2];
      const float Bx = Fp[3] + g.b0[0], By = Fp[4] + g.b0[1], Bz = Fp[5] + g.b0[2];
      // ---- Boris push (Sec. 3.2, Eq. momentum-update)
      float ux = pu[r][0], uy = pu[r][1], uz = pu[r][2];
      const float mx = ux + h * Ex, my = uy + h * Ey, mz = uz + h * Ez;
      const float gim = rsqrtf(1.0f + mx * mx + my * my + mz * mz);
      const float tx = h * Bx * gim, ty = h * By * gim, tz = h * Bz * gim;
      const float sfac = 2.0f * __builtin_amdgcn_rcpf(1.0f + tx * tx + ty * ty + tz * tz);
      const float px = mx + (my * tz - mz * ty);
      const float py = my + (mz * tx - mx * tz);
      const float pz = mz + (mx * ty - my * tx);
      const float sx_ = sfac * tx, sy_ = sfac * ty, sz_ = sfac * tz;
      ux = mx + (py * sz_ - pz * sy_) + h * Ex;
      uy = my + (pz * sx_ - px * sz_) + h * Ey;
      uz = mz + (px * sy_ - py * sx_) + h * Ez;
      // ---- advance (Eq. 2d-position-update, all three axes)
      const float uu2 = ux * ux + uy * uy + uz * uz;
      const float gi = rsqrtf(1.0f + uu2);
      const float uu[3] = {ux, uy, uz};
      int mv[3];
      float en[3];
#pragma unroll
      for (int d = 0; d < 3; d++) {
        const float x = e[d] + g.dt * g.rdx[d] * (uu[d] * gi);
        const float f = floorf(x);
        int c = (int)f;
        float rr = x - f;
        if (rr >= 1.0f) {  // rounding edge: keep the offset in [0,1)
          rr = 0.0f;
          c += 1;
        }
        // the Courant condition keeps |move| below one cell
        if (c > 1) {
          c = 1;
          rr = 0.99999994f;
        } else if (c < -1) {
          c = -1;
          rr = 0.0f;
        }
        en[d] = rr;
        mv[d] = c;
      }
      // ---- the new state (stored after the item's interleaved slots are known)
      int nc[3], lk[3];
#pragma unroll
      for (int d = 0; d < 3; d++) {
        nc[d] = cc[d] + mv[d];
        if (nc[d] < 0) nc[d] += g.nx[d];
        if (nc[d] >= g.nx[d]) nc[d] -= g.nx[d];
        const int ln = pic_local(nc[d], org[d], ext[d], g.nx[d]);
        strayed = strayed || ln < -g.flag_slack || ln >= ext[d] + g.flag_slack;
        dd[d] = ln < 0 ? -1 : (ln >= ext[d] ? 1 : 0);
        // cell class: a particle strays at most a tile extent outside its tile
        lk[d] = ln < 0 ? ln + ext[d] : (ln >= ext[d] ? ln - ext[d] : ln);
        sen[r][d] = en[d];
      }
      sncell[r] = pic_pack(g, nc[0], nc[1], nc[2]);
      skey[r] = (lk[0] + ext[0] * (lk[1] + ext[1] * lk[2])) & 63;
      snu[r][0] = ux;
      snu[r][1] = uy;
      snu[r][2] = uz;
      // ---- what the deposit needs
      const bool moved = mv[0] != 0 || mv[1] != 0 || mv[2] != 0 || en[0] != e[0] || en[1] != e[1] || en[2] != e[2];
      if (moved) {
#pragma unroll
        for (int d = 0; d < 3; d++) se0[r][d] = e[d];
        smv[r] = (mv[0] + 1) | ((mv[1] + 1) << 2) | ((mv[2] + 1) << 4);
        sjc[r] = (jlo[2] + l[2]) * js01 + (jlo[1] + l[1]) * js0 + jlo[0] + l[0];
        swq[r] = pw[r];
        bmax = fmaxf(bmax, fabsf(pw[r]) * (sqrtf(uu2) * gi));
      }
    }
    {
      // wave-aggregated count per rebin slot (almost every particle is in slot 13)
      const int slt = live ? pic_slot(dd[0], dd[1], dd[2]) : -1;
      unsigned long long todo = __ballot(slt >= 0);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int ls = __shfl(slt, leader);
        const unsigned long long m = __ballot(slt == ls);
        if ((int)(threadIdx.x & 63) == leader) atomicAdd(&scnt[ls], (int)__popcll(m));
        todo &= ~m;
      }
    }
  }
  // the item's bound on a single contribution: max of |w| |v| over its particles
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) bmax = fmaxf(bmax, __shfl_xor(bmax, off));
  if ((tid & 63) == 0) sred[tid >> 6] = bmax;
  const int any_strayed = __syncthreads_or(strayed ? 1 : 0);  // also: phase A done, fields dead
  const int any_bad = __syncthreads_or(bad ? 1 : 0);
  float btop = 0.0f;
  for (int k = 0; k < (nthr >> 6); k++) btop = fmaxf(btop, sred[k]);
  // (the int64 mode: the instance's own fixed point, as in the one-phase kernel)
  int eg = 0;
  (void)frexpf(g.jscale, &eg);  // jscale = 2^(eg-1)
  const int e_item = __builtin_amdgcn_readfirstlane(
      kWide ? (g.acc_mode == 2 ? eg - 1 : item_exponent(btop)) : item_exponent32(btop, it.end - it.begin));
  const float Q = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(ldexpf(1.0f, e_item))));

  // 3. store the new state at the item's interleaved slots (the LDS of the
  // staged fields is free), then clear the current tile over it
  {
    int pos[R];
    interleave_slots(skey, pos, smem);
#pragma unroll
    for (int r = 0; r < R; r++) {
      if (pos[r] < 0) continue;
      const int q = it.begin + pos[r];
      cellp[q] = sncell[r];
      ep0[q] = sen[r][0];
      ep1[q] = sen[r][1];
      ep2[q] = sen[r][2];
      up0[q] = snu[r][0];
      up1[q] = snu[r][1];
      up2[q] = snu[r][2];
      wp[q] = pw[r];
      idp[q] = pid[r];
    }
  }
  for (int idx = tid; idx < 3 * jpl; idx += nthr) sJ[idx] = (Acc)0;
  if (tid == 0) {
    if (any_strayed) S.ctl->flag = 1;
    if (any_bad) S.ctl->bad = 1;
  }
  if (tid < PIC_NSLOT) S.cnt[ii * PIC_NSLOT + tid] = scnt[tid];
  __syncthreads();

  // 4. phase B: ISIS ordering average in Esirkepov's closed form, core of the
  // old support unconditional, each extra block under one branch
  const int st[3] = {1, js0, js01};
#pragma unroll
  for (int r = 0; r < R; r++) {
    if (sjc[r] < 0) continue;
    const int mv[3] = {(smv[r] & 3) - 1, ((smv[r] >> 2) & 3) - 1, ((smv[r] >> 4) & 3) - 1};
    int wb[3], p0[3];
    bool wide[3];
    float S0[3][W], D[3][W];
#pragma unroll
    for (int d = 0; d < 3; d++) deposit_shape<ORDER>(se0[r][d], sen[r][d], mv[d], wb[d], p0[d], wide[d], S0[d], D[d]);
    DepAxis<K> ax[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const float qd = -swq[r] * g.cdt[d] * Q;
      float P[W - 1];
      float a = 0.0f;
#pragma unroll
      for (int k = 0; k < W - 1; k++) {
        a += D[d][k];
        P[k] = qd * a;
      }
      const bool pd = p0[d] != 0;
#pragma unroll
      for (int k = 0; k < K; k++) {
        const float sk = pd ? S0[d][k + 1] : S0[d][k], dk = pd ? D[d][k + 1] : D[d][k];
        ax[d].H[k] = fmaf(0.5f, dk, sk);
        ax[d].G[k] = 0.28867513f * dk;  // 1/sqrt(12)
      }
#pragma unroll
      for (int k = 0; k < K - 1; k++) ax[d].P[k] = pd ? P[k + 1] : P[k];
      {
        const float se = pd ? S0[d][0] : S0[d][K], de = pd ? D[d][0] : D[d][K];
        ax[d].He = fmaf(0.5f, de, se);
        ax[d].Ge = 0.28867513f * de;
      }
      ax[d].Pe = wide[d] ? (pd ? P[0] : P[K - 1]) : 0.0f;
      ax[d].oS = pd ? -1 : K;
      ax[d].oP = pd ? -1 : K - 1;
      ax[d].wide = wide[d];
    }
    const int cb = sjc[r] + (wb[0] + p0[0]) + (wb[1] + p0[1]) * st[1] + (wb[2] + p0[2]) * st[2];
    dep3_comp<K, 0>(sJ, cb, st, ax);
    dep3_comp<K, 1>(sJ + jpl, cb, st, ax);
    dep3_comp<K, 2>(sJ + 2 * jpl, cb, st, ax);
  }
  __syncthreads();

  // 5. fold the tile into the global current (periodic wrap); the int64 mode
  // sums in the instance's own fixed point, so its global sums stay order-free
  const float qinv = ldexpf(1.0f, -e_item);
  BoxWalk bj(tid, nthr, JR);
  for (int idx = tid; idx < jn; idx += nthr, bj.advance(JR)) {
    const int gx = wrap_fast(org[0] - jlo[0] + bj.x, g.nx[0]);
    const int gy = wrap_fast(org[1] - jlo[1] + bj.y, g.nx[1]);
    const int gz = wrap_fast(org[2] - jlo[2] + bj.z, g.nx[2]);
    const int gidx = gx + g.nx[0] * (gy + g.nx[1] * gz);
    const int lj = bj.x + bj.y * js0 + bj.z * js01;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      if constexpr (kWide) {
        const long long q = (long long)sJ[c * jpl + lj];
        if (q != 0) {
          if (g.acc_mode == 2) {
            atomicAdd(S.J64[jp] + (size_t)c * ncell + gidx, (acc_t)q);
          } else {
            __builtin_amdgcn_global_atomic_fadd_f32((gfloat*)S.Jacc[jp] + (size_t)c * ncell + gidx,
                                                    item_sum_f32(q, qinv));
          }
        }
      } else {
        // one rounding, as for the int64 sums
        const int q = (int)sJ[c * jpl + lj];
        if (q != 0)
          __builtin_amdgcn_global_atomic_fadd_f32((gfloat*)S.Jacc[jp] + (size_t)c * ncell + gidx, (float)q * qinv);
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// periodic 2D work item in two phases
// ---------------------------------------------------------------------------
//
// The 2D counterpart of process_item3, for periodic Cartesian instances with
// Esirkepov's deposit and FP32 accumulation: phase A stages E and B and
// pushes every particle of the item (up to kSplitR2 per thread), keeping
// what the deposit needs in registers; phase B deposits into a 32-bit
// current tile in the same LDS, in the item's own fixed point
// (item_exponent32: a contribution to one node is at most |w| |v|, the
// out-of-plane one |w v_3| times a shape average at most one).  Fields and
// current never coexist, so a workgroup needs the larger region, not their
// sum, and no per-store unit has to be prepared before the launch.
constexpr int kSplitR2 = 4;  // particles per thread per 2D work item

template <int ORDER>
__device__ void process_item2(const StoreDesc& S, int cur, const Item it, int ii, int jp, int kstep, float* smem,
                              int* scnt, float* sred) {
  constexpr int NG = ORDER + 1;  // gather taps per axis
  constexpr int W = ORDER + 2;   // deposit window per axis
  constexpr int K = ORDER + 1;   // deposit core per axis
  constexpr int R = kSplitR2;
  const GridDesc& g = S.g;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;

  const int set = cur;
  gint* __restrict__ cellp = (gint*)S.cell[set];
  gfloat* __restrict__ ep0 = (gfloat*)S.eps[set][0];
  gfloat* __restrict__ ep1 = (gfloat*)S.eps[set][1];
  gfloat* __restrict__ up0 = (gfloat*)S.u[set][0];
  gfloat* __restrict__ up1 = (gfloat*)S.u[set][1];
  gfloat* __restrict__ up2 = (gfloat*)S.u[set][2];
  const gfloat* __restrict__ wp = (const gfloat*)S.w[set];

  int tc[3];
  pic_tile_coords(g, it.tile, tc);
  // stray bound of this step (as in the one-phase kernel)
  const int s0 = __builtin_amdgcn_readfirstlane(S.ctl->sorted) ? 0 : g.flag_slack;
  int sl[2], org[2], ext[2], flo[2], jlo[2];
  int FR[3] = {1, 1, 1}, JR[3] = {1, 1, 1};
#pragma unroll
  for (int d = 0; d < 2; d++) {
    sl[d] = __builtin_amdgcn_readfirstlane(min(s0 + (int)ceilf((float)kstep * g.vstep[d]), g.slk[d]));
    org[d] = tc[d] * g.tile[d];
    ext[d] = min(g.tile[d], g.nx[d] - org[d]);
    flo[d] = sl[d] + g.fa;
    jlo[d] = sl[d] + g.ja;
    FR[d] = ext[d] + 2 * sl[d] + g.fa + g.fb;
    JR[d] = ext[d] + 2 * sl[d] + g.ja + g.jb;
  }
  const int fn = FR[0] * FR[1];
  const int jn = JR[0] * JR[1];
  float* sF = smem;                // phase A: [6][fn]
  unsigned* sJ = (unsigned*)smem;  // phase B: [3][jn]

  // this thread's particles: requested before the fields are staged
  int pc[R];
  float pe[R][2], pu[R][3], pw[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int p = it.begin + tid + r * nthr;
    pc[r] = -1;
    pe[r][0] = pe[r][1] = 0.0f;
    pu[r][0] = pu[r][1] = pu[r][2] = 0.0f;
    pw[r] = 0.0f;
    if (p < it.end) {
      pc[r] = cellp[p];
      pe[r][0] = ep0[p];
      pe[r][1] = ep1[p];
      pu[r][0] = up0[p];
      pu[r][1] = up1[p];
      pu[r][2] = up2[p];
      pw[r] = wp[p];
    }
  }

  // 1. stage E, B with periodic wrap: four nodes per thread per batch, every
  // load of a batch in flight before its LDS writes
  const int ncell = g.ncell;
  {
    const gfloat* Fg = (const gfloat*)S.F[jp];
    BoxWalk bw(tid, nthr, FR);
    for (int base = 0; base < fn; base += 4 * nthr) {
      float v[4][6];
      int gi[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int gx = wrap_fast(org[0] - flo[0] + bw.x, g.nx[0]);
        const int gy = wrap_fast(org[1] - flo[1] + bw.y, g.nx[1]);
        gi[q] = gx + g.nx[0] * gy;
        bw.advance(FR);
      }
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (base + q * nthr + tid < fn) {
#pragma unroll
          for (int c = 0; c < 6; c++) v[q][c] = Fg[(size_t)c * ncell + gi[q]];
        }
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int li = base + q * nthr + tid;
        if (li < fn) {
#pragma unroll
          for (int c = 0; c < 6; c++) sF[c * fn + li] = v[q][c];
        }
      }
    }
  }
  if (tid < PIC_NSLOT) scnt[tid] = 0;
  __syncthreads();

  // 2. phase A: gather, Boris push, advance; store the new state
  const float h = 0.5f * S.qm * g.dt;
  bool strayed = false, bad = false;
  float bmax = 0.0f;
  // kept for the deposit: old and new offsets, the move, the old cell in
  // current-region coordinates (-1: no particle), the weight and w v_3
  float se0[R][2], sen[R][2], swq[R], sv3[R];
  int smv[R], sjc[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int p = it.begin + tid + r * nthr;
    smv[r] = 0;
    sjc[r] = -1;
    swq[r] = sv3[r] = 0.0f;
    se0[r][0] = se0[r][1] = sen[r][0] = sen[r][1] = 0.0f;
    int dd[2] = {0, 0};
    const bool live = p < it.end;
    if (live) {
      int cc[3];
      pic_unpack(g, pc[r], cc);
      int l[2];
      bool ok = true;
#pragma unroll
      for (int d = 0; d < 2; d++) {
        l[d] = pic_local(cc[d], org[d], ext[d], g.nx[d]);
        ok = ok && (l[d] >= -sl[d]) && (l[d] < ext[d] + sl[d]);
      }
      if (!ok) {
        // reported as a failed step; the particle is clamped into the
        // staged region so that every access stays inside it
        bad = true;
#pragma unroll
        for (int d = 0; d < 2; d++) l[d] = min(max(l[d], -sl[d]), ext[d] + sl[d] - 1);
      }
      const float e[2] = {pe[r][0], pe[r][1]};
      // ---- gather: weights at offset 0 and 1/2 per axis
      int b0[2], bh[2];
      float w0[2][NG], wh[2][NG];
#pragma unroll
      for (int d = 0; d < 2; d++) {
        gather_weights<ORDER>(e[d], false, b0[d], w0[d]);
        gather_weights<ORDER>(e[d], true, bh[d], wh[d]);
      }
      const int FR0 = FR[0];
      const int gb0 = (flo[1] + l[1] + b0[1]) * FR0 + flo[0] + l[0] + b0[0];
      const int dgx = bh[0] - b0[0];
      const int dgy = bh[1] == b0[1] ? 0 : (bh[1] < b0[1] ? -FR0 : FR0);
      float Fp[6];
#pragma unroll
      for (int c = 0; c < 6; c++) {
        // component c: E_c staggered half along axis c, B_c half along the others
        const bool hx = (c < 3) ? (c == 0) : (c != 3);
        const bool hy = (c < 3) ? (c == 1) : (c != 4);
        const float* wx = hx ? wh[0] : w0[0];
        const float* wy = hy ? wh[1] : w0[1];
        const float* row = sF + c * fn + gb0 + (hx ? dgx : 0) + (hy ? dgy : 0);
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < NG; j++) {
          float rr = 0.0f;
#pragma unroll
          for (int i = 0; i < NG; i++) rr += wx[i] * row[i];
          acc += wy[j] * rr;
          row += FR0;
        }
        Fp[c] = acc;
      }
      const float Ex = Fp[0] + g.e0[0], Ey = Fp[1] + g.e0[1], Ez = Fp[2] + g.e0[2];
      const float Bx = Fp[3] + g.b0[0], By = Fp[4] + g.b0[1], Bz = Fp[5] + g.b0[2];
      // ---- Boris push (Sec. 3.2, Eq. momentum-update)
      float ux = pu[r][0], uy = pu[r][1], uz = pu[r][2];
      const float mx = ux + h * Ex, my = uy + h * Ey, mz = uz + h * Ez;
      const float gim = rsqrtf(1.0f + mx * mx + my * my + mz * mz);
      const float tx = h * Bx * gim, ty = h * By * gim, tz = h * Bz * gim;
      const float sfac = 2.0f * __builtin_amdgcn_rcpf(1.0f + tx * tx + ty * ty + tz * tz);
      const float px = mx + (my * tz - mz * ty);
      const float py = my + (mz * tx - mx * tz);
      const float pz = mz + (mx * ty - my * tx);
      const float sx_ = sfac * tx, sy_ = sfac * ty, sz_ = sfac * tz;
      ux = mx + (py * sz_ - pz * sy_) + h * Ex;
      uy = my + (pz * sx_ - px * sz_) + h * Ey;
      uz = mz + (px * sy_ - py * sx_) + h * Ez;
      // ---- advance (Eq. 2d-position-update, in-plane)
      const float uu2 = ux * ux + uy * uy + uz * uz;
      const float gi = rsqrtf(1.0f + uu2);
      const float uu[2] = {ux, uy};
      int mv[2];
      float en[2];
#pragma unroll
      for (int d = 0; d < 2; d++) {
        const float x = e[d] + g.dt * g.rdx[d] * (uu[d] * gi);
        const float f = floorf(x);
        int c = (int)f;
        float rr = x - f;
        if (rr >= 1.0f) {  // rounding edge: keep the offset in [0,1)
          rr = 0.0f;
          c += 1;
        }
        // the Courant condition keeps |move| below one cell
        if (c > 1) {
          c = 1;
          rr = 0.99999994f;
        } else if (c < -1) {
          c = -1;
          rr = 0.0f;
        }
        en[d] = rr;
        mv[d] = c;
      }
      // ---- the new state
      int nc[2];
#pragma unroll
      for (int d = 0; d < 2; d++) {
        nc[d] = cc[d] + mv[d];
        if (nc[d] < 0) nc[d] += g.nx[d];
        if (nc[d] >= g.nx[d]) nc[d] -= g.nx[d];
        const int ln = pic_local(nc[d], org[d], ext[d], g.nx[d]);
        strayed = strayed || ln < -g.flag_slack || ln >= ext[d] + g.flag_slack;
        dd[d] = ln < 0 ? -1 : (ln >= ext[d] ? 1 : 0);
      }
      cellp[p] = pic_pack(g, nc[0], nc[1], 0);
      ep0[p] = en[0];
      ep1[p] = en[1];
      up0[p] = ux;
      up1[p] = uy;
      up2[p] = uz;
      // ---- what the deposit needs
#pragma unroll
      for (int d = 0; d < 2; d++) {
        se0[r][d] = e[d];
        sen[r][d] = en[d];
      }
      smv[r] = (mv[0] + 1) | ((mv[1] + 1) << 2);
      sjc[r] = (jlo[1] + l[1]) * JR[0] + jlo[0] + l[0];
      swq[r] = pw[r];
      sv3[r] = pw[r] * uz * gi;
      bmax = fmaxf(bmax, fabsf(pw[r]) * (sqrtf(uu2) * gi));
    }
    {
      // wave-aggregated count per rebin slot (almost every particle is in slot 13)
      const int slt = live ? pic_slot(dd[0], dd[1], 0) : -1;
      unsigned long long todo = __ballot(slt >= 0);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int ls = __shfl(slt, leader);
        const unsigned long long m = __ballot(slt == ls);
        if ((int)(threadIdx.x & 63) == leader) atomicAdd(&scnt[ls], (int)__popcll(m));
        todo &= ~m;
      }
    }
  }
  // the item's bound on a single contribution: max of |w| |v| over its particles
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) bmax = fmaxf(bmax, __shfl_xor(bmax, off));
  if ((tid & 63) == 0) sred[tid >> 6] = bmax;
  const int any_strayed = __syncthreads_or(strayed ? 1 : 0);  // also: phase A done, fields dead
  const int any_bad = __syncthreads_or(bad ? 1 : 0);
  float btop = 0.0f;
  for (int k = 0; k < (nthr >> 6); k++) btop = fmaxf(btop, sred[k]);
  const int e_item = __builtin_amdgcn_readfirstlane(item_exponent32(btop, it.end - it.begin));
  const float Q = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(ldexpf(1.0f, e_item))));

  // 3. clear the current tile over the dead field tile
  for (int idx = tid; idx < 3 * jn; idx += nthr) sJ[idx] = 0u;
  if (tid == 0) {
    if (any_strayed) S.ctl->flag = 1;
    if (any_bad) S.ctl->bad = 1;
  }
  if (tid < PIC_NSLOT) S.cnt[ii * PIC_NSLOT + tid] = scnt[tid];
  __syncthreads();

  // 4. phase B: ISIS ordering average in Esirkepov's closed form (2D3V): the
  // core of the old support unconditional, the extra column, row and corner
  // under one branch each; J3 skipped by lanes without out-of-plane motion
  unsigned* J1 = sJ;
  unsigned* J2 = sJ + jn;
  unsigned* J3 = sJ + 2 * jn;
  const int RJ = JR[0];
#pragma unroll
  for (int r = 0; r < R; r++) {
    if (sjc[r] < 0) continue;
    const int mv[2] = {(smv[r] & 3) - 1, ((smv[r] >> 2) & 3) - 1};
    int wb[2], p0[2];
    bool wide[2];
    float S0[2][W], D[2][W];
#pragma unroll
    for (int d = 0; d < 2; d++) deposit_shape<ORDER>(se0[r][d], sen[r][d], mv[d], wb[d], p0[d], wide[d], S0[d], D[d]);
    const float q1 = -swq[r] * g.cdt[0] * Q, q2 = -swq[r] * g.cdt[1] * Q;
    float P1[W - 1], P2[W - 1];
    {
      float a = 0.0f, b = 0.0f;
#pragma unroll
      for (int k = 0; k < W - 1; k++) {
        a += D[0][k];
        b += D[1][k];
        P1[k] = q1 * a;
        P2[k] = q2 * b;
      }
    }
    const float v3 = sv3[r] * Q;
    const bool px = p0[0] != 0, py = p0[1] != 0;
    float Sx[K], Dx[K], Sy[K], Dy[K], Px[K - 1], Py[K - 1];
#pragma unroll
    for (int k = 0; k < K; k++) {
      Sx[k] = px ? S0[0][k + 1] : S0[0][k];
      Dx[k] = px ? D[0][k + 1] : D[0][k];
      Sy[k] = py ? S0[1][k + 1] : S0[1][k];
      Dy[k] = py ? D[1][k + 1] : D[1][k];
    }
#pragma unroll
    for (int k = 0; k < K - 1; k++) {
      Px[k] = px ? P1[k + 1] : P1[k];
      Py[k] = py ? P2[k + 1] : P2[k];
    }
    const float Sxe = px ? S0[0][0] : S0[0][K], Dxe = px ? D[0][0] : D[0][K];
    const float Sye = py ? S0[1][0] : S0[1][K], Dye = py ? D[1][0] : D[1][K];
    const float Pxe = wide[0] ? (px ? P1[0] : P1[K - 1]) : 0.0f;
    const float Pye = wide[1] ? (py ? P2[0] : P2[K - 1]) : 0.0f;
    const int exS = px ? -1 : K, exP = px ? -1 : K - 1;
    const int cb = sjc[r] + (wb[0] + p0[0]) + (wb[1] + p0[1]) * RJ;
    const int ey = py ? -RJ : K * RJ;
    const int eyp = py ? -RJ : (K - 1) * RJ;
    // y factors of J1 and J3 (S0 + D/2, S0/2 + D/3) and x factor of J2
    float T1[K], U2[K], X2[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
      T1[k] = Sy[k] + 0.5f * Dy[k];
      U2[k] = 0.5f * Sy[k] + (1.0f / 3.0f) * Dy[k];
      X2[k] = Sx[k] + 0.5f * Dx[k];
    }
    const float T1e = Sye + 0.5f * Dye, U2e = 0.5f * Sye + (1.0f / 3.0f) * Dye;
    const float X2e = Sxe + 0.5f * Dxe;
#pragma unroll
    for (int j = 0; j < K; j++) {
#pragma unroll
      for (int i = 0; i < K - 1; i++) lds_add_any(J1 + cb + j * RJ + i, Px[i] * T1[j]);
      if (v3 != 0.0f) {
#pragma unroll
        for (int i = 0; i < K; i++) lds_add_any(J3 + cb + j * RJ + i, v3 * (Sx[i] * T1[j] + Dx[i] * U2[j]));
      }
    }
#pragma unroll
    for (int j = 0; j < K - 1; j++) {
#pragma unroll
      for (int i = 0; i < K; i++) lds_add_any(J2 + cb + j * RJ + i, Py[j] * X2[i]);
    }
    if (wide[0]) {
#pragma unroll
      for (int j = 0; j < K; j++) {
        lds_add_any(J1 + cb + j * RJ + exP, Pxe * T1[j]);
        if (v3 != 0.0f) lds_add_any(J3 + cb + j * RJ + exS, v3 * (Sxe * T1[j] + Dxe * U2[j]));
      }
#pragma unroll
      for (int j = 0; j < K - 1; j++) lds_add_any(J2 + cb + j * RJ + exS, Py[j] * X2e);
    }
    if (wide[1]) {
#pragma unroll
      for (int i = 0; i < K - 1; i++) lds_add_any(J1 + cb + ey + i, Px[i] * T1e);
#pragma unroll
      for (int i = 0; i < K; i++) {
        if (v3 != 0.0f) lds_add_any(J3 + cb + ey + i, v3 * (Sx[i] * T1e + Dx[i] * U2e));
        lds_add_any(J2 + cb + eyp + i, Pye * X2[i]);
      }
    }
    if (wide[0] && wide[1]) {
      lds_add_any(J1 + cb + ey + exP, Pxe * T1e);
      if (v3 != 0.0f) lds_add_any(J3 + cb + ey + exS, v3 * (Sxe * T1e + Dxe * U2e));
      lds_add_any(J2 + cb + eyp + exS, Pye * X2e);
    }
  }
  __syncthreads();

  // 5. fold the tile into the global current (periodic wrap), one rounding
  // of each node's sum
  const float qinv = ldexpf(1.0f, -e_item);
  BoxWalk bj(tid, nthr, JR);
  for (int idx = tid; idx < jn; idx += nthr, bj.advance(JR)) {
    const int gx = wrap_fast(org[0] - jlo[0] + bj.x, g.nx[0]);
    const int gy = wrap_fast(org[1] - jlo[1] + bj.y, g.nx[1]);
    const int gidx = gx + g.nx[0] * gy;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const int q = (int)sJ[c * jn + idx];
      if (q != 0)
        __builtin_amdgcn_global_atomic_fadd_f32((gfloat*)S.Jacc[jp] + (size_t)c * ncell + gidx, (float)q * qinv);
    }
  }
  __syncthreads();
}

template <int DIM, int ORDER, int MODE>
__device__ __forceinline__ void gpd_body(const StoreDesc* __restrict__ stores, int nstores, int jp, int kstep) {
  // 16-byte aligned: the int64 current tile inside it takes 8-byte LDS atomics
  extern __shared__ __align__(16) float smem[];
  __shared__ int s_pref[kMaxGroup + 1];
  __shared__ int s_cur[kMaxGroup];
  __shared__ int s_cnt[PIC_NSLOT];
  __shared__ float s_red[kBlock / 64];
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int s = 0; s < nstores; s++) {
      int cur = pic_cur(*stores[s].ctl);
      s_cur[s] = cur;
      s_pref[s] = acc;
      acc += stores[s].ctl->n_items[cur];
    }
    s_pref[nstores] = acc;
  }
  __syncthreads();
  const int total = s_pref[nstores];
  // Items are listed in tile order.  Workgroup b runs on XCD b % 8 (the
  // dispatcher deals workgroups to the eight XCDs in turn), so a plain
  // grid-stride walk would scatter neighbouring tiles, whose staged halos
  // overlap, over eight separate L2 caches.  With a grid that is a multiple
  // of 8, the workgroups of each XCD walk one contiguous eighth of the list
  // (two-phase 3D kernel only; the 2D kernels keep the plain walk).
  int lo = 0, hi = total, first = blockIdx.x, stride = gridDim.x;
  if (MODE >= 4 && (gridDim.x & 7) == 0 && total >= (int)gridDim.x) {
    const int per = (total + 7) >> 3;
    lo = min(total, (int)(blockIdx.x & 7) * per);
    hi = min(total, lo + per);
    first = lo + (int)(blockIdx.x >> 3);
    stride = gridDim.x >> 3;
  }
  int s = 0;
  for (int gi = first; gi < hi; gi += stride) {
    while (gi >= s_pref[s + 1]) s++;
    // the store, its buffer set and the item are the workgroup's own: read
    // into scalar registers, so the descriptor's fields load as scalars
    s = __builtin_amdgcn_readfirstlane(s);
    const StoreDesc& S = stores[s];
    const int cur = __builtin_amdgcn_readfirstlane(s_cur[s]);
    const int ii = __builtin_amdgcn_readfirstlane(gi - s_pref[s]);
    Item it = S.items[cur][ii];
    it.tile = __builtin_amdgcn_readfirstlane(it.tile);
    it.begin = __builtin_amdgcn_readfirstlane(it.begin);
    it.end = __builtin_amdgcn_readfirstlane(it.end);
    if constexpr (MODE == 7)
      process_item2<ORDER>(S, cur, it, ii, jp, kstep, smem, s_cnt, s_red);
    else if constexpr (MODE >= 4)
      process_item3<ORDER, MODE == 5, typename std::conditional<MODE == 4, acc_t, unsigned>::type>(
          S, cur, it, ii, jp, kstep, smem, s_cnt, s_red);
    else
      process_item<DIM, ORDER, MODE>(S, cur, it, ii, jp, kstep, smem, s_cnt);
  }
  (void)lo;
}

// The periodic 2D kernels of orders 1 and 2 are held to the registers of
// five waves per SIMD (96 VGPRs, no spills): where the LDS of a tile allows
// five workgroups per CU this is up to 8 % faster (16x8 tiles, the batched
// parameter scan); where LDS allows only four (32x8 tiles late in a sort
// cycle) it changes nothing.  The two-phase 3D kernels are held to four
// waves (128 VGPRs; their LDS allows four workgroups of 4x4x4 tiles), except
// the cubic one with runtime strides, which would spill there and takes
// three.  The other variants would spill; they keep the compiler's choice.
template <int DIM, int ORDER, int MODE>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(DIM == 2 && ORDER <= 2 && MODE == 0 ? 5 : (MODE == 4 && ORDER == 3 ? 3 : (MODE >= 4 ? 4 : 1))))) gpd_kernel(const StoreDesc* __restrict__ stores, int nstores, int jp,
                                                     int kstep) {
  gpd_body<DIM, ORDER, MODE>(stores, nstores, jp, kstep);
}

template <int DIM, int ORDER, int MODE>
const void* gpd_entry() {
  return (const void*)gpd_kernel<DIM, ORDER, MODE>;
}

template <int DIM, int ORDER, int MODE>
hipError_t prepare_mode(size_t lds) {
  return hipFuncSetAttribute(gpd_entry<DIM, ORDER, MODE>(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int DIM, int ORDER, int MODE>
void launch_mode(const StoreDesc* stores, int nstores, int grid, size_t lds, int jp, int kstep, hipStream_t st,
                 hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0 || ev1)
    // the command processor stamps the events at the kernel's own start and end
    hipExtLaunchKernelGGL(gpd_kernel<DIM, ORDER, MODE>, dim3(grid), dim3(kBlock), (std::uint32_t)lds, st, ev0, ev1, 0,
                          stores, nstores, jp, kstep);
  else
    gpd_kernel<DIM, ORDER, MODE><<<dim3(grid), dim3(kBlock), lds, st>>>(stores, nstores, jp, kstep);
}

template <int DIM, int ORDER>
hipError_t prepare_one(int mode, size_t lds) {
  if (mode == 1) return prepare_mode<DIM, ORDER, 1>(lds);
  if constexpr (DIM == 2) {
    if (mode == 2) return prepare_mode<DIM, ORDER, 2>(lds);
    if (mode == 3) return prepare_mode<DIM, ORDER, 3>(lds);
    if (mode == 7) return prepare_mode<DIM, ORDER, 7>(lds);
  } else {
    if (mode == 4) return prepare_mode<DIM, ORDER, 4>(lds);
    if (mode == 5) return prepare_mode<DIM, ORDER, 5>(lds);
    if (mode == 6) return prepare_mode<DIM, ORDER, 6>(lds);
  }
  if (mode == 0) return prepare_mode<DIM, ORDER, 0>(lds);
  return hipErrorInvalidValue;
}

template <int DIM, int ORDER>
hipError_t launch_one(int mode, const StoreDesc* stores, int nstores, int grid, size_t lds, int jp, int kstep,
                      hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (mode == 1)
    launch_mode<DIM, ORDER, 1>(stores, nstores, grid, lds, jp, kstep, st, ev0, ev1);
  else if (mode == 0)
    launch_mode<DIM, ORDER, 0>(stores, nstores, grid, lds, jp, kstep, st, ev0, ev1);
  else if constexpr (DIM == 2) {
    if (mode == 2)
      launch_mode<DIM, ORDER, 2>(stores, nstores, grid, lds, jp, kstep, st, ev0, ev1);
    else if (mode == 3)
      launch_mode<DIM, ORDER, 3>(stores, nstores, grid, lds, jp, kstep, st, ev0, ev1);
    else if (mode == 7)
      launch_mode<DIM, ORDER, 7>(stores, nstores, grid, lds, jp, kstep, st, ev0, ev1);
    else
      return hipErrorInvalidValue;
  } else {
    if (mode == 4)
      launch_mode<DIM, ORDER, 4>(stores, nstores, grid, lds, jp, kstep, st, ev0, ev1);
    else if (mode == 5)
      launch_mode<DIM, ORDER, 5>(stores, nstores, grid, lds, jp, kstep, st, ev0, ev1);
    else if (mode == 6)
      launch_mode<DIM, ORDER, 6>(stores, nstores, grid, lds, jp, kstep, st, ev0, ev1);
    else
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

// LDS bytes one workgroup of the fused kernel needs for a grid.
// Padded LDS strides of the two-phase kernel's regions.  The lanes of a
// wavefront hold one particle of each of 64 consecutive cells of the tile
// (the binning interleaves the cells, x fastest), and every lane of an LDS
// instruction reads or adds at the same offset from its own cell, so the
// banks the lanes hit are set by the row and plane strides.  Among strides
// up to 8 nodes above the region's extents, take the one whose 64 addresses
// spread best over 64 four-byte banks (field reads) or over 32 eight-byte
// bank pairs per half-wave (int64 current adds), then the smallest plane.
static void split_stride_pick(const GridDesc& g, int ex, int ey, bool wide8, int& s0, int& s01) {
  int lx[64], ly[64], lz[64];
  const int vol = g.tile[0] * g.tile[1] * g.tile[2];
  for (int c = 0; c < 64; c++) {
    const int k = c % vol;
    lx[c] = k % g.tile[0];
    ly[c] = (k / g.tile[0]) % g.tile[1];
    lz[c] = k / (g.tile[0] * g.tile[1]);
  }
  int best = 1 << 30;
  s0 = ex;
  s01 = ex * ey;
  for (int a = ex; a < ex + 8; a++)
    for (int b = ey; b < ey + 8; b++) {
      int cost = 0;
      for (int h = 0; h < (wide8 ? 2 : 1); h++) {
        int cnt[64] = {0};
        const int n = wide8 ? 32 : 64, m = wide8 ? 32 : 64;
        for (int c = h * n; c < h * n + n; c++) {
          const int addr = lx[c] + ly[c] * a + lz[c] * a * b;
          cost = std::max(cost, ++cnt[addr % m]);
        }
      }
      const int key = cost * (1 << 20) + a * b;
      if (key < best) {
        best = key;
        s0 = a;
        s01 = a * b;
      }
    }
}

void pic_gpd_split_strides(GridDesc& g) {
  split_stride_pick(g, g.tile[0] + 2 * g.slk[0] + g.fa + g.fb, g.tile[1] + 2 * g.slk[1] + g.fa + g.fb, false, g.fs0,
                    g.fs01);
  split_stride_pick(g, g.tile[0] + 2 * g.slk[0] + g.ja + g.jb, g.tile[1] + 2 * g.slk[1] + g.ja + g.jb, true, g.js0,
                    g.js01);
}

// LDS of the two-phase kernel: six field planes or three current planes
// (int64 for the deterministic accumulation, else 32-bit) over the padded
// strides of the largest region of a sort cycle.
static size_t split_lds_bytes(const GridDesc& g0) {
  GridDesc g = g0;
  pic_gpd_split_strides(g);
  const size_t f2 = (size_t)(g.tile[2] + 2 * g.slk[2] + g.fa + g.fb);
  const size_t j2 = (size_t)(g.tile[2] + 2 * g.slk[2] + g.ja + g.jb);
  const size_t jw = g.acc_mode == 2 ? sizeof(unsigned long long) : sizeof(unsigned);  // 2: int64 accumulation
  return std::max(std::max(6 * (size_t)g.fs01 * f2 * sizeof(float), 3 * (size_t)g.js01 * j2 * jw), kInterleaveLds);
}

// Whether the two-phase periodic 2D kernel (mode 7) runs a grid (the host
// decides at set-up; see setup_grid).
bool pic_gpd_two_phase2(const GridDesc& g) { return g.tp2 != 0; }

// Its LDS: six field planes or three 32-bit current planes, whichever is larger.
static size_t two_phase2_lds_bytes(size_t fn, size_t jn) {
  return std::max(6 * fn, 3 * jn) * sizeof(float);
}

size_t pic_gpd_lds_bytes(const GridDesc& g) {
  size_t fn = 1, jn = 1;
  for (int d = 0; d < g.dim; d++) {
    fn *= (size_t)(g.tile[d] + 2 * g.slk[d] + g.fa + g.fb);
    jn *= (size_t)(g.tile[d] + 2 * g.slk[d] + g.ja + g.jb);
  }
  if (pic_gpd_split(g)) return split_lds_bytes(g);
  if (pic_gpd_two_phase2(g)) return two_phase2_lds_bytes(fn, jn);
  return ((6 * fn + 1) & ~(size_t)1) * sizeof(float) + 3 * jn * sizeof(unsigned long long);
}

// LDS the step kstep of a sort cycle needs: its stray bound with the largest
// base the kernel can read (flag_slack, after a check that did not re-sort),
// computed with the same float arithmetic as the kernel's.
size_t pic_gpd_lds_bytes_step(const GridDesc& g, int kstep) {
  size_t fn = 1, jn = 1;
  for (int d = 0; d < g.dim; d++) {
    const int sl = min(g.flag_slack + (int)ceilf((float)kstep * g.vstep[d]), g.slk[d]);
    fn *= (size_t)(g.tile[d] + 2 * sl + g.fa + g.fb);
    jn *= (size_t)(g.tile[d] + 2 * sl + g.ja + g.jb);
  }
  if (pic_gpd_split(g)) return split_lds_bytes(g);
  if (pic_gpd_two_phase2(g)) return two_phase2_lds_bytes(fn, jn);
  return ((6 * fn + 1) & ~(size_t)1) * sizeof(float) + 3 * jn * sizeof(unsigned long long);
}

// Particles one work item of the two-phase 3D kernel can hold.
int pic_gpd_split_chunk() { return kSplitR * kBlock; }

// Particles one work item of the two-phase 2D kernel can hold.
int pic_gpd_two_phase2_chunk() { return kSplitR2 * kBlock; }

int pic_gpd_block() { return kBlock; }
int pic_gpd_max_group() { return kMaxGroup; }

hipError_t pic_gpd_prepare(int dim, int order, int mode, size_t lds) {
  if (dim == 2) {
    if (order == 1) return prepare_one<2, 1>(mode, lds);
    if (order == 2) return prepare_one<2, 2>(mode, lds);
    if (order == 3) return prepare_one<2, 3>(mode, lds);
  } else if (dim == 3) {
    if (order == 1) return prepare_one<3, 1>(mode, lds);
    if (order == 2) return prepare_one<3, 2>(mode, lds);
    if (order == 3) return prepare_one<3, 3>(mode, lds);
  }
  return hipErrorInvalidValue;
}

template <int DIM, int ORDER>
int resident_one(int mode, size_t lds) {
  int n = 0;
  const void* f = mode == 1 ? gpd_entry<DIM, ORDER, 1>() : gpd_entry<DIM, ORDER, 0>();
  if constexpr (DIM == 2) {
    if (mode == 2) f = gpd_entry<DIM, ORDER, 2>();
    if (mode == 3) f = gpd_entry<DIM, ORDER, 3>();
    if (mode == 7) f = gpd_entry<DIM, ORDER, 7>();
  } else {
    if (mode == 4) f = gpd_entry<DIM, ORDER, 4>();
    if (mode == 5) f = gpd_entry<DIM, ORDER, 5>();
    if (mode == 6) f = gpd_entry<DIM, ORDER, 6>();
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlock, lds) != hipSuccess) return 1;
  return n < 1 ? 1 : n;
}

int pic_gpd_resident(int dim, int order, int mode, size_t lds) {
  if (dim == 2) {
    if (order == 1) return resident_one<2, 1>(mode, lds);
    if (order == 2) return resident_one<2, 2>(mode, lds);
    if (order == 3) return resident_one<2, 3>(mode, lds);
  } else if (dim == 3) {
    if (order == 1) return resident_one<3, 1>(mode, lds);
    if (order == 2) return resident_one<3, 2>(mode, lds);
    if (order == 3) return resident_one<3, 3>(mode, lds);
  }
  return 1;
}

hipError_t pic_launch_gpd(int dim, int order, int mode, const StoreDesc* d_stores, int nstores, int grid,
                          size_t lds, int parity, int kstep, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (dim == 2) {
    if (order == 1) return launch_one<2, 1>(mode, d_stores, nstores, grid, lds, parity, kstep, st, ev0, ev1);
    if (order == 2) return launch_one<2, 2>(mode, d_stores, nstores, grid, lds, parity, kstep, st, ev0, ev1);
    if (order == 3) return launch_one<2, 3>(mode, d_stores, nstores, grid, lds, parity, kstep, st, ev0, ev1);
  } else if (dim == 3) {
    if (order == 1) return launch_one<3, 1>(mode, d_stores, nstores, grid, lds, parity, kstep, st, ev0, ev1);
    if (order == 2) return launch_one<3, 2>(mode, d_stores, nstores, grid, lds, parity, kstep, st, ev0, ev1);
    if (order == 3) return launch_one<3, 3>(mode, d_stores, nstores, grid, lds, parity, kstep, st, ev0, ev1);
  }
  return hipErrorInvalidValue;
}
