// Minimax line of a partition (section 3.1's fixed-width objective): the
// smallest slope minimising the vertical width of the strip that holds every
// point (t, v_t).  The width, as a function of the slope, is convex and bends
// only at edge slopes of the upper and lower convex hulls of the points; its
// right derivative there is t_lo - t_up, the positions of the lower-hull and
// upper-hull vertices that touch the strip just above the bend.  The answer
// is the smallest bend at which t_lo >= t_up, as the exact fraction dy / dt of
// the hull edge it comes from (an upper edge when an upper and a lower edge
// have the same slope).
//
// GPU layout, a group of kT threads per partition (a workgroup of 256, tiles
// of 4096 points, or one wavefront of 64, partitions of at most 1024):
//   * every thread builds the hulls of its 16 consecutive points in LDS;
//   * log2(kT) rounds merge neighbouring hulls pairwise: one thread per pair
//     and side walks to the bridge (the common tangent), then the group
//     moves the right hull's kept vertices next to the left hull's;
//   * a partition of several tiles merges each tile's hulls into a running
//     hull held in global scratch, in the same way;
//   * every hull edge is tested as the answer at once: its right-derivative
//     sign needs one binary search over the other hull; a workgroup
//     minimum picks the smallest passing edge.
// Cross products are exact: positions differ by less than 2^20 and values by
// less than 2^61, so differences fit int64 and products int128.  A hull tile
// whose values span less than 2^40 holds them as binary64 offsets from the
// partition minimum instead: positions below 2^12 and offsets below 2^40
// give differences below 2^41 and products below 2^53, so the same tests
// are exact in binary64, at a few instructions instead of two 128-bit
// products.
#pragma once

#include "fit.hpp"

namespace leco {

constexpr uint32_t kHullChunk = 16;                        // points per thread
constexpr uint32_t kHullTile = kEncBlock * kHullChunk;     // points per tile

struct HullPoint {
  uint32_t t;   // position in the partition
  uint64_t v;   // value
};

// A point of a tile held in binary64: position and offset from the minimum.
struct HullPointF {
  double t, y;
};

// Offsets below this bound take the binary64 tests (tiles of at most 4096
// points).
constexpr uint64_t kHullF64Range = uint64_t(1) << 40;

// Whether q leaves the upper (lower) hull of p, q, r with p.t < q.t < r.t:
// r lies on or above (on or below) the line through p and q.
__device__ inline bool hull_drops(bool upper, HullPoint p, HullPoint q, HullPoint r) {
  const __int128 a = __int128(int64_t(q.t - p.t)) * int64_t(r.v - p.v);
  const __int128 b = __int128(int64_t(q.v - p.v)) * int64_t(r.t - p.t);
  return upper ? a >= b : a <= b;
}

__device__ inline bool hull_drops(bool upper, HullPointF p, HullPointF q, HullPointF r) {
  const double a = __dmul_rn(q.t - p.t, r.y - p.y);
  const double b = __dmul_rn(q.y - p.y, r.t - p.t);
  return upper ? a >= b : a <= b;
}

// Tile point x with its LDS word: the value itself, or (kF) the bits of its
// binary64 offset.
template <bool kF>
__device__ __attribute__((always_inline)) inline auto hull_pt(uint32_t x, uint64_t word) {
  if constexpr (kF)
    return HullPointF{double(x), __longlong_as_double(static_cast<long long>(word))};
  else
    return HullPoint{x, word};
}

struct EdgeSlope {
  int64_t dy;
  uint32_t dt;  // > 0
};

__device__ inline EdgeSlope edge_slope(HullPoint a, HullPoint b) {
  return EdgeSlope{int64_t(b.v - a.v), b.t - a.t};
}

__device__ inline bool slope_le(EdgeSlope a, EdgeSlope b) {
  return __int128(a.dy) * b.dt <= __int128(b.dy) * a.dt;
}

__device__ inline bool slope_lt(EdgeSlope a, EdgeSlope b) {
  return __int128(a.dy) * b.dt < __int128(b.dy) * a.dt;
}

// The same on binary64 points (offsets below 2^40, positions below 2^12:
// dy and dt exact, products below 2^52).
struct EdgeSlopeF {
  double dy, dt;
};

__device__ inline EdgeSlopeF edge_slope(HullPointF a, HullPointF b) {
  return EdgeSlopeF{b.y - a.y, b.t - a.t};
}

__device__ inline bool slope_le(EdgeSlopeF a, EdgeSlopeF b) {
  return __dmul_rn(a.dy, b.dt) <= __dmul_rn(b.dy, a.dt);
}

__device__ inline bool slope_lt(EdgeSlopeF a, EdgeSlopeF b) {
  return __dmul_rn(a.dy, b.dt) < __dmul_rn(b.dy, a.dt);
}

__device__ inline EdgeSlope shfl_xor_slope(EdgeSlope s, uint32_t m) {
  return EdgeSlope{static_cast<int64_t>(__shfl_xor(static_cast<long long>(s.dy), int(m), 64)),
                   static_cast<uint32_t>(__shfl_xor(static_cast<int>(s.dt), int(m), 64))};
}
__device__ inline EdgeSlopeF shfl_xor_slope(EdgeSlopeF s, uint32_t m) {
  return EdgeSlopeF{__shfl_xor(s.dy, int(m), 64), __shfl_xor(s.dt, int(m), 64)};
}

__device__ inline EdgeSlope edge_int(EdgeSlope s) { return s; }
__device__ inline EdgeSlope edge_int(EdgeSlopeF s) {
  return EdgeSlope{static_cast<int64_t>(s.dy), static_cast<uint32_t>(s.dt)};
}
__device__ inline uint32_t hull_pos(HullPoint p) { return p.t; }
__device__ inline uint32_t hull_pos(HullPointF p) { return static_cast<uint32_t>(p.t); }

// Bridge of hull A (p vertices) and hull B (q vertices), A entirely left of
// B: the union's hull is A[0, keep) followed by B[from, q).  A(i) and B(j)
// return vertices.  Walks inwards from the facing ends until neither end
// can move.
template <class PA, class PB>
__device__ __attribute__((always_inline)) inline void hull_bridge(bool upper, const PA& A, uint32_t p, const PB& B, uint32_t q,
                                   uint32_t& keep, uint32_t& from) {
  uint32_t i = p - 1, j = 0;
  auto a = A(i);
  auto b = B(j);
  for (;;) {
    bool moved = false;
    while (i > 0) {
      const auto a0 = A(i - 1);
      if (!hull_drops(upper, a0, a, b)) break;
      a = a0;
      --i;
      moved = true;
    }
    while (j + 1 < q) {
      const auto b1 = B(j + 1);
      if (!hull_drops(upper, a, b, b1)) break;
      b = b1;
      ++j;
      moved = true;
    }
    if (!moved) break;
  }
  keep = i + 1;
  from = j;
}

// The same bridge found by hg lanes of one wavefront at once (an aligned
// block of lanes; this lane is l of them), without a dependent walk.  For
// the upper hulls: the tangent from B's vertex j to A touches the vertex k
// of smallest slope(A[k], B[j]), and the common tangent is the one of
// largest slope over j; the walk passes collinear vertices, so it ends on
// the leftmost such k and the rightmost such j, which the ties below
// reproduce.  The lower hulls mirror it (largest slope to A, smallest over
// j).  Lane l takes j = l, l + hg, ...; every lane of the block receives
// the bridge.  Since b = B[j] lies right of every vertex of A, the slope
// from A[k] to b falls strictly while b is strictly below the line through
// A[k] and A[k+1] (upper hulls; above, for the lower), and that holds for
// a prefix of k because A is convex: a binary search for the end of the
// prefix finds the leftmost tangent vertex in log2(p) steps.
template <class PA, class PB>
__device__ __attribute__((always_inline)) inline void hull_bridge_lanes(
    bool upper, const PA& A, uint32_t p, const PB& B, uint32_t q, uint32_t l, uint32_t hg,
    uint32_t& keep, uint32_t& from) {
  using S = decltype(edge_slope(A(0), B(0)));
  // x before y in the order of preference: upper, smaller tangent slope to
  // A and larger over B; lower, the reverse
  const auto ahead = [&](S x, S y) { return upper ? slope_lt(x, y) : slope_lt(y, x); };
  bool have = false;
  S best = edge_slope(A(0), B(0));
  uint32_t bi = 0, bj = 0;
  for (uint32_t j = l; j < q; j += hg) {
    const auto b = B(j);
    uint32_t i = 0, hi = p - 1;
    while (i < hi) {
      const uint32_t mid = (i + hi) >> 1;
      if (ahead(edge_slope(A(mid + 1), b), edge_slope(A(mid), b)))
        i = mid + 1;
      else
        hi = mid;
    }
    const S s = edge_slope(A(i), b);
    if (!have || !ahead(s, best)) {  // j grows: the rightmost j on ties
      best = s;
      bi = i;
      bj = j;
      have = true;
    }
  }
  for (uint32_t m = 1; m < hg; m <<= 1) {
    const bool oh = __shfl_xor(int(have), int(m), 64) != 0;
    const S os = shfl_xor_slope(best, m);
    const uint32_t oi = uint32_t(__shfl_xor(int(bi), int(m), 64));
    const uint32_t oj = uint32_t(__shfl_xor(int(bj), int(m), 64));
    const bool tie = !ahead(os, best) && !ahead(best, os);
    if (oh && (!have || ahead(best, os) || (tie && oj > bj))) {
      best = os;
      bi = oi;
      bj = oj;
      have = true;
    }
  }
  keep = bi + 1;
  from = bj;
}

// Rounds of kLaneBridgeMin to kLaneBridgeMax threads find their bridges
// with all of them, at most a wavefront per side (hull_bridge_lanes); the
// others with one thread per side (hull_bridge).
constexpr uint32_t kLaneBridgeMin = 16;
constexpr uint32_t kLaneBridgeMax = 64;

template <int kT>
struct HullSharedT {
  static constexpr uint32_t kTile = kT * kHullChunk;
  uint64_t v[kTile];                // the tile's values
  uint16_t h[2][kTile];             // upper, lower hull vertices (tile positions)
  uint16_t cnt[2][kT];              // hull sizes, at each group's first thread
  uint16_t keep[2][kT];             // bridge results, at each group's first thread
  uint16_t from[2][kT];
  uint32_t rcnt[2];                 // running hull sizes (partitions of several tiles)
  uint32_t rkeep[2], rfrom[2];      // bridge of the running hull and the tile's
  int64_t red_dy[kT / 64];
  uint32_t red_dt[kT / 64];
  uint32_t red_flag[kT / 64];
};
using HullShared = HullSharedT<kEncBlock>;

// Makes the group's LDS writes visible to the whole group: a workgroup
// barrier, or for a single wavefront a wave barrier with wavefront fences.
template <int kT>
__device__ __attribute__((always_inline)) inline void group_sync() {
  if constexpr (kT == 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Upper and lower hulls of the tile's points 0 .. cnt-1 (sh.v: values, or
// with kF the bits of binary64 offsets below kHullF64Range), left in
// sh.h[side][0 .. sh.cnt[side][0]).  Called by every thread tid of the group.
template <int kT, bool kF>
__device__ __attribute__((always_inline)) inline void tile_hulls(HullSharedT<kT>& sh, uint32_t cnt,
                                                                 uint32_t tid) {
  const uint32_t c0 = tid * kHullChunk;
  const uint32_t c1 = c0 + kHullChunk < cnt ? c0 + kHullChunk : (c0 < cnt ? cnt : c0);
  // the thread's points in registers; the chain keeps its top two vertices
  // in registers too, so a test reads no LDS and a removal reads one vertex
  uint64_t pv[kHullChunk];
#pragma unroll
  for (uint32_t j = 0; j < kHullChunk; ++j) pv[j] = c0 + j < c1 ? sh.v[c0 + j] : 0;
  for (uint32_t side = 0; side < 2; ++side) {
    uint16_t* H = sh.h[side] + c0;
    uint32_t k = 0;
    auto below = hull_pt<kF>(0, 0), top = below;  // H[k-2] and H[k-1] when k >= 2
#pragma unroll
    for (uint32_t j = 0; j < kHullChunk; ++j) {
      const uint32_t t = c0 + j;
      if (t < c1) {
        const auto r = hull_pt<kF>(t, pv[j]);
        while (k >= 2 && hull_drops(side == 0, below, top, r)) {
          --k;
          top = below;
          if (k >= 2) below = hull_pt<kF>(H[k - 2], sh.v[H[k - 2]]);
        }
        H[k++] = uint16_t(t);
        below = top;
        top = r;
      }
    }
    sh.cnt[side][tid] = uint16_t(k);
  }
  // A round of G <= 64 threads reads and writes only its group's hulls,
  // which lie in one wavefront: a wavefront barrier orders it.  Wider
  // rounds take the workgroup barrier, and the first of them one more
  // before it starts (the wavefronts' narrow rounds ran unsynchronised).
  const auto round_sync = [](uint32_t G) {
    if (kT > 64 && G > 64)
      __syncthreads();
    else
      group_sync<64>();
  };
  round_sync(2);
  for (uint32_t G = 2; G <= uint32_t(kT); G <<= 1) {
    if (kT > 64 && G == 128) __syncthreads();
    const uint32_t half = G >> 1, r = tid & (G - 1), g = tid - r;
    if (G >= kLaneBridgeMin && G <= kLaneBridgeMax) {
      // half of the group per side, of which the first wavefront (or all
      // of them, in a narrower round) searches
      const uint32_t side = r / half, l = r - side * half;
      const uint32_t hg = half < 64 ? half : 64;
      const uint32_t p = sh.cnt[side][g], q = sh.cnt[side][g + half];
      uint32_t keep = p, from = q;  // an empty right hull adds nothing
      if (q > 0 && p == 0) {
        keep = 0;
        from = 0;
      } else if (q > 0 && l < hg) {
        const uint16_t* HA = sh.h[side] + kHullChunk * g;
        const uint16_t* HB = sh.h[side] + kHullChunk * (g + half);
        const auto A = [&](uint32_t i) { return hull_pt<kF>(HA[i], sh.v[HA[i]]); };
        const auto B = [&](uint32_t j) { return hull_pt<kF>(HB[j], sh.v[HB[j]]); };
        hull_bridge_lanes(side == 0, A, p, B, q, l, hg, keep, from);
      }
      if (l == 0) {
        sh.keep[side][g] = uint16_t(keep);
        sh.from[side][g] = uint16_t(from);
      }
    } else if (r < 2) {
      const uint32_t side = r;
      const uint32_t p = sh.cnt[side][g], q = sh.cnt[side][g + half];
      uint32_t keep = p, from = q;  // an empty right hull adds nothing
      if (q > 0 && p == 0) {
        keep = 0;
        from = 0;
      } else if (q > 0) {
        const uint16_t* HA = sh.h[side] + kHullChunk * g;
        const uint16_t* HB = sh.h[side] + kHullChunk * (g + half);
        const auto A = [&](uint32_t i) { return hull_pt<kF>(HA[i], sh.v[HA[i]]); };
        const auto B = [&](uint32_t j) { return hull_pt<kF>(HB[j], sh.v[HB[j]]); };
        hull_bridge(side == 0, A, p, B, q, keep, from);
      }
      sh.keep[side][g] = uint16_t(keep);
      sh.from[side][g] = uint16_t(from);
    }
    round_sync(G);
    // the right hull's kept vertices, staged so that moving them left never
    // overwrites one not yet read: at most 16 * half / G = 8 per thread
    constexpr uint32_t kStage = kHullChunk / 2;
    uint16_t stage[2][kStage];
    uint32_t moved[2];
    for (uint32_t side = 0; side < 2; ++side) {
      const uint32_t q = sh.cnt[side][g + half], from = sh.from[side][g];
      moved[side] = q - from;
      const uint16_t* HB = sh.h[side] + kHullChunk * (g + half) + from;
#pragma unroll
      for (uint32_t s = 0; s < kStage; ++s) {
        const uint32_t x = r + s * G;
        if (x >= moved[side]) break;  // most rounds move a few vertices
        stage[side][s] = HB[x];
      }
    }
    round_sync(G);
    for (uint32_t side = 0; side < 2; ++side) {
      const uint32_t keep = sh.keep[side][g];
      uint16_t* HA = sh.h[side] + kHullChunk * g + keep;
#pragma unroll
      for (uint32_t s = 0; s < kStage; ++s) {
        const uint32_t x = r + s * G;
        if (x >= moved[side]) break;
        HA[x] = stage[side][s];
      }
      if (r == side) sh.cnt[side][g] = uint16_t(keep + moved[side]);
    }
    round_sync(G);
  }
}

// The smallest hull edge slope at which the strip width stops decreasing,
// over hulls U (nu vertices) and L (nl vertices) given by accessors (of
// HullPoint or HullPointF vertices: the binary searches compare slopes of
// the accessors' type, the answer is kept as an exact EdgeSlope).  Every
// thread receives the answer.  Called by every thread tid of the group.
template <int kT, class PU, class PL>
__device__ __attribute__((always_inline)) inline EdgeSlope minimax_bend(HullSharedT<kT>& sh,
                                                                        const PU& U, uint32_t nu,
                                                                        const PL& L, uint32_t nl,
                                                                        uint32_t tid) {
  bool found = false, from_upper = false;
  EdgeSlope best{0, 1};
  const uint32_t edges = (nu - 1) + (nl - 1);
  for (uint32_t e = tid; e < edges; e += kT) {
    EdgeSlope th;
    uint32_t t_up, t_lo;
    bool upper_edge;
    if (e < nu - 1) {
      // upper edge e: just above its slope the strip touches U[e] from above
      upper_edge = true;
      const auto a = U(e);
      const auto s = edge_slope(a, U(e + 1));
      t_up = hull_pos(a);
      // and L[c] from below, c = number of lower edges with slope <= th
      uint32_t lo = 0, hi = nl - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (slope_le(edge_slope(L(mid), L(mid + 1)), s)) lo = mid + 1; else hi = mid;
      }
      t_lo = hull_pos(L(lo));
      th = edge_int(s);
    } else {
      upper_edge = false;
      const uint32_t j = e - (nu - 1);
      const auto b = L(j + 1);
      const auto s = edge_slope(L(j), b);
      t_lo = hull_pos(b);
      // U[k], k = first upper edge with slope <= th (upper slopes decrease)
      uint32_t lo = 0, hi = nu - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (slope_le(edge_slope(U(mid), U(mid + 1)), s)) hi = mid; else lo = mid + 1;
      }
      t_up = hull_pos(U(lo));
      th = edge_int(s);
    }
    if (t_lo >= t_up) {
      const bool better = !found || slope_lt(th, best) || (!slope_lt(best, th) && upper_edge && !from_upper);
      if (better) {
        found = true;
        best = th;
        from_upper = upper_edge;
      }
    }
  }
  // workgroup minimum: by value, upper edges first among equal values
  uint32_t flag = (found ? 2u : 0u) | (from_upper ? 1u : 0u);
  const auto take = [&](int64_t dy, uint32_t dt, uint32_t f) {
    if (!(f & 2)) return;
    const EdgeSlope o{dy, dt};
    if (!(flag & 2) || slope_lt(o, best) || (!slope_lt(best, o) && (f & 1) && !(flag & 1))) {
      best = o;
      flag = f;
    }
  };
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const int64_t dy = static_cast<int64_t>(__shfl_xor(static_cast<long long>(best.dy), m, 64));
    const uint32_t dt = static_cast<uint32_t>(__shfl_xor(static_cast<int>(best.dt), m, 64));
    const uint32_t f = static_cast<uint32_t>(__shfl_xor(static_cast<int>(flag), m, 64));
    take(dy, dt, f);
  }
  if constexpr (kT > 64) {
    const uint32_t lane = tid & 63, wave = tid >> 6;
    if (lane == 0) {
      sh.red_dy[wave] = best.dy;
      sh.red_dt[wave] = best.dt;
      sh.red_flag[wave] = flag;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kT / 64; ++w) take(sh.red_dy[w], sh.red_dt[w], sh.red_flag[w]);
    __syncthreads();
  }
  return best;
}

}  // namespace leco
