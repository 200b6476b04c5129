// Cutoff pair kernels.
//
//  * excluded volume: eq. u_ex for every pair within rc (all beads);
//  * real-space electrostatics: the bracket of eq. ewald,
//    lB z_i z_j [erf(alpha_ij r) - erf(beta r)]/r, over the charged beads only
//    (their own cell list and compacted arrays), so the transcendental-heavy
//    term costs nothing for neutral beads and the kernels never branch on
//    charge.
//
// Both work on "clusters": CI consecutive beads of the cell-sorted order
// (CI = 2, 4 or 8; spatially compact because the order is by cell), one
// wavefront per cluster, either with a neighbour list in HBM (two launches)
// or list-free (one launch, k_pair_fused):
//
//  1. k_nl_build: one wavefront per cluster.  The lanes enumerate the cell
//     columns within reach of the cluster's bounding box (culled by the exact
//     box-to-column distance, z runs clipped to the cutoff sphere), expand the
//     runs into an LDS candidate buffer, and test each candidate against every
//     bead of the cluster with the exact minimum-image distance.  A candidate
//     within rc of at least one cluster bead is appended (ballot compaction,
//     candidate order) to the cluster's list: the list is the union of the
//     beads' cutoff spheres, not a bounding-box shell.
//  2. k_nl_force: one wavefront per cluster, lanes laid out as
//     CI cluster beads x (64/CI) list entries.  Every lane evaluates its
//     (bead, entry) pair, masked by the exact cutoff test, so the hot loop has
//     no per-lane walk and no divergence beyond the mask.  Each pair is seen
//     from both ends (no scatter of forces to j); the partial forces of a bead
//     are combined with xor shuffles in a fixed order and added once to the
//     64-bit fixed-point accumulator.
//
//  k_pair_fused does both in one pass: the candidates that pass the list
//  test go to a small LDS ring instead of HBM, and every 64 of them are
//  evaluated at once with the force pass's lane layout.
//
// Lists are rebuilt every evaluation, so they need no skin.  The minimum
// image is the wrapped 32-bit difference of the fractional fixed-point
// coordinates (valid because rc <= L/2 is enforced).
#include <type_traits>
#include <utility>

#include "gcme_internal.h"

namespace gcme {

namespace {

// hardware 2^x (1 ulp; results below the smallest normal flush to zero,
// far below anything the single-precision sums resolve)
__device__ inline float gexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline double gexp2(double x) { return exp2(x); }
__device__ inline float gexp(float x) { return expf(x); }
__device__ inline double gexp(double x) { return exp(x); }
__device__ inline float gerfc(float x) { return erfcf(x); }
__device__ inline double gerfc(double x) { return erfc(x); }
__device__ inline float gsqrt(float x) { return sqrtf(x); }
__device__ inline double gsqrt(double x) { return sqrt(x); }

// erfc(x) e^(x^2), x >= 0, in single precision by the rational
// approximation of Abramowitz and Stegun (Handbook of Mathematical
// Functions, 7.1.26): with t = 1/(1 + p x), erfc(x) = (a1 t + a2 t^2 +
// a3 t^3 + a4 t^4 + a5 t^5) e^(-x^2), absolute error at most 1.5e-7.  The
// factor e^(-x^2) is left to the caller, who needs it for the force too.
__device__ inline float erfc_scaled(float x) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
  return t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f),
                  0.254829592f);
}

template <typename T>
struct Series;
template <>
struct Series<float> {
  static constexpr int n = 8;
};
template <>
struct Series<double> {
  static constexpr int n = NSER;
};

constexpr int NL_WAVES = 4;    // wavefronts (clusters) per workgroup
constexpr int NL_CAND = 1024;  // LDS candidate buffer per wavefront
constexpr int NL_SEG = 128;    // LDS segment list per wavefront (two per column)

__device__ inline int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ inline int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Number of set bits of m below this lane.
__device__ inline int lanes_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ inline uint32_t read_lane(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }

// A wave-uniform float kept in a scalar register (the VALU reads it as an
// operand, so it costs no vector register).
__device__ inline float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }

// Fixed-order sum over the block (NL_WAVES waves); result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < NL_WAVES; ++w) t += sh[w];
  }
  return t;
}

__device__ inline long long to_fixed(double f, double scale, unsigned int* status) {
  double v = f * scale;
  if (!(fabs(v) < 4.0e18)) {
    atomicOr(status, (unsigned)STATUS_FORCE_OVERFLOW);
    return 0;
  }
  return (long long)llrint(v);
}

// ---------------------------------------------------------------------------
// Candidate enumeration, shared by the list build and the list-free kernel
// ---------------------------------------------------------------------------

// A cluster as wave-uniform values.  Its geometry is kept in float relative
// to the lower corner of bead 0's cell: every value is a few cells at most,
// so float carries it to ~1e-7 of a cell, and the margin in rclm keeps each
// cell range conservative.
template <int CI>
struct Cluster {
  uint32_t ux[CI], uy[CI], uz[CI];  // fixed-point positions (slots beyond ni repeat bead 0)
  float lo[3], hi[3];               // bounding box relative to bead 0
  int c0[3];                        // cell of bead 0
  float p0[3];                      // bead 0 within its cell
  float h[3], ih[3];                // cell edges and their inverses
  float qx[CI], qy[CI], qz[CI];     // -2 x (positions relative to bead 0)
  float nn[CI];                     // squared distances from bead 0
  bool compact;                     // every bead within 3 rcl of bead 0
  float rcl;                        // list cutoff, a hair above rc
  float rclm;                       // enumeration radius: rcl plus a margin
  int clo[3], chi[3];               // cell ranges relative to c0 (absolute when whole)
  bool whole[3];                    // the range spans the whole axis
};

// The cluster's geometry from its bead records (lane k < ni holds bead k's
// record in `me`; slots beyond ni repeat bead 0).
template <int CI>
__device__ inline void make_cluster(Cluster<CI>& K, const uint4 me, const RepDesc& R) {
#pragma unroll
  for (int k = 0; k < CI; ++k) {
    K.ux[k] = read_lane(me.x, k);
    K.uy[k] = read_lane(me.y, k);
    K.uz[k] = read_lane(me.z, k);
  }
  float rx[CI], ry[CI], rz[CI];  // positions relative to bead 0
#pragma unroll
  for (int k = 0; k < CI; ++k) {
    rx[k] = (float)(int)(K.ux[k] - K.ux[0]) * R.scalef[0];
    ry[k] = (float)(int)(K.uy[k] - K.uy[0]) * R.scalef[1];
    rz[k] = (float)(int)(K.uz[k] - K.uz[0]) * R.scalef[2];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) K.lo[k] = K.hi[k] = 0.f;
#pragma unroll
  for (int k = 1; k < CI; ++k) {
    K.lo[0] = fminf(K.lo[0], rx[k]);
    K.hi[0] = fmaxf(K.hi[0], rx[k]);
    K.lo[1] = fminf(K.lo[1], ry[k]);
    K.hi[1] = fmaxf(K.hi[1], ry[k]);
    K.lo[2] = fminf(K.lo[2], rz[k]);
    K.hi[2] = fmaxf(K.hi[2], rz[k]);
  }
  const uint32_t u0[3] = {K.ux[0], K.uy[0], K.uz[0]};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const unsigned long long pp = (unsigned long long)u0[k] * (unsigned)R.nc[k];
    K.c0[k] = (int)(pp >> 32);
    K.h[k] = R.hf[k];
    K.ih[k] = 1.0f / K.h[k];
    K.p0[k] = (float)(uint32_t)(pp & 0xffffffffu) * 2.3283064365386963e-10f * K.h[k];
  }
  // the float list test with rcl never drops a pair that the pair kernels'
  // own test (in their precision) keeps
  K.rcl = (float)(R.rc * (1.0 + 1e-5));
  K.rclm = K.rcl + 1e-4f * fmaxf(K.h[0], fmaxf(K.h[1], K.h[2]));
  float nmax = 0.f;
#pragma unroll
  for (int k = 0; k < CI; ++k) {
    K.qx[k] = uni(-2.f * rx[k]);
    K.qy[k] = uni(-2.f * ry[k]);
    K.qz[k] = uni(-2.f * rz[k]);
    K.nn[k] = uni(rx[k] * rx[k] + ry[k] * ry[k] + rz[k] * rz[k]);
    nmax = fmaxf(nmax, K.nn[k]);
  }
  K.compact = nmax <= 9.f * K.rcl * K.rcl;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    K.clo[k] = (int)floorf((K.p0[k] + K.lo[k] - K.rclm) * K.ih[k]);
    K.chi[k] = (int)floorf((K.p0[k] + K.hi[k] + K.rclm) * K.ih[k]);
    K.whole[k] = K.chi[k] - K.clo[k] + 1 >= R.nc[k];
    if (K.whole[k]) {
      K.clo[k] = 0;
      K.chi[k] = R.nc[k] - 1;
    }
  }
}

template <int CI>
__device__ inline void load_cluster(Cluster<CI>& K, const uint4* __restrict__ pk, int first, int ni,
                                    const RepDesc& R) {
  const int lane = threadIdx.x & 63;
  make_cluster(K, pk[first + (lane < ni ? lane : 0)], R);
}

// Sign of the periodic offset from cell index a to cell index c along an
// axis of n cells: +1 when c lies less than half the axis ahead of a, -1
// when less than half behind, 0 when equal; at exactly half the axis the
// smaller index counts as behind.  ahead(c, a, n) = -ahead(a, c, n).
__device__ inline int ahead(int c, int a, int n) {
  int d = c - a;
  if (d == 0) return 0;
  if (d < 0) d += n;
  if (2 * d < n) return 1;
  if (2 * d > n) return -1;
  return a < c ? 1 : -1;
}

// One round of the enumeration: the columns cbase .. cbase + 63 of the
// cluster's reach, one per lane, culled by the exact box-to-column distance,
// each z run clipped to the sphere of radius rclm around the box and split
// at the periodic end into up to two bead ranges; the non-empty ranges go to
// seg_b / seg_l (wave-level, no block barriers).  Returns their number.
template <int CI, bool HALF>
__device__ inline int column_segments(const Cluster<CI>& K, const RepDesc& R, const int* __restrict__ start,
                                      int first, int cbase, int* seg_b, int* seg_l) {
  const int lane = threadIdx.x & 63;
  const int nx = R.nc[0], ny = R.nc[1], nz = R.nc[2];
  const int ncx = K.chi[0] - K.clo[0] + 1, ncy = K.chi[1] - K.clo[1] + 1;
  const int ncol = ncx * ncy;
  const float rclm2 = K.rclm * K.rclm;
  int b0[2] = {0, 0}, ln[2] = {0, 0};
  const int k = cbase + lane;
  if (k < ncol) {
    const int rx = K.clo[0] + k / ncy, ry = K.clo[1] + k % ncy;
    const float gx = K.whole[0] ? 0.f
                                : fmaxf(0.f, fmaxf(rx * K.h[0] - (K.p0[0] + K.hi[0]),
                                                   (K.p0[0] + K.lo[0]) - (rx + 1) * K.h[0]));
    const float gy = K.whole[1] ? 0.f
                                : fmaxf(0.f, fmaxf(ry * K.h[1] - (K.p0[1] + K.hi[1]),
                                                   (K.p0[1] + K.lo[1]) - (ry + 1) * K.h[1]));
    const float d2 = gx * gx + gy * gy;
    if (d2 < rclm2) {
      int cx = K.whole[0] ? rx : K.c0[0] + rx;
      int cy = K.whole[1] ? ry : K.c0[1] + ry;
      cx += cx < 0 ? nx : (cx >= nx ? -nx : 0);
      cy += cy < 0 ? ny : (cy >= ny ? -ny : 0);
      const int sx = HALF ? ahead(cx, K.c0[0], nx) : 1, sy = HALF ? ahead(cy, K.c0[1], ny) : 1;
      const bool owned = sx > 0 || (sx == 0 && sy >= 0);
      int zlo = 0, zhi = nz - 1;
      if (!K.whole[2]) {
        const float zr = sqrtf(rclm2 - d2);
        zlo = K.c0[2] + (int)floorf((K.p0[2] + K.lo[2] - zr) * K.ih[2]);
        zhi = K.c0[2] + (int)floorf((K.p0[2] + K.hi[2] + zr) * K.ih[2]);
        if (zhi - zlo + 1 >= nz) {
          zlo = 0;
          zhi = nz - 1;
        }
      }
      const int colbase = R.cell_off + (cx * ny + cy) * nz;
      if (zlo < 0) {
        b0[0] = start[colbase + zlo + nz];
        ln[0] = start[colbase + nz] - b0[0];
        b0[1] = start[colbase];
        ln[1] = start[colbase + zhi + 1] - b0[1];
      } else if (zhi >= nz) {
        b0[0] = start[colbase + zlo];
        ln[0] = start[colbase + nz] - b0[0];
        b0[1] = start[colbase];
        ln[1] = start[colbase + zhi - nz + 1] - b0[1];
      } else {
        b0[0] = start[colbase + zlo];
        ln[0] = start[colbase + zhi + 1] - b0[0];
      }
      if (HALF && !owned) ln[0] = ln[1] = 0;
      if (HALF && sx == 0 && sy == 0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int e = b0[q] + ln[q], nb = max(b0[q], first);
          ln[q] = max(0, e - nb);
          b0[q] = nb;
        }
      }
    }
  }
  int nseg = 0;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const bool has = ln[q] > 0;
    const unsigned long long m = __ballot(has);
    if (has) {
      const int p = nseg + lanes_below(m);
      seg_b[p] = b0[q];
      seg_l[p] = ln[q];
    }
    nseg += __popcll(m);
  }
  __builtin_amdgcn_wave_barrier();
  return nseg;
}

// Every bead of the cells within reach of the cluster: the columns whose
// distance to the cluster's box is below rclm, each with its z run clipped to
// the sphere of radius rclm around the box.  The beads are handed over in
// rounds: a round leaves up to NL_CAND bead indices in cand[0, total) and
// calls visit(total).  Wavefront-level only (no block barriers); seg_b and
// seg_l are the wavefront's NL_SEG-entry segment scratch.
// With HALF, only the columns the cluster owns pairs with are enumerated:
// the cluster's own column (bead 0's; a column cluster never leaves it),
// clipped to the beads from `first` on, and the columns ahead of it (ahead
// along x, or level along x and ahead along y).  A column pair is owned by
// exactly one side, so every unordered pair within rc is visited by one
// cluster only (within the own column: by the lower sorted index).
template <int CI, bool HALF = false, class V>
__device__ inline void for_candidates(const Cluster<CI>& K, const RepDesc& R, const int* __restrict__ start,
                                      int* seg_b, int* seg_l, int* cand, V&& visit, int first = 0) {
  const int lane = threadIdx.x & 63;
  const int ncol = (K.chi[0] - K.clo[0] + 1) * (K.chi[1] - K.clo[1] + 1);
  for (int cbase = 0; cbase < ncol; cbase += 64) {
    const int nseg = column_segments<CI, HALF>(K, R, start, first, cbase, seg_b, seg_l);
    // expand segments into the candidate buffer (a segment too long for the
    // room left is split across rounds), then visit the round
    int sn = 0, soff = 0;
    while (sn < nseg) {
      const int s = sn + lane;
      int sb = 0, sl = 0;
      if (s < nseg) {
        sb = seg_b[s];
        sl = seg_l[s];
        if (lane == 0) {
          sb += soff;
          sl -= soff;
        }
      }
      const int inc = wave_incl_scan(sl);
      const int exc = inc - sl;
      const int take = max(0, min(sl, NL_CAND - exc));
      const int mt = wave_max(take);
      for (int t = 0; t < mt; ++t)
        if (t < take) cand[exc + t] = sb + t;
      const int total = min((int)read_lane((uint32_t)inc, 63), NL_CAND);
      const unsigned long long partial = __ballot(take < sl);
      if (partial == 0ull) {
        sn += 64;
        soff = 0;
      } else {
        const int f = __ffsll((long long)partial) - 1;
        const int tf = (int)read_lane((uint32_t)take, f);
        soff = (f == 0 ? soff : 0) + tf;
        sn += f;
      }
      __builtin_amdgcn_wave_barrier();
      visit(total);
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// The candidates cand[0, total) in chunks of 64, one per lane: the index and
// bead-record loads of NCH chunks are issued together (one memory latency
// covers them), then f(record, valid, index) runs per chunk in order.
template <int NCH, class F>
__device__ inline void for_chunks(const int* cand, int total, const uint4* __restrict__ pk, int fallback, F&& f) {
  const int lane = threadIdx.x & 63;
  for (int p = 0; p < total; p += 64 * NCH) {
    int jj[NCH];
    uint4 rr[NCH];
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
      const int q = p + 64 * u + lane;
      jj[u] = q < total ? cand[q] : -1;
    }
#pragma unroll
    for (int u = 0; u < NCH; ++u) rr[u] = pk[jj[u] < 0 ? fallback : jj[u]];
#pragma unroll
    for (int u = 0; u < NCH; ++u)
      if (u == 0 || p + 64 * u < total) f(rr[u], jj[u] >= 0, jj[u] < 0 ? fallback : jj[u]);
  }
}

// ---------------------------------------------------------------------------
// List build
// ---------------------------------------------------------------------------

// Whether the cluster takes the fast path: in the frame of bead 0,
// separations equal the per-pair minimum image for every pair within rc as
// long as each cluster bead lies within L/2 - rc of bead 0 on each axis (then
// |d| < rc cannot wrap); and the cluster is compact (every bead within 3 rcl
// of bead 0), which bounds the rounding of the frame-relative arithmetic.
template <int CI>
__device__ inline bool in_frame(const Cluster<CI>& K, const RepDesc& R) {
  bool frame = K.compact;
#pragma unroll
  for (int k = 0; k < 3; ++k) frame = frame && fmaxf(-K.lo[k], K.hi[k]) < 0.5f * (float)R.L[k] - K.rclm;
  return frame;
}

// Whether bead record pj lies within the list cutoff of at least one bead of
// the cluster (float), for a compact cluster in bead 0's frame; D receives
// pj's position relative to bead 0.  |D - r_i|^2 < rcl^2 is tested as
// |r_i|^2 - 2 D.r_i < rcl^2 - |D|^2: three fused multiply-adds per bead.  The
// candidates that can pass lie within 4 rcl of bead 0, so the rounding of the
// expanded form stays below 1e-5 rcl^2, inside the margin of rcl over rc: no
// pair within rc is dropped.
template <int CI>
__device__ inline bool near_frame(const Cluster<CI>& K, const uint4& pj, const RepDesc& R, float& Dx, float& Dy,
                                  float& Dz) {
  Dx = (float)(int)(pj.x - K.ux[0]) * R.scalef[0];
  Dy = (float)(int)(pj.y - K.uy[0]) * R.scalef[1];
  Dz = (float)(int)(pj.z - K.uz[0]) * R.scalef[2];
  const float thr = K.rcl * K.rcl - (Dx * Dx + Dy * Dy + Dz * Dz);
  bool hit = false;
#pragma unroll
  for (int i = 0; i < CI; ++i) hit |= fmaf(K.qx[i], Dx, fmaf(K.qy[i], Dy, fmaf(K.qz[i], Dz, K.nn[i]))) < thr;
  return hit;
}

// The same test by the minimum image of each pair (any cluster).
template <int CI>
__device__ inline bool near_exact(const Cluster<CI>& K, const uint4& pj, const RepDesc& R) {
  const float rcl2f = K.rcl * K.rcl;
  bool hit = false;
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    const float dx = (float)(int)(K.ux[i] - pj.x) * R.scalef[0];
    const float dy = (float)(int)(K.uy[i] - pj.y) * R.scalef[1];
    const float dz = (float)(int)(K.uz[i] - pj.z) * R.scalef[2];
    hit |= dx * dx + dy * dy + dz * dz < rcl2f;
  }
  return hit;
}

template <int CI>
__device__ inline bool near_cluster(const Cluster<CI>& K, bool fast, const uint4& pj, const RepDesc& R) {
  float Dx, Dy, Dz;
  return fast ? near_frame(K, pj, R, Dx, Dy, Dz) : near_exact(K, pj, R);
}

// Compiled for five wavefronts per SIMD (102 VGPRs; a few spilled for CI =
// 8): the 256 batched replicas' step went 0.763 -> 0.748 ms.
template <int CI>
__global__ __launch_bounds__(NL_WAVES * 64) __attribute__((amdgpu_waves_per_eu(5))) void k_nl_build(PairLaunch a) {
  __shared__ int s_sb[NL_WAVES][NL_SEG];
  __shared__ int s_sl[NL_WAVES][NL_SEG];
  __shared__ int s_cand[NL_WAVES][NL_CAND];
  wave_stamp(a.stamps, 0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = xcd_item(blockIdx.x, gridDim.x) * NL_WAVES + wave;
  if (c >= a.ncl) return;  // whole wavefront; no block barriers below
  const int2 info = a.cl[c];
  const int first = info.x, rep = info.y & 0xffff, ni = info.y >> 16;
  const RepDesc& R = a.rep[rep];
  const uint4* __restrict__ pk = a.pk;
  Cluster<CI> K;
  load_cluster(K, pk, first, ni, R);
  const bool frame = in_frame(K, R);
  uint32_t* __restrict__ out = a.list + (size_t)c * a.cap;
  int nent = 0;
  // one candidate per lane; hits are appended in candidate order
  auto test = [&](const uint4 pj, bool v, int j) {
    const bool hit = near_cluster(K, frame, pj, R) && v;
    const unsigned long long m = __ballot(hit);
    if (hit) {
      const int idx = nent + lanes_below(m);
      if (idx < a.cap) out[idx] = (uint32_t)j;
    }
    nent += __popcll(m);
  };
  const int* cand = s_cand[wave];
  for_candidates(K, R, a.start, s_sb[wave], s_sl[wave], s_cand[wave], [&](int total) {
    for_chunks<2>(cand, total, pk, first, test);
  });
  if (lane == 0) {
    a.count[c] = min(nent, a.cap);
    if (nent > a.cap) atomicOr(a.status, (unsigned)STATUS_LIST_OVERFLOW);
  }
  wave_stamp(a.stamps, 1);
}

// ---------------------------------------------------------------------------
// Pair evaluation
// ---------------------------------------------------------------------------

// Per-lane accumulators.
template <typename T>
struct Lane {
  T fx, fy, fz;
  double e, w0, w1, w2, w3, w4, w5;  // energy and virial summed in FP64
  T eA[MAXT], dj[MAXT], di;          // adjoint sums of the lane's bead i
  T ett[MAXT * MAXT];                // adjoint: type-pair energies (ti, tj)
  T dsg[MAXT];                       // adjoint: d/dsigma_t (excluded volume) or d/da_t (real space)
  unsigned long long cnt;
};

template <typename T>
__device__ inline void lane_zero(Lane<T>& L) {
  L.fx = L.fy = L.fz = 0;
  L.e = L.w0 = L.w1 = L.w2 = L.w3 = L.w4 = L.w5 = 0;
  for (int t = 0; t < MAXT; ++t) L.eA[t] = L.dj[t] = L.dsg[t] = 0;
  for (int t = 0; t < MAXT * MAXT; ++t) L.ett[t] = 0;
  L.di = 0;
  L.cnt = 0;
}

// The real-space bracket of eq. ewald for one type pair at r^2 = r2 > 0:
// phi = [erf(alpha r) - erf(beta r)]/r and g = -(1/r) dphi/dr; ea receives
// exp(-alpha^2 r^2) where the evaluation computes it (left as is in the
// series branch).  cexpb = -beta^2 log2(e), tsb = (2/sqrt(pi)) beta.
template <typename T>
__device__ __attribute__((always_inline)) inline void bracket(const ElecPar<T>& p, T r2, T beta, T beta2, T cexpb,
                                                              T tsb, T& phi, T& g, T& ea) {
  constexpr T TSP = (T)1.1283791670955126;  // 2/sqrt(pi)
  if (r2 < p.rs2) {
    // series in r^2, free of the cancellation near contact
    phi = p.cphi[Series<T>::n - 1];
    g = p.cg[Series<T>::n - 1];
#pragma unroll
    for (int n = Series<T>::n - 2; n >= 0; --n) {
      phi = phi * r2 + p.cphi[n];
      g = g * r2 + p.cg[n];
    }
  } else if constexpr (std::is_same<T, float>::value) {
    // single precision: both error functions from their Gaussians, which
    // the force needs anyway (one reciprocal square root, two 2^x, two
    // reciprocals)
    // each product rounded on its own (no multiply-add fused across a
    // difference), so that alpha == beta gives exactly zero
#pragma clang fp contract(off)
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * rinv;
    ea = gexp2(p.cexp * r2);
    const float eb = gexp2(cexpb * r2);
    phi = (erfc_scaled(beta * r) * eb - erfc_scaled(p.alpha * r) * ea) * rinv;
    g = (phi - (p.tsa * ea - tsb * eb)) * rinv * rinv;
    (void)beta2;
  } else {
    T r = gsqrt(r2);
    T rinv = (T)1 / r;
    ea = gexp(-p.alpha2 * r2);
    phi = (gerfc(beta * r) - gerfc(p.alpha * r)) * rinv;
    g = (phi - TSP * (p.alpha * ea - beta * gexp(-beta2 * r2))) * rinv * rinv;
    (void)cexpb;
    (void)tsb;
  }
}

// One ordered pair (i, j) with separation d = r_i - r_j, r2 < rc^2.
template <typename T, bool ELEC, bool EV, bool ADJ, bool COUNT>
__device__ inline void interact(Lane<T>& L, T dx, T dy, T dz, T r2, uint32_t pj, const GcmPar<T>* grow,
                                const ElecPar<T>* erow, const AdjPar<T>* arow, T zi, T beta, T beta2, T lB,
                                T vx = 0, T vy = 0, T vz = 0, bool vjp = false, T cexpb = 0, T tsb = 0) {
  const int tj = param_type(pj);
  T fs, en;
  if (!ELEC) {
    const GcmPar<T> g = grow[tj];
    en = g.C * gexp2(-g.bl * r2);
    fs = g.twob * en;
    if (ADJ) {
      const AdjPar<T> ap = arow[tj];
      // du/ds = u (3 r^2/s^3 - 3/s), s = s_ij
      T duds = en * ((T)3 * r2 * ap.inv_s2 - (T)3) * ap.s_inv;
      T eA = en;
      if (vjp) {
        // force vector-Jacobian product: (v_i . d) dfs/dtheta with
        // dfs/dA = fs/A (divided by A with the energies) and
        // dfs/ds = (u/s^3)(9 r^2/s^2 - 15)
        const T vd = vx * dx + vy * dy + vz * dz;
        eA = vd * fs;
        duds = vd * en * ap.inv_s2 * ap.s_inv * ((T)9 * r2 * ap.inv_s2 - (T)15);
      }
      L.di += duds * ap.dsig_i;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        if (t == tj) {
          L.eA[t] += eA;
          L.dj[t] += duds * ap.dsig_j;
        }
      }
    }
  } else {
    const ElecPar<T>& p = erow[tj];
    const T zz = zi * (T)param_z(pj);
    T phi, g, ea = 0;  // ea: exp(-alpha^2 r^2) where computed
    bracket(p, r2, beta, beta2, cexpb, tsb, phi, g, ea);
    fs = lB * zz * g;
    en = lB * zz * phi;
    if (ADJ) {
      const AdjPar<T> ap = arow[tj];
      // d/da_ij of lB zz erf(alpha r)/r = -lB zz (2/sqrt(pi)) (alpha/a_ij) exp(-alpha^2 r^2)
      if (r2 < p.rs2) ea = gexp(-p.alpha2 * r2);
      T dd = -lB * zz * ap.ea * ea;
      // force vector-Jacobian product: dg/dalpha = 2 (2/sqrt(pi)) alpha^2
      // exp(-alpha^2 r^2), so dfs/da_ij = 2 alpha^2 dd
      if (vjp) dd = (vx * dx + vy * dy + vz * dz) * (T)2 * p.alpha2 * dd;
      L.di += dd * ap.daij_i;
#pragma unroll
      for (int t = 0; t < MAXT; ++t)
        if (t == tj) L.dj[t] += dd * ap.daij_j;
    }
  }
  L.fx += fs * dx;
  L.fy += fs * dy;
  L.fz += fs * dz;
  if (EV) {
    const double fxd = (double)(fs * dx), fyd = (double)(fs * dy), fzd = (double)(fs * dz);
    L.e += (double)en;
    L.w0 += fxd * (double)dx;
    L.w1 += fyd * (double)dy;
    L.w2 += fzd * (double)dz;
    L.w3 += fxd * (double)dy;
    L.w4 += fxd * (double)dz;
    L.w5 += fyd * (double)dz;
  }
  if (COUNT) ++L.cnt;
}

// Move the adjoint sums of bead i (type ti) into the per-type accumulators.
template <typename T, bool ELEC>
__device__ inline void flush_adj(Lane<T>& L, int ti) {
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
#pragma unroll
    for (int t = 0; t < MAXT; ++t)
      if (q == ti && !ELEC) L.ett[q * MAXT + t] += L.eA[t];
    if (q == ti) L.dsg[q] += L.di;
    L.dsg[q] += L.dj[q];
  }
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    L.eA[q] = 0;
    L.dj[q] = 0;
  }
  L.di = 0;
}

// What a lane needs to evaluate the pairs of its bead i.
template <typename T>
struct PairCtx {
  T sx, sy, sz, rc2, beta, beta2, lB, zi;
  T cexpb, tsb;  // -beta^2 log2(e), (2/sqrt(pi)) beta
  T vx, vy, vz;  // force vector-Jacobian product: v of bead i (adjoint only)
  bool vjp;
  const GcmPar<T>* grow;
  const ElecPar<T>* erow;
  const AdjPar<T>* arow;
};

// The replica's type-pair tables, staged once per workgroup.
template <typename T, bool ELEC, bool ADJ>
struct Tables {
  GcmPar<T> g[ELEC ? 1 : MAXT * MAXT];
  ElecPar<T> e[ELEC ? MAXT * MAXT : 1];
  AdjPar<T> a[ADJ ? MAXT * MAXT : 1];
};

template <typename T, bool ELEC, bool ADJ>
__device__ inline void stage_tables(Tables<T, ELEC, ADJ>& S, const PairLaunch& a, int rep) {
  const size_t tb = (size_t)rep * MAXT * MAXT;
  if (!ELEC && threadIdx.x < MAXT * MAXT) S.g[threadIdx.x] = reinterpret_cast<const GcmPar<T>*>(a.gcm)[tb + threadIdx.x];
  if (ELEC && threadIdx.x < MAXT * MAXT) S.e[threadIdx.x] = reinterpret_cast<const ElecPar<T>*>(a.elec)[tb + threadIdx.x];
  if (ADJ && threadIdx.x < MAXT * MAXT) S.a[threadIdx.x] = reinterpret_cast<const AdjPar<T>*>(a.adj)[tb + threadIdx.x];
  __syncthreads();
}

template <typename T, bool ELEC, bool ADJ>
__device__ inline PairCtx<T> make_ctx(const Tables<T, ELEC, ADJ>& S, const RepDesc& R, uint32_t pi,
                                      const PairLaunch& a, int i) {
  const int ti = param_type(pi);
  PairCtx<T> P;
  P.sx = (T)R.scaled[0];
  P.sy = (T)R.scaled[1];
  P.sz = (T)R.scaled[2];
  P.rc2 = (T)R.rc2;
  P.beta = (T)R.beta;
  P.beta2 = (T)(R.beta * R.beta);
  if constexpr (std::is_same<T, float>::value) {
    // float operations matching the host's for alpha (see build_tables)
    const float bf = (float)R.beta;
    P.cexpb = -(bf * bf) * 1.44269504088896341f;
    P.tsb = 1.12837916709551257f * bf;
  } else {
    P.cexpb = -R.beta * R.beta * 1.4426950408889634;
    P.tsb = 1.1283791670955126 * R.beta;
  }
  P.lB = (T)R.lB;
  P.zi = (T)param_z(pi);
  P.grow = S.g + (ELEC ? 0 : ti * MAXT);
  P.erow = S.e + (ELEC ? ti * MAXT : 0);
  P.arow = S.a + (ADJ ? ti * MAXT : 0);
  P.vjp = false;
  P.vx = P.vy = P.vz = 0;
  if (ADJ && a.vjp) {
    const int fi = ELEC ? a.qidx[i] : i;
    P.vjp = true;
    P.vx = (T)a.vjp[fi];
    P.vy = (T)a.vjp[(size_t)a.nbeads + fi];
    P.vz = (T)a.vjp[2 * (size_t)a.nbeads + fi];
  }
  return P;
}

// Pair (i, j) when ok (j a real bead other than i) and r < rc: separation by
// the exact minimum image in T, the one cutoff test of the method's sums.
template <typename T, bool ELEC, bool EV, bool ADJ, bool COUNT>
__device__ inline void pair_at(Lane<T>& L, const PairCtx<T>& P, T dx, T dy, T dz, uint32_t pw, bool ok) {
  const T r2 = dx * dx + dy * dy + dz * dz;
  const bool in = ok && r2 < P.rc2;
  if (!ELEC && !ADJ && !COUNT) {
    // excluded volume: cheap enough to evaluate for every lane, which keeps
    // the unrolled pairs free of branches; a pair that does not count gets
    // the exponent -inf, hence exactly zero
    const GcmPar<T> g = P.grow[param_type(pw)];
    const T ex = gexp2(in ? -g.bl * r2 : -(T)INFINITY);
    const T fs = g.fC * ex;
    L.fx += fs * dx;
    L.fy += fs * dy;
    L.fz += fs * dz;
    if (EV) {
      const T en = g.C * ex;
      const double fxd = (double)(fs * dx), fyd = (double)(fs * dy), fzd = (double)(fs * dz);
      L.e += (double)en;
      L.w0 += fxd * (double)dx;
      L.w1 += fyd * (double)dy;
      L.w2 += fzd * (double)dz;
      L.w3 += fxd * (double)dy;
      L.w4 += fxd * (double)dz;
      L.w5 += fyd * (double)dz;
    }
  } else if (in) {
    interact<T, ELEC, EV, ADJ, COUNT>(L, dx, dy, dz, r2, pw, P.grow, P.erow, P.arow, P.zi, P.beta, P.beta2, P.lB,
                                      P.vx, P.vy, P.vz, P.vjp, P.cexpb, P.tsb);
  }
}

template <typename T, bool ELEC, bool EV, bool ADJ, bool COUNT>
__device__ inline void try_pair(Lane<T>& L, const PairCtx<T>& P, const uint4& mi, const uint4& pj, bool ok) {
  const T dx = (T)(int)(mi.x - pj.x) * P.sx;
  const T dy = (T)(int)(mi.y - pj.y) * P.sy;
  const T dz = (T)(int)(mi.z - pj.z) * P.sz;
  pair_at<T, ELEC, EV, ADJ, COUNT>(L, P, dx, dy, dz, pj.w, ok);
}

// Combine the partial forces of bead i over its CJ lanes (xor shuffles, fixed
// order) and add them once to the fixed-point accumulator.
template <typename T, int CI, bool ELEC, bool ADJ>
__device__ inline void flush_bead(const PairLaunch& a, Lane<T>& L, bool vi, int i, int ti) {
  constexpr int CJ = 64 / CI;
  const int jl = (threadIdx.x & 63) % CJ;
  if (ADJ && a.dbead) {
    // the bead's own-radius derivative: every bead is in one cluster, so one
    // store per bead, summed over its lanes in a fixed order
    T d = L.di;
#pragma unroll
    for (int o = CJ >> 1; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if (vi && jl == 0) a.dbead[ELEC ? a.qidx[i] : i] = (double)d;
  }
  if (ADJ && vi) flush_adj<T, ELEC>(L, ti);
  T fx = L.fx, fy = L.fy, fz = L.fz;
#pragma unroll
  for (int o = CJ >> 1; o > 0; o >>= 1) {
    fx += __shfl_xor(fx, o, 64);
    fy += __shfl_xor(fy, o, 64);
    fz += __shfl_xor(fz, o, 64);
  }
  if (vi && jl == 0) {
    const int fi = ELEC ? a.qidx[i] : i;
    atomicAdd((unsigned long long*)&a.F[0][fi], (unsigned long long)to_fixed((double)fx, a.fscale, a.status));
    atomicAdd((unsigned long long*)&a.F[1][fi], (unsigned long long)to_fixed((double)fy, a.fscale, a.status));
    atomicAdd((unsigned long long*)&a.F[2][fi], (unsigned long long)to_fixed((double)fz, a.fscale, a.status));
  }
}

// Workgroup partial sums (every pair was seen from both ends: halved).
// Reached by every thread of the workgroup.
template <typename T, bool ELEC, bool EV, bool ADJ, bool COUNT>
__device__ inline void block_outputs(const PairLaunch& a, const Lane<T>& L, double* red, int item) {
  const int lane = threadIdx.x & 63;
  if (COUNT) {
    unsigned long long cc = L.cnt;
    for (int o = 32; o > 0; o >>= 1) cc += __shfl_xor(cc, o, 64);
    if (lane == 0 && cc) atomicAdd(a.pair_count, cc);
  }
  if (EV) {
    double v[7] = {L.e, L.w0, L.w1, L.w2, L.w3, L.w4, L.w5};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      double t = block_sum(v[k], red);
      if (threadIdx.x == 0) a.part[(size_t)item * PART_W + k] = 0.5 * t;
    }
  }
  if (ADJ) {
    constexpr int W = MAXT * MAXT + 2 * MAXT;
    if (!ELEC) {
      for (int q = 0; q < MAXT * MAXT; ++q) {
        double t = block_sum((double)L.ett[q], red);
        if (threadIdx.x == 0) a.adj_part[(size_t)item * W + q] = 0.5 * t;
      }
    }
    for (int t = 0; t < MAXT; ++t) {
      double s = block_sum((double)L.dsg[t], red);
      if (threadIdx.x == 0) a.adj_part[(size_t)item * W + MAXT * MAXT + (ELEC ? MAXT : 0) + t] = 0.5 * s;
    }
  }
}

// List-driven pairs: one wavefront per cluster, lanes = CI beads x 64/CI
// list entries.
template <typename T, int CI, bool ELEC, bool EV, bool ADJ, bool COUNT>
__global__ __launch_bounds__(NL_WAVES * 64) void k_nl_force(PairLaunch a) {
  constexpr int CJ = 64 / CI;
  __shared__ double red[NL_WAVES];
  __shared__ Tables<T, ELEC, ADJ> S;
  wave_stamp(a.stamps, 0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const Tile tl = a.tiles[item];
  const RepDesc& R = a.rep[tl.rep];
  stage_tables(S, a, tl.rep);
  const int il = lane / CJ, jl = lane % CJ;
  Lane<T> L;
  lane_zero(L);
  if (wave < tl.count) {
    const int c = tl.first + wave;
    const int2 info = a.cl[c];
    const int first = info.x, ni = info.y >> 16;
    const bool vi = il < ni;
    const int i = first + (vi ? il : 0);
    const uint4 mi = a.pk[i];
    const PairCtx<T> P = make_ctx(S, R, mi.w, a, i);
    const int cnt = a.count[c];
    const uint32_t* __restrict__ lst = a.list + (size_t)c * a.cap;
    const uint4* __restrict__ pk = a.pk;
    // NU entries per lane per round: the list loads, then the dependent
    // bead-record loads, are issued back to back so one memory latency
    // covers NU pairs
    constexpr int NU = 4;
    for (int e0 = jl; e0 < cnt; e0 += NU * CJ) {
      int jj[NU];
      uint4 pp[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int e = e0 + u * CJ;
        jj[u] = e < cnt ? (int)lst[e] : -1;
      }
#pragma unroll
      for (int u = 0; u < NU; ++u) pp[u] = pk[jj[u] < 0 ? i : jj[u]];
#pragma unroll
      for (int u = 0; u < NU; ++u) try_pair<T, ELEC, EV, ADJ, COUNT>(L, P, mi, pp[u], vi && jj[u] >= 0 && jj[u] != i);
    }
    flush_bead<T, CI, ELEC, ADJ>(a, L, vi, i, param_type(mi.w));
  }
  block_outputs<T, ELEC, EV, ADJ, COUNT>(a, L, red, item);
  wave_stamp(a.stamps, 1);
}

// List-free pairs: one wavefront per cluster enumerates the candidates of
// its cell columns (as the list build does), keeps those within the list
// cutoff of some cluster bead (the list build's test), and evaluates them at
// once from an LDS ring of pending pairs: whenever 64 are pending they are
// taken by the lanes laid out as CI beads x 64/CI entries.  The same pairs
// and cutoff test as the list path, with no list in HBM.
constexpr int RING = 128;  // pending-pair ring per wavefront (entries)
static_assert(RING == 128, "the drain relies on a ring of exactly two 64-entry halves");

// Wavefronts per SIMD the list-free kernel is compiled for: the per-step
// variant (single precision, forces only) is held to 128 VGPRs, so four
// wavefronts share each SIMD instead of three (it then has no spills: the
// excluded-volume pairs of N = 2,097,152 took 1.34 -> 1.08 ms, of N = 32,768
// 48 -> 36 us); the others keep the compiler's choice, since the bound would
// make them spill.
template <typename T, bool EV, bool ADJ, bool COUNT>
struct FusedWaves {
  static constexpr int value = std::is_same<T, float>::value && !EV && !ADJ && !COUNT ? 4 : 1;
};

template <typename T, int CI, bool ELEC, bool EV, bool ADJ, bool COUNT>
__global__ __launch_bounds__(NL_WAVES * 64) __attribute__((amdgpu_waves_per_eu(FusedWaves<T, EV, ADJ, COUNT>::value)))
void k_pair_fused(PairLaunch a) {
  constexpr int CJ = 64 / CI;
  __shared__ double red[NL_WAVES];
  __shared__ Tables<T, ELEC, ADJ> S;
  __shared__ int s_sb[NL_WAVES][NL_SEG];
  __shared__ int s_sl[NL_WAVES][NL_SEG];
  __shared__ int s_cand[NL_WAVES][NL_CAND];
  __shared__ uint4 s_ring[NL_WAVES][RING];
  wave_stamp(a.stamps, 0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const Tile tl = a.tiles[item];
  const RepDesc& R = a.rep[tl.rep];
  const int il = lane / CJ, jl = lane % CJ;
  const uint4* __restrict__ pk = a.pk;
  // this wave's cluster: CI consecutive beads from bead0 + wave CI (the
  // replica's last cluster may be short).  Its records are requested before
  // the tables are staged, so the two loads overlap.
  const bool active = wave < tl.count;
  const int first = tl.bead0 + wave * CI;
  const int ni = active ? min(CI, (ELEC ? R.q_off + R.nq : R.bead_off + R.n) - first) : 1;
  const bool vi = il < ni;
  const int i = first + (vi ? il : 0);
  uint4 me = make_uint4(0u, 0u, 0u, 0u), mi = me;
  if (active) {
    me = pk[first + (lane < ni ? lane : 0)];
    mi = pk[i];
  }
  stage_tables(S, a, tl.rep);
  Lane<T> L;
  lane_zero(L);
  if (active) {
    Cluster<CI> K;
    make_cluster(K, me, R);
    const bool frame = in_frame(K, R);
    const PairCtx<T> P = make_ctx(S, R, mi.w, a, i);
    // Ring records carry, in place of the replica bits, 1 + the cluster slot
    // of a candidate that is itself a cluster bead (0 otherwise).  In single
    // precision with the cluster in bead 0's frame they hold the candidate's
    // position relative to bead 0 as floats (computed once, by the filter),
    // so a pair costs one subtraction per axis; otherwise the fixed-point
    // record, and each pair takes its own minimum image.  (Not for the
    // electrostatics, whose pair cost that would hardly change.)
    constexpr bool REL = std::is_same<T, float>::value && !ELEC && !COUNT;
    const bool rel = REL && frame;
    const float rxi = (float)(int)(mi.x - K.ux[0]) * R.scalef[0];
    const float ryi = (float)(int)(mi.y - K.uy[0]) * R.scalef[1];
    const float rzi = (float)(int)(mi.z - K.uz[0]) * R.scalef[2];
    const uint32_t self = (uint32_t)(il + 1);
    uint4* ring = s_ring[wave];
    // Every slot of both ring halves is written before any drain can read
    // it: in the frame with a record 1e18 away, otherwise with position 0
    // and parameter word 0 (type 0, a valid table index).  No drain variant
    // can then read LDS this wave never wrote.
    {
      const uint32_t far = __float_as_uint(1e18f);
      const uint4 init = rel ? make_uint4(far, far, far, 0u) : make_uint4(0u, 0u, 0u, 0u);
      ring[lane] = init;
      ring[64 + lane] = init;
      __builtin_amdgcn_wave_barrier();
    }
    int head = 0, tail = 0;  // wave-uniform: pairs evaluated / appended
    // evaluate the n <= 64 pending entries from head: lane (il, jl) takes
    // entries jl + k CJ, k < CI.  head is a multiple of 64 here (every drain
    // but the last takes exactly 64), so the entries do not wrap.
    //
    // In the frame, the slots past the last entry of the final drain are
    // filled with a record 1e18 away: the branch-free excluded-volume pair
    // multiplies every lane's separation by its (zero) force factor, so no
    // slot may hold a stale or never-written LDS value (NaN or inf times zero
    // is NaN).  Forces alone (BARE) then need no per-pair validity test: a
    // bead paired with itself has zero separation, so zero force; lanes of
    // missing cluster beads (vi false) are never flushed; and the padding
    // lies beyond the cutoff.
    constexpr bool BARE = REL && !EV && !ADJ;
    auto drain = [&](int n) {
      uint4* base = ring + (head & 64);
      if (rel && n < 64) {
        const uint32_t far = __float_as_uint(1e18f);
        if (lane >= n) base[lane] = make_uint4(far, far, far, 0u);
        __builtin_amdgcn_wave_barrier();
      }
      // the lane's CI entries in groups of at most four (the records of a
      // group are read together; fewer live registers for CI = 8)
      constexpr int G = CI < 4 ? CI : 4;
#pragma unroll
      for (int k0 = 0; k0 < CI; k0 += G) {
        uint4 pp[G];
#pragma unroll
        for (int g = 0; g < G; ++g) pp[g] = base[jl + (k0 + g) * CJ];
        if (rel) {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const int k = k0 + g;
            const T dx = (T)(rxi - __uint_as_float(pp[g].x));
            const T dy = (T)(ryi - __uint_as_float(pp[g].y));
            const T dz = (T)(rzi - __uint_as_float(pp[g].z));
            pair_at<T, ELEC, EV, ADJ, COUNT>(L, P, dx, dy, dz, pp[g].w,
                                             BARE || (vi && jl + k * CJ < n && (pp[g].w >> 16) != self));
          }
        } else {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const int k = k0 + g;
            // slots past the last entry of a final drain may never have been
            // written by this wave (fewer than 64 candidates, as in sparse
            // regions): their parameter word would index the pair tables out
            // of range, so it is replaced by 0 (the positions are integers,
            // always finite, and the pair is masked)
            const bool live = jl + k * CJ < n;
            uint4 q = pp[g];
            q.w = live ? q.w : 0u;
            try_pair<T, ELEC, EV, ADJ, COUNT>(L, P, mi, q, vi && live && (q.w >> 16) != self);
          }
        }
      }
      head += n;
    };
    auto filter = [&](const uint4 pj, bool v, int j) {
      float Dx = 0.f, Dy = 0.f, Dz = 0.f;
      const bool near = frame ? near_frame(K, pj, R, Dx, Dy, Dz) : near_exact(K, pj, R);
      const bool hit = near && v;
      const unsigned long long m = __ballot(hit);
      if (hit) {
        const uint32_t d = (uint32_t)(j - first);
        const uint32_t w = (pj.w & 0xffffu) | ((d < (uint32_t)ni ? d + 1u : 0u) << 16);
        ring[(tail + lanes_below(m)) & (RING - 1)] =
            rel ? make_uint4(__float_as_uint(Dx), __float_as_uint(Dy), __float_as_uint(Dz), w)
                : make_uint4(pj.x, pj.y, pj.z, w);
      }
      tail += __popcll(m);
      __builtin_amdgcn_wave_barrier();
      if (tail - head >= 64) drain(64);
    };
    const int* cand = s_cand[wave];
    for_candidates(K, R, a.start, s_sb[wave], s_sl[wave], s_cand[wave], [&](int total) {
      for_chunks<2>(cand, total, pk, first, filter);
    });
    if (tail > head) drain(tail - head);
    flush_bead<T, CI, ELEC, ADJ>(a, L, vi, i, param_type(mi.w));
  }
  block_outputs<T, ELEC, EV, ADJ, COUNT>(a, L, red, item);
  wave_stamp(a.stamps, 1);
}

// ---------------------------------------------------------------------------
// Half-shell excluded-volume pairs
// ---------------------------------------------------------------------------
//
// One wavefront per column cluster (at most CI consecutive sorted beads of
// one cell column).  Its beads are wave-uniform; each lane takes one
// candidate of the owned columns (for_candidates<HALF>) and evaluates it
// against every cluster bead, so a pair is evaluated once and both beads
// get its force: the cluster beads' sums stay in registers until the end
// (one fixed-order lane reduction), a candidate's goes to the fixed-point
// accumulator after its chunk.  Integer accumulation keeps reruns
// bit-identical whatever the order of the atomics.

// Fixed point of a single-precision force component at `scale`, rounded to
// the nearest integer (ties to even) as llrint would: the fused multiply-add
// with 1.5 2^52 leaves the integer in the low mantissa bits.  Needs
// |f| scale < 2^51 (|f| < lim); beyond, or not finite, the status bit is set
// and 0 returned.
__device__ inline long long fixed_of(float f, double scale, float lim, unsigned int* status) {
  if (!(fabsf(f) < lim)) {
    atomicOr(status, (unsigned)STATUS_FORCE_OVERFLOW);
    return 0;
  }
  return __double_as_longlong(fma((double)f, scale, 6755399441055744.0)) - 0x4338000000000000LL;
}
__device__ inline long long fixed_of(double f, double scale, float, unsigned int* status) {
  return to_fixed(f, scale, status);
}

// DPP lane moves within rows of 16 lanes (all sources valid).
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ inline double dpp_f(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int DPP_ROW_ROR8 = 0x128, DPP_ROW_HALF_MIRROR = 0x141, DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E;

// a + b after exchanging the upper 32 lanes of a with the lower 32 of b
// (lanes 0-31: the sum of a over lanes l and l + 32; lanes 32-63: of b).
__device__ inline float swap32_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// The same within each half for rows of 16 (rows 0, 2: a; rows 1, 3: b).
__device__ inline float swap16_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline double swap32_sum(double a, double b) {
  const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false, false);
  const double p = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  const double q = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
  return p + q;
}
__device__ inline double swap16_sum(double a, double b) {
  const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)y, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false, false);
  const double p = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  const double q = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
  return p + q;
}

// Sums of V per-lane values over the wavefront, in a fixed order: lanes of
// row r (lanes 16 r .. 16 r + 15) end with u[m] = the total of
// v[r V/4 + m], m < V/4.
template <typename T, int V>
__device__ inline void reduce_rows(const T (&v)[V], T (&u)[V / 4]) {
  static_assert(V % 4 == 0, "four rows");
  T w[V / 2];
#pragma unroll
  for (int m = 0; m < V / 2; ++m) w[m] = swap32_sum(v[m], v[m + V / 2]);
#pragma unroll
  for (int m = 0; m < V / 4; ++m) {
    T t = swap16_sum(w[m], w[m + V / 4]);
    t += dpp_f<DPP_ROW_ROR8>(t);
    t += dpp_f<DPP_ROW_HALF_MIRROR>(t);
    t += dpp_f<DPP_XOR1>(t);
    t += dpp_f<DPP_XOR2>(t);
    u[m] = t;
  }
}

// Pair tables of the half-shell kernel: (-bl, fC) and C per type pair.
template <typename T>
struct HalfPar {
  T nb, fc;
};
// Pair tables of the half-shell kernels: excluded volume (-bl, fC) and C per
// type pair, or the real-space bracket's coefficients.
template <typename T, bool ELEC>
struct HalfTab {
  HalfPar<T> p[ELEC ? 1 : MAXT * MAXT];
  T c[ELEC ? 1 : MAXT * MAXT];
  ElecPar<T> e[ELEC ? MAXT * MAXT : 1];
};

// f(integral_constant<int, 0>) ... f(integral_constant<int, N - 1>) in
// order: a loop unrolled whatever the size of its body, so that register
// arrays indexed by the counter stay in registers.
template <class F, int... I>
__device__ __attribute__((always_inline)) inline void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __attribute__((always_inline)) inline void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// A cluster bead as the half-shell kernels read it.
template <typename T>
struct IBead {
  T x, y, z;  // relative to bead 0
  int trow;   // type x MAXT: its row of the pair tables
  T q;        // charge number
};

// ELEC: the charged beads (their compacted records and cell list), the
// real-space bracket of eq. ewald in place of eq. u_ex; forces go to the
// sorted index of each charged bead.
//
// Per cluster: the owned column runs (column_segments<HALF>) are read 64
// consecutive beads at a time, one per lane; a bead within the list cutoff
// of the cluster's bounding box joins a 128-entry LDS ring of pending
// candidates, and every 64 pending candidates are evaluated at once, a lane
// per candidate against every cluster bead.  In the cluster's frame (bead 0's;
// every column cluster in bulk) the ring holds the candidate's position
// relative to bead 0, so a pair costs a subtraction per axis; otherwise the
// fixed-point record, and each pair takes its own minimum image.
//
// HALF false: every column within reach (both ends of each pair; no
// candidate atomics, each pair's energy and virial halved), the same ring
// and evaluation otherwise.
template <typename T, int CI, bool EV, bool ELEC, bool HALF>
__global__ __launch_bounds__(NL_WAVES * 64) void k_pair_col(PairLaunch a) {
  constexpr int NV = 3 * CI;
  __shared__ double red[NL_WAVES];
  __shared__ HalfTab<T, ELEC> S;
  __shared__ int s_sb[NL_WAVES][NL_SEG];
  __shared__ int s_sl[NL_WAVES][NL_SEG];
  __shared__ uint4 s_ring[NL_WAVES][RING];
  __shared__ int s_rj[NL_WAVES][RING];  // candidate index
  __shared__ int s_rf[NL_WAVES][RING];  // its force slot (sorted bead index)
  __shared__ int s_cand[NL_WAVES][NL_CAND];
  __shared__ IBead<T> s_ib[NL_WAVES][ELEC ? 1 : CI];
  wave_stamp(a.stamps, 0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const Tile tl = a.tiles[item];
  const RepDesc& R = a.rep[tl.rep];
  const uint4* __restrict__ pk = a.pk;
  const int slot = tl.first + wave;
  // tl.bead0: the replica's first cluster slot
  const bool active = wave < tl.count && slot - tl.bead0 < a.hncl[tl.rep];
  int2 info = make_int2(0, 1);
  if (active) info = a.cl[slot];
  const int first = info.x, ni = info.y;
  uint4 me = make_uint4(0u, 0u, 0u, 0u);
  if (active) me = pk[first + (lane < ni ? lane : 0)];
  if (threadIdx.x < MAXT * MAXT) {
    const size_t tb = (size_t)tl.rep * MAXT * MAXT + threadIdx.x;
    if (ELEC) {
      S.e[threadIdx.x] = reinterpret_cast<const ElecPar<T>*>(a.elec)[tb];
    } else {
      const GcmPar<T> g = reinterpret_cast<const GcmPar<T>*>(a.gcm)[tb];
      S.p[threadIdx.x] = HalfPar<T>{-g.bl, g.fC};
      S.c[threadIdx.x] = g.C;
    }
  }
  __syncthreads();
  double e = 0, w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0;
  if (active) {
    Cluster<CI> K;
    make_cluster(K, me, R);
    const bool frame = in_frame(K, R);
    const T sx = (T)R.scaled[0], sy = (T)R.scaled[1], sz = (T)R.scaled[2];
    const T rc2 = (T)R.rc2;
    // the real-space bracket's constants (as the cluster kernels take them)
    const T beta = (T)R.beta, beta2 = (T)(R.beta * R.beta), lB = (T)R.lB;
    T cexpb, tsb;
    if constexpr (std::is_same<T, float>::value) {
      const float bf = (float)R.beta;
      cexpb = -(bf * bf) * 1.44269504088896341f;
      tsb = 1.12837916709551257f * bf;
    } else {
      cexpb = -R.beta * R.beta * 1.4426950408889634;
      tsb = 1.1283791670955126 * R.beta;
    }
    // the cluster beads, wave-uniform: positions relative to bead 0, the
    // type row of the pair tables and the charge (slots beyond ni: far from
    // everything, so the unrolled pairs need no branch; the general path
    // masks them)
    // (excluded volume: in LDS, every lane reading the same entry, which
    // keeps the kernel within three wavefronts' registers per SIMD; the
    // charged pairs' branchy bracket keeps them in registers)
    IBead<T> ib[CI];
    IBead<T>* ibl = s_ib[wave];
#pragma unroll
    for (int k = 0; k < CI; ++k) {
      const uint32_t wk = read_lane(me.w, k);
      ib[k].x = k < ni ? (T)(int)(K.ux[k] - K.ux[0]) * sx : (T)1e18f;
      ib[k].y = k < ni ? (T)(int)(K.uy[k] - K.uy[0]) * sy : (T)1e18f;
      ib[k].z = k < ni ? (T)(int)(K.uz[k] - K.uz[0]) * sz : (T)1e18f;
      ib[k].trow = param_type(wk) * MAXT;
      ib[k].q = (T)param_z(wk);
      if (!ELEC && lane == k) ibl[k] = ib[k];
    }
    T fx[CI], fy[CI], fz[CI];
#pragma unroll
    for (int k = 0; k < CI; ++k) fx[k] = fy[k] = fz[k] = 0;
    const float lim = (float)(2251799813685248.0 / a.fscale);  // 2^51 / scale
    const bool rel = std::is_same<T, float>::value && frame;
    uint4* ring = s_ring[wave];
    int* rj = s_rj[wave];
    int* rf = s_rf[wave];
    // every slot of the ring is written before a drain can read it
    ring[lane] = ring[64 + lane] = make_uint4(0u, 0u, 0u, 0u);
    rj[lane] = rj[64 + lane] = -1;
    rf[lane] = rf[64 + lane] = 0;
    __builtin_amdgcn_wave_barrier();
    int head = 0, tail = 0;  // wave-uniform: candidates evaluated / appended
    // n <= 64 pending candidates from head, one per lane (head is a multiple
    // of 64 here: every drain but the last takes exactly 64).  FRAME: ring
    // positions relative to bead 0; MASK: the drain holds cluster beads,
    // whose pairs with the cluster count only for k < j - first.
    auto drain = [&](int n) __attribute__((always_inline)) {
      const int q = (head & 64) + lane;
      const bool valid = lane < n;
      const uint4 rec = ring[q];
      const int j = valid ? rj[q] : -1;
      const int fj = rf[q];
      const unsigned jrel = j < 0 ? 0u : (unsigned)(j - first);
      const bool intra = __ballot(j >= 0 && jrel < (unsigned)ni) != 0ull;
      auto eval = [&](auto frame_tag, auto mask_tag) __attribute__((always_inline)) {
        constexpr bool FR = decltype(frame_tag)::value, MASK = decltype(mask_tag)::value;
        T Dx = 0, Dy = 0, Dz = 0;
        if (FR) {
          if (std::is_same<T, float>::value) {
            Dx = (T)__uint_as_float(rec.x);
            Dy = (T)__uint_as_float(rec.y);
            Dz = (T)__uint_as_float(rec.z);
          } else {
            Dx = (T)(int)(rec.x - K.ux[0]) * sx;
            Dy = (T)(int)(rec.y - K.uy[0]) * sy;
            Dz = (T)(int)(rec.z - K.uz[0]) * sz;
          }
          if (!valid) Dx = Dy = Dz = (T)-1e18f;  // beyond the cutoff of every bead
        }
        const int tj = param_type(rec.w);
        const T qj = (T)param_z(rec.w);
        T gx = 0, gy = 0, gz = 0;
        bool any = false;
        static_for<CI>([&](auto kc) __attribute__((always_inline)) {
          constexpr int k = decltype(kc)::value;
          const IBead<T> bi = ELEC ? ib[k] : ibl[k];
          T dx, dy, dz;
          if (FR) {
            dx = bi.x - Dx;
            dy = bi.y - Dy;
            dz = bi.z - Dz;
          } else {
            dx = (T)(int)(K.ux[k] - rec.x) * sx;
            dy = (T)(int)(K.uy[k] - rec.y) * sy;
            dz = (T)(int)(K.uz[k] - rec.z) * sz;
          }
          const T r2 = dx * dx + dy * dy + dz * dz;
          bool in = r2 < rc2;
          // half shell: within the cluster, pairs (k, j) with k < j; both
          // ends: every cluster bead but the candidate itself
          if (MASK || !FR) in = in && (HALF ? jrel > (unsigned)k : jrel != (unsigned)k);
          if (!FR) in = in && k < ni && valid;
          const int ix = bi.trow + tj;
          T fs = 0, en = 0;
          if (ELEC) {
            if (in) {
              T phi, g, ea;
              bracket(S.e[ix], r2, beta, beta2, cexpb, tsb, phi, g, ea);
              const T c = lB * (bi.q * qj);
              fs = c * g;
              en = c * phi;
            }
          } else {
            const HalfPar<T> hp = S.p[ix];
            const T ex = gexp2(in ? hp.nb * r2 : -(T)INFINITY);
            fs = hp.fc * ex;
            en = EV ? S.c[ix] * ex : (T)0;
          }
          // the candidate's sum is kept with the cluster bead's sign and
          // negated once: two fused multiply-adds per axis
          fx[k] = fma(fs, dx, fx[k]);
          fy[k] = fma(fs, dy, fy[k]);
          fz[k] = fma(fs, dz, fz[k]);
          gx = fma(fs, dx, gx);
          gy = fma(fs, dy, gy);
          gz = fma(fs, dz, gz);
          any = any || in;
          if (EV) {
            const double fxd = (double)(fs * dx), fyd = (double)(fs * dy), fzd = (double)(fs * dz);
            e += (double)en;
            w0 += fxd * (double)dx;
            w1 += fyd * (double)dy;
            w2 += fzd * (double)dz;
            w3 += fxd * (double)dy;
            w4 += fxd * (double)dz;
            w5 += fyd * (double)dz;
          }
        });
        if (HALF && j >= 0 && any) {
          atomicAdd((unsigned long long*)&a.F[0][fj], (unsigned long long)fixed_of(-gx, a.fscale, lim, a.status));
          atomicAdd((unsigned long long*)&a.F[1][fj], (unsigned long long)fixed_of(-gy, a.fscale, lim, a.status));
          atomicAdd((unsigned long long*)&a.F[2][fj], (unsigned long long)fixed_of(-gz, a.fscale, lim, a.status));
        }
      };
      using TT = std::true_type;
      using FF = std::false_type;
      if (!frame)
        eval(FF{}, TT{});
      else if (intra)
        eval(TT{}, TT{});
      else
        eval(TT{}, FF{});
      head += n;
    };
    // the list cutoff around the cluster's bounding box (relative to bead 0)
    const float rcl2 = K.rcl * K.rcl;
    int* cand = s_cand[wave];
    // the candidates cand[0, total), 64 per chunk (one per lane): those within
    // the list cutoff of the box join the ring
    auto filter = [&](int total) __attribute__((always_inline)) {
      // the records of FB chunks are requested together (one memory latency
      // for all of them), and the charged beads' sorted indices with them
      constexpr int FB = 4;
      for (int p0 = 0; p0 < total; p0 += 64 * FB) {
        int jj[FB], ff[FB];
        uint4 pp[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) {
          const int q = p0 + 64 * u + lane;
          jj[u] = q < total ? cand[q] : -1;
        }
#pragma unroll
        for (int u = 0; u < FB; ++u) {
          pp[u] = pk[jj[u] < 0 ? first : jj[u]];
          ff[u] = ELEC ? a.qidx[jj[u] < 0 ? first : jj[u]] : jj[u];
        }
#pragma unroll
        for (int u = 0; u < FB; ++u) {
          if (p0 + 64 * u >= total) break;
          const int j = jj[u];
          const bool valid = j >= 0;
          const uint4 pj = pp[u];
          bool hit;
          uint4 rec = pj;
          if (frame) {
            const float Dx = (float)(int)(pj.x - K.ux[0]) * R.scalef[0];
            const float Dy = (float)(int)(pj.y - K.uy[0]) * R.scalef[1];
            const float Dz = (float)(int)(pj.z - K.uz[0]) * R.scalef[2];
            const float bx = fmaxf(0.f, fmaxf(K.lo[0] - Dx, Dx - K.hi[0]));
            const float by = fmaxf(0.f, fmaxf(K.lo[1] - Dy, Dy - K.hi[1]));
            const float bz = fmaxf(0.f, fmaxf(K.lo[2] - Dz, Dz - K.hi[2]));
            hit = valid && bx * bx + by * by + bz * bz < rcl2;
            if (rel) rec = make_uint4(__float_as_uint(Dx), __float_as_uint(Dy), __float_as_uint(Dz), pj.w);
          } else {
            hit = valid && near_exact(K, pj, R);
          }
          const unsigned long long m = __ballot(hit);
          if (hit) {
            const int q = (tail + lanes_below(m)) & (RING - 1);
            ring[q] = rec;
            rj[q] = j;
            rf[q] = ff[u];
          }
          tail += __popcll(m);
          __builtin_amdgcn_wave_barrier();
          if (tail - head >= 64) drain(64);
          __builtin_amdgcn_wave_barrier();
        }
      }
    };
    const int ncol = (K.chi[0] - K.clo[0] + 1) * (K.chi[1] - K.clo[1] + 1);
    for (int cbase = 0; cbase < ncol; cbase += 64) {
      const int nseg = column_segments<CI, HALF>(K, R, a.start, first, cbase, s_sb[wave], s_sl[wave]);
      // the owned column runs packed into the candidate buffer (filtered
      // whenever it fills), so that filter chunks are full
      int pos = 0;
      for (int sg = 0; sg < nseg; ++sg) {
        const int sb = __builtin_amdgcn_readfirstlane(s_sb[wave][sg]);
        const int sl = __builtin_amdgcn_readfirstlane(s_sl[wave][sg]);
        for (int off = 0; off < sl;) {
          const int take = min(sl - off, NL_CAND - pos);
          for (int t = lane; t < take; t += 64) cand[pos + t] = sb + off + t;
          pos += take;
          off += take;
          __builtin_amdgcn_wave_barrier();
          if (pos == NL_CAND) {
            filter(pos);
            pos = 0;
          }
        }
      }
      if (pos > 0) filter(pos);
    }
    if (tail > head) drain(tail - head);
    // the cluster beads' sums: row r of the wavefront holds beads
    // r CI/4 .. r CI/4 + CI/4 - 1 (CI/4 beads x 3 axes per row)
    T v[NV], u[NV / 4];
#pragma unroll
    for (int k = 0; k < CI; ++k) {
      v[3 * k] = fx[k];
      v[3 * k + 1] = fy[k];
      v[3 * k + 2] = fz[k];
    }
    reduce_rows<T, NV>(v, u);
    const int row = lane >> 4, t = lane & 15;
    if (t < CI / 4) {
      T f3[3] = {0, 0, 0};
#pragma unroll
      for (int b = 0; b < CI / 4; ++b)
        if (t == b) {
          f3[0] = u[3 * b];
          f3[1] = u[3 * b + 1];
          f3[2] = u[3 * b + 2];
        }
      const int k = row * (CI / 4) + t;
      if (k < ni) {
        const int fi = ELEC ? a.qidx[first + k] : first + k;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          atomicAdd((unsigned long long*)&a.F[c][fi],
                    (unsigned long long)fixed_of(f3[c], a.fscale, lim, a.status));
      }
    }
  }
  if (EV) {
    // half shell: every pair once; both ends: twice, halved
    double v7[7] = {e, w0, w1, w2, w3, w4, w5};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const double t = block_sum(v7[k], red);
      if (threadIdx.x == 0) a.part[(size_t)item * PART_W + k] = HALF ? t : 0.5 * t;
    }
  }
  wave_stamp(a.stamps, 1);
}

template <typename T, int CI, bool ELEC, bool EV, bool ADJ, bool COUNT>
void launch_one(hipStream_t s, const PairLaunch& a) {
  dim3 g(a.ntiles), b(NL_WAVES * 64);
  if (a.direct)
    hipLaunchKernelGGL((k_pair_fused<T, CI, ELEC, EV, ADJ, COUNT>), g, b, 0, s, a);
  else
    hipLaunchKernelGGL((k_nl_force<T, CI, ELEC, EV, ADJ, COUNT>), g, b, 0, s, a);
}

template <typename T, int CI, bool ELEC>
void dispatch_mode(hipStream_t s, const PairLaunch& a, bool ev, bool adj, bool count) {
  if (count)
    launch_one<T, CI, ELEC, false, false, true>(s, a);
  else if (adj)
    launch_one<T, CI, ELEC, true, true, false>(s, a);
  else if (ev)
    launch_one<T, CI, ELEC, true, false, false>(s, a);
  else
    launch_one<T, CI, ELEC, false, false, false>(s, a);
}

template <typename T, bool ELEC>
void dispatch_ci(hipStream_t s, const PairLaunch& a, bool ev, bool adj, bool count) {
  switch (a.ci) {
    case 2: dispatch_mode<T, 2, ELEC>(s, a, ev, adj, count); break;
    case 8: dispatch_mode<T, 8, ELEC>(s, a, ev, adj, count); break;
    default: dispatch_mode<T, 4, ELEC>(s, a, ev, adj, count); break;
  }
}

}  // namespace

void launch_nl_build(hipStream_t s, const PairLaunch& a) {
  if (a.ncl <= 0 || a.direct) return;
  dim3 g((a.ncl + NL_WAVES - 1) / NL_WAVES), b(NL_WAVES * 64);
  switch (a.ci) {
    case 2: hipLaunchKernelGGL(k_nl_build<2>, g, b, 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_nl_build<8>, g, b, 0, s, a); break;
    default: hipLaunchKernelGGL(k_nl_build<4>, g, b, 0, s, a); break;
  }
}

void launch_pair_gcm(hipStream_t s, const PairLaunch& a, bool fp64, bool ev, bool adjoint) {
  if (a.ntiles <= 0) return;
  bool count = a.pair_count != nullptr;
  if (fp64)
    dispatch_ci<double, false>(s, a, ev, adjoint, count);
  else
    dispatch_ci<float, false>(s, a, ev, adjoint, count);
}

void launch_pair_elec(hipStream_t s, const PairLaunch& a, bool fp64, bool ev, bool adjoint) {
  if (a.ntiles <= 0) return;
  if (fp64)
    dispatch_ci<double, true>(s, a, ev, adjoint, false);
  else
    dispatch_ci<float, true>(s, a, ev, adjoint, false);
}

template <bool ELEC>
void launch_col(hipStream_t s, const PairLaunch& a, bool fp64, bool ev, bool half) {
  if (a.ntiles <= 0) return;
  dim3 g(a.ntiles), b(NL_WAVES * 64);
#define GCME_COL(T, CI, H)                                                        \
  do {                                                                             \
    if (ev)                                                                        \
      hipLaunchKernelGGL((k_pair_col<T, CI, true, ELEC, H>), g, b, 0, s, a);      \
    else                                                                           \
      hipLaunchKernelGGL((k_pair_col<T, CI, false, ELEC, H>), g, b, 0, s, a);     \
  } while (0)
#define GCME_COL_H(T, CI) \
  do {                    \
    if (half)             \
      GCME_COL(T, CI, true); \
    else                  \
      GCME_COL(T, CI, false); \
  } while (0)
  if (fp64) {
    if (a.ci == 8)
      GCME_COL_H(double, 8);
    else
      GCME_COL_H(double, 4);
  } else {
    if (a.ci == 8)
      GCME_COL_H(float, 8);
    else
      GCME_COL_H(float, 4);
  }
#undef GCME_COL_H
#undef GCME_COL
}

void launch_pair_gcm_col(hipStream_t s, const PairLaunch& a, bool fp64, bool ev, bool half) {
  launch_col<false>(s, a, fp64, ev, half);
}

void launch_pair_elec_col(hipStream_t s, const PairLaunch& a, bool fp64, bool ev, bool half) {
  launch_col<true>(s, a, fp64, ev, half);
}

int pair_waves_per_block() { return NL_WAVES; }

}  // namespace gcme
