// Cutoff pair kernels.
//
//  * excluded volume: eq. u_ex for every pair within rc (all beads);
//  * real-space electrostatics: the bracket of eq. ewald,
//    lB z_i z_j [erf(alpha_ij r) - erf(beta r)]/r, over the charged beads only
//    (their own cell list and compacted arrays), so the transcendental-heavy
//    term costs nothing for neutral beads and the kernels never branch on
//    charge.
//
// Both run in two launches per evaluation over "clusters": CI consecutive
// beads of the cell-sorted order (CI = 2, 4 or 8; spatially compact because
// the order is by cell).
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
// Lists are rebuilt every evaluation, so they need no skin.  The minimum
// image is the wrapped 32-bit difference of the fractional fixed-point
// coordinates (valid because rc <= L/2 is enforced).
#include "gcme_internal.h"

namespace gcme {

namespace {

__device__ inline float gexp2(float x) { return exp2f(x); }
__device__ inline double gexp2(double x) { return exp2(x); }
__device__ inline float gexp(float x) { return expf(x); }
__device__ inline double gexp(double x) { return exp(x); }
__device__ inline float gerfc(float x) { return erfcf(x); }
__device__ inline double gerfc(double x) { return erfc(x); }
__device__ inline float gsqrt(float x) { return sqrtf(x); }
__device__ inline double gsqrt(double x) { return sqrt(x); }

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
// List build
// ---------------------------------------------------------------------------

template <int CI>
__global__ __launch_bounds__(NL_WAVES * 64) void k_nl_build(PairLaunch a) {
  __shared__ int s_sb[NL_WAVES][NL_SEG];
  __shared__ int s_sl[NL_WAVES][NL_SEG];
  __shared__ int s_cand[NL_WAVES][NL_CAND];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * NL_WAVES + wave;
  if (c >= a.ncl) return;  // whole wavefront; no block barriers below
  const int2 info = a.cl[c];
  const int first = info.x, rep = info.y & 0xffff, ni = info.y >> 16;
  const RepDesc& R = a.rep[rep];
  const int* __restrict__ start = a.start;
  const uint4* __restrict__ pk = a.pk;

  // cluster beads, as wave-uniform values (slots beyond ni repeat bead 0)
  const int mine = first + (lane < ni ? lane : 0);
  const uint4 me = pk[mine];
  const uint32_t ux = me.x, uy = me.y, uz = me.z;
  uint32_t cxs[CI], cys[CI], czs[CI];
#pragma unroll
  for (int k = 0; k < CI; ++k) {
    cxs[k] = read_lane(ux, k);
    cys[k] = read_lane(uy, k);
    czs[k] = read_lane(uz, k);
  }
  // Cluster geometry in float, relative to the lower corner of bead 0's cell:
  // every value is a few cells at most, so float carries it to ~1e-7 of a
  // cell, and the margin dl keeps each cell range conservative.
  float rfx[CI], rfy[CI], rfz[CI];
#pragma unroll
  for (int k = 0; k < CI; ++k) {
    rfx[k] = (float)(int)(cxs[k] - cxs[0]) * R.scalef[0];
    rfy[k] = (float)(int)(cys[k] - cys[0]) * R.scalef[1];
    rfz[k] = (float)(int)(czs[k] - czs[0]) * R.scalef[2];
  }
  float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 1; k < CI; ++k) {
    lo[0] = fminf(lo[0], rfx[k]);
    hi[0] = fmaxf(hi[0], rfx[k]);
    lo[1] = fminf(lo[1], rfy[k]);
    hi[1] = fmaxf(hi[1], rfy[k]);
    lo[2] = fminf(lo[2], rfz[k]);
    hi[2] = fmaxf(hi[2], rfz[k]);
  }
  const uint32_t u0[3] = {cxs[0], cys[0], czs[0]};
  int c0[3];
  float p0[3], h[3], ih[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const unsigned long long pp = (unsigned long long)u0[k] * (unsigned)R.nc[k];
    c0[k] = (int)(pp >> 32);
    h[k] = R.hf[k];
    ih[k] = 1.0f / h[k];
    p0[k] = (float)(uint32_t)(pp & 0xffffffffu) * 2.3283064365386963e-10f * h[k];
  }
  // list cutoff: a hair above rc, so the float test below never drops a pair
  // the force kernel's own test (in its precision) would keep
  const float rcl = (float)(R.rc * (1.0 + 1e-5));
  const float rcl2f = rcl * rcl;
  const float dl = 1e-4f * fmaxf(h[0], fmaxf(h[1], h[2]));
  const float rclm = rcl + dl;
  int clo[3], chi[3];  // cell ranges relative to c0 (absolute when whole)
  bool whole[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    clo[k] = (int)floorf((p0[k] + lo[k] - rclm) * ih[k]);
    chi[k] = (int)floorf((p0[k] + hi[k] + rclm) * ih[k]);
    whole[k] = chi[k] - clo[k] + 1 >= R.nc[k];
    if (whole[k]) {
      clo[k] = 0;
      chi[k] = R.nc[k] - 1;
    }
  }
  // In the frame of bead 0, separations equal the per-pair minimum image for
  // every pair within rc as long as each cluster bead lies within L/2 - rc of
  // bead 0 on each axis (then |d| < rc cannot wrap); otherwise the test
  // takes the minimum image of each pair.
  bool frame = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) frame = frame && fmaxf(-lo[k], hi[k]) < 0.5f * (float)R.L[k] - rclm;
  const int nx = R.nc[0], ny = R.nc[1], nz = R.nc[2];
  const int ncx = chi[0] - clo[0] + 1, ncy = chi[1] - clo[1] + 1;
  const int ncol = ncx * ncy;
  const float sx = R.scalef[0], sy = R.scalef[1], sz = R.scalef[2];
  uint32_t* __restrict__ out = a.list + (size_t)c * a.cap;
  int nent = 0;

  for (int cbase = 0; cbase < ncol; cbase += 64) {
    // 1. this lane's column: culled, z run clipped, as up to two bead ranges
    int b0[2] = {0, 0}, ln[2] = {0, 0};
    const int k = cbase + lane;
    if (k < ncol) {
      const int rx = clo[0] + k / ncy, ry = clo[1] + k % ncy;
      // distance from the column to the bounding box in x and y
      const float gx = whole[0] ? 0.f : fmaxf(0.f, fmaxf(rx * h[0] - (p0[0] + hi[0]), (p0[0] + lo[0]) - (rx + 1) * h[0]));
      const float gy = whole[1] ? 0.f : fmaxf(0.f, fmaxf(ry * h[1] - (p0[1] + hi[1]), (p0[1] + lo[1]) - (ry + 1) * h[1]));
      const float d2 = gx * gx + gy * gy;
      if (d2 < rclm * rclm) {
        int cx = whole[0] ? rx : c0[0] + rx;
        int cy = whole[1] ? ry : c0[1] + ry;
        cx += cx < 0 ? nx : (cx >= nx ? -nx : 0);
        cy += cy < 0 ? ny : (cy >= ny ? -ny : 0);
        int zlo = 0, zhi = nz - 1;
        if (!whole[2]) {
          const float zr = sqrtf(rclm * rclm - d2);
          zlo = c0[2] + (int)floorf((p0[2] + lo[2] - zr) * ih[2]);
          zhi = c0[2] + (int)floorf((p0[2] + hi[2] + zr) * ih[2]);
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
      }
    }
    // 2. compact the non-empty ranges into the wave's LDS segment list
    int nseg = 0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const bool has = ln[q] > 0;
      const unsigned long long m = __ballot(has);
      if (has) {
        const int p = nseg + lanes_below(m);
        s_sb[wave][p] = b0[q];
        s_sl[wave][p] = ln[q];
      }
      nseg += __popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    // 3. expand segments into the candidate buffer (a segment too long for
    //    the room left is split across rounds), then test the candidates
    int sn = 0, soff = 0;
    while (sn < nseg) {
      const int s = sn + lane;
      int sb = 0, sl = 0;
      if (s < nseg) {
        sb = s_sb[wave][s];
        sl = s_sl[wave][s];
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
        if (t < take) s_cand[wave][exc + t] = sb + t;
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
      // test one candidate per lane against every cluster bead; hits are
      // appended in candidate order
      auto test = [&](const uint4 pj, bool v, int j) {
        bool hit = false;
        if (frame) {
          // candidate relative to bead 0 once, then one subtraction per bead
          const float Dx = (float)(int)(pj.x - cxs[0]) * sx;
          const float Dy = (float)(int)(pj.y - cys[0]) * sy;
          const float Dz = (float)(int)(pj.z - czs[0]) * sz;
#pragma unroll
          for (int i = 0; i < CI; ++i) {
            const float dx = Dx - rfx[i], dy = Dy - rfy[i], dz = Dz - rfz[i];
            hit |= dx * dx + dy * dy + dz * dz < rcl2f;
          }
        } else {
#pragma unroll
          for (int i = 0; i < CI; ++i) {
            const float dx = (float)(int)(cxs[i] - pj.x) * sx;
            const float dy = (float)(int)(cys[i] - pj.y) * sy;
            const float dz = (float)(int)(czs[i] - pj.z) * sz;
            hit |= dx * dx + dy * dy + dz * dz < rcl2f;
          }
        }
        hit = hit && v;
        const unsigned long long m = __ballot(hit);
        if (hit) {
          const int idx = nent + lanes_below(m);
          if (idx < a.cap) out[idx] = (uint32_t)j;
        }
        nent += __popcll(m);
      };
      // two chunks per round, their loads issued together
      for (int p = 0; p < total; p += 128) {
        const int q0 = p + lane, q1 = p + 64 + lane;
        const bool v0 = q0 < total, v1 = q1 < total;
        const int j0 = v0 ? s_cand[wave][q0] : first;
        const int j1 = v1 ? s_cand[wave][q1] : first;
        const uint4 p0 = pk[j0];
        const uint4 p1 = pk[j1];
        test(p0, v0, j0);
        if (p + 64 < total) test(p1, v1, j1);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (lane == 0) {
    a.count[c] = min(nent, a.cap);
    if (nent > a.cap) atomicOr(a.status, (unsigned)STATUS_LIST_OVERFLOW);
  }
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

// One ordered pair (i, j) with separation d = r_i - r_j, r2 < rc^2.
template <typename T, bool ELEC, bool EV, bool ADJ, bool COUNT>
__device__ inline void interact(Lane<T>& L, T dx, T dy, T dz, T r2, uint32_t pj, const GcmPar<T>* grow,
                                const ElecPar<T>* erow, const AdjPar<T>* arow, T zi, T beta, T beta2, T lB) {
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
      L.di += duds * ap.dsig_i;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        if (t == tj) {
          L.eA[t] += en;
          L.dj[t] += duds * ap.dsig_j;
        }
      }
    }
  } else {
    constexpr T TSP = (T)1.1283791670955126;  // 2/sqrt(pi)
    const ElecPar<T>& p = erow[tj];
    const T zz = zi * (T)param_z(pj);
    T phi, g;
    if (r2 < p.rs2) {
      // series in r^2, free of the cancellation near contact
      phi = p.cphi[Series<T>::n - 1];
      g = p.cg[Series<T>::n - 1];
#pragma unroll
      for (int n = Series<T>::n - 2; n >= 0; --n) {
        phi = phi * r2 + p.cphi[n];
        g = g * r2 + p.cg[n];
      }
    } else {
      T r = gsqrt(r2);
      T rinv = (T)1 / r;
      phi = (gerfc(beta * r) - gerfc(p.alpha * r)) * rinv;
      g = (phi - TSP * (p.alpha * gexp(-p.alpha2 * r2) - beta * gexp(-beta2 * r2))) * rinv * rinv;
    }
    fs = lB * zz * g;
    en = lB * zz * phi;
    if (ADJ) {
      const AdjPar<T> ap = arow[tj];
      // d/da_ij of lB zz erf(alpha r)/r = -lB zz (2/sqrt(pi)) (alpha/a_ij) exp(-alpha^2 r^2)
      T dd = -lB * zz * ap.ea * gexp(-p.alpha2 * r2);
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

template <typename T, int CI, bool ELEC, bool EV, bool ADJ, bool COUNT>
__global__ __launch_bounds__(NL_WAVES * 64) void k_nl_force(PairLaunch a) {
  constexpr int CJ = 64 / CI;
  __shared__ double red[NL_WAVES];
  // the replica's type-pair tables, staged once per workgroup
  __shared__ GcmPar<T> s_g[ELEC ? 1 : MAXT * MAXT];
  __shared__ ElecPar<T> s_e[ELEC ? MAXT * MAXT : 1];
  __shared__ AdjPar<T> s_a[ADJ ? MAXT * MAXT : 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const Tile tl = a.tiles[blockIdx.x];
  const RepDesc& R = a.rep[tl.rep];
  {
    const size_t tb = (size_t)tl.rep * MAXT * MAXT;
    if (!ELEC && threadIdx.x < MAXT * MAXT) s_g[threadIdx.x] = reinterpret_cast<const GcmPar<T>*>(a.gcm)[tb + threadIdx.x];
    if (ELEC && threadIdx.x < MAXT * MAXT) s_e[threadIdx.x] = reinterpret_cast<const ElecPar<T>*>(a.elec)[tb + threadIdx.x];
    if (ADJ && threadIdx.x < MAXT * MAXT) s_a[threadIdx.x] = reinterpret_cast<const AdjPar<T>*>(a.adj)[tb + threadIdx.x];
    __syncthreads();
  }
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
    const uint32_t pi = mi.w;
    const int ti = param_type(pi);
    const T zi = (T)param_z(pi);
    const GcmPar<T>* grow = s_g + (ELEC ? 0 : ti * MAXT);
    const ElecPar<T>* erow = s_e + (ELEC ? ti * MAXT : 0);
    const AdjPar<T>* arow = s_a + (ADJ ? ti * MAXT : 0);
    const T sx = (T)R.scaled[0], sy = (T)R.scaled[1], sz = (T)R.scaled[2];
    const T rc2 = (T)R.rc2;
    const T beta = (T)R.beta, beta2 = (T)(R.beta * R.beta), lB = (T)R.lB;
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
      for (int u = 0; u < NU; ++u) {
        const uint4 pj = pp[u];
        const T dx = (T)(int)(mi.x - pj.x) * sx;
        const T dy = (T)(int)(mi.y - pj.y) * sy;
        const T dz = (T)(int)(mi.z - pj.z) * sz;
        const T r2 = dx * dx + dy * dy + dz * dz;
        if (vi && jj[u] >= 0 && r2 < rc2 && jj[u] != i)
          interact<T, ELEC, EV, ADJ, COUNT>(L, dx, dy, dz, r2, pj.w, grow, erow, arow, zi, beta, beta2, lB);
      }
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
      if (threadIdx.x == 0) a.part[(size_t)blockIdx.x * PART_W + k] = 0.5 * t;
    }
  }
  if (ADJ) {
    constexpr int W = MAXT * MAXT + 2 * MAXT;
    if (!ELEC) {
      for (int q = 0; q < MAXT * MAXT; ++q) {
        double t = block_sum((double)L.ett[q], red);
        if (threadIdx.x == 0) a.adj_part[(size_t)blockIdx.x * W + q] = 0.5 * t;
      }
    }
    for (int t = 0; t < MAXT; ++t) {
      double s = block_sum((double)L.dsg[t], red);
      if (threadIdx.x == 0) a.adj_part[(size_t)blockIdx.x * W + MAXT * MAXT + (ELEC ? MAXT : 0) + t] = 0.5 * s;
    }
  }
}

template <typename T, int CI, bool ELEC>
void dispatch_mode(hipStream_t s, const PairLaunch& a, bool ev, bool adj, bool count) {
  dim3 g(a.ntiles), b(NL_WAVES * 64);
  if (count)
    hipLaunchKernelGGL((k_nl_force<T, CI, ELEC, false, false, true>), g, b, 0, s, a);
  else if (adj)
    hipLaunchKernelGGL((k_nl_force<T, CI, ELEC, true, true, false>), g, b, 0, s, a);
  else if (ev)
    hipLaunchKernelGGL((k_nl_force<T, CI, ELEC, true, false, false>), g, b, 0, s, a);
  else
    hipLaunchKernelGGL((k_nl_force<T, CI, ELEC, false, false, false>), g, b, 0, s, a);
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
  if (a.ncl <= 0) return;
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

int pair_waves_per_block() { return NL_WAVES; }

}  // namespace gcme
