// Cutoff pair kernels.
//
//  * excluded volume: eq. u_ex for every pair within rc (all beads);
//  * real-space electrostatics: the bracket of eq. ewald,
//    lB z_i z_j [erf(alpha_ij r) - erf(beta r)]/r, over the charged beads only
//    (their own cell list), so the transcendental-heavy term costs nothing for
//    neutral beads and the kernels never branch on charge.
//
// One workgroup takes a brick of cells.  It first stages the brick's cutoff
// neighbourhood -- every cell within reach, with the periodic image shift of
// each cell applied -- into LDS, as coordinates relative to the brick corner
// (so no per-pair minimum image is needed, and boxes smaller than the
// neighbourhood work unchanged: a bead may appear at several images, and with
// rc <= L/2 at most one of them lies within rc).  In the mixed-precision
// kernels the staged coordinates are 32-bit integers in units of
// max(cell edge)/2^26, so separations are exact integer differences and
// float rounding enters only once (a float offset from the corner would carry
// an absolute error of its own ulp, too coarse for 1e-6 energies).
//
// TPA lanes share one home bead.  They first compute, cooperatively, the
// bead's culled column ranges (columns dropped by the exact distance from the
// bead to the column, z runs clipped to the cutoff sphere; each run is one
// contiguous LDS range) into an LDS list, then walk the list with a balanced
// interleave (candidate c of the concatenated ranges goes to lane c mod TPA).
// Every pair is visited from both ends (no scatter of forces to j); the TPA
// partial forces are combined with xor shuffles in a fixed order and added
// once to the 64-bit fixed-point accumulator.  A neighbourhood that does not
// fit in LDS falls back to the same walk over global memory.
#include <map>
#include <mutex>

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

// Staged bead: position relative to the brick corner, parameter word.
template <typename T>
struct StageRec;
template <>
struct StageRec<float> {
  int x, y, z;  // units of max(cell edge) / 2^26
  uint32_t p;
};
template <>
struct StageRec<double> {
  double x, y, z;
  uint32_t p, pad;
};

constexpr double STAGE_FRAC = 67108864.0;  // 2^26

template <typename T>
__device__ inline T lane_reduce(T v, int tpa) {
  for (int o = tpa >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum over the block (up to 16 waves); result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0) {
    int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) t += sh[w];
  }
  return t;
}

// Inclusive scan of one int per thread over the block (up to 16 waves).
__device__ inline int block_inclusive_scan(int v, int* sh) {
  int lane = threadIdx.x & 63;
  int wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  __syncthreads();
  if (lane == 63) sh[wid] = v;
  __syncthreads();
  int add = 0;
  for (int w = 0; w < wid; ++w) add += sh[w];
  return v + add;
}

__device__ inline long long to_fixed(double f, double scale, unsigned int* status) {
  double v = f * scale;
  if (!(fabs(v) < 4.0e18)) {
    atomicOr(status, (unsigned)STATUS_FORCE_OVERFLOW);
    return 0;
  }
  return (long long)llrint(v);
}

__device__ inline int wrap_cell(int c, int n, int& shift) {
  int q = c >= 0 ? c / n : -((-c + n - 1) / n);
  shift = q;
  return c - q * n;
}

// Global-memory walk of the cutoff neighbourhood of bead i (fixed-point
// position u): calls f(j) for every candidate j (j may be i).  Used when a
// brick's neighbourhood does not fit in LDS.
template <int TPA, typename F>
__device__ inline void for_each_candidate(const RepDesc& R, const uint32_t u[3], const int* __restrict__ start,
                                          int sub, F&& f) {
  int c[3];
  float off[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    unsigned long long p = (unsigned long long)u[k] * (unsigned)R.nc[k];
    c[k] = (int)(p >> 32);
    off[k] = (float)(uint32_t)(p & 0xffffffffu) * 2.3283064365386963e-10f;
  }
  const float rcc = sqrtf(R.rc2f) * 1.0001f + 1e-6f;
  const float rcc2 = rcc * rcc;
  const int nx = R.nc[0], ny = R.nc[1], nz = R.nc[2];
  const int rx = R.reach[0], ry = R.reach[1];
  const int xlo = rx < 0 ? 0 : -rx, xhi = rx < 0 ? nx - 1 : rx;
  const int ylo = ry < 0 ? 0 : -ry, yhi = ry < 0 ? ny - 1 : ry;
  for (int dx = xlo; dx <= xhi; ++dx) {
    float gx = 0.f;
    int cx;
    if (rx < 0) {
      cx = dx;
    } else {
      gx = dx > 0 ? (float)dx - off[0] : (dx < 0 ? off[0] + (float)(-dx - 1) : 0.f);
      gx *= R.hf[0];
      cx = c[0] + dx;
      cx += cx < 0 ? nx : 0;
      cx -= cx >= nx ? nx : 0;
    }
    for (int dy = ylo; dy <= yhi; ++dy) {
      float gy = 0.f;
      int cy;
      if (ry < 0) {
        cy = dy;
      } else {
        gy = dy > 0 ? (float)dy - off[1] : (dy < 0 ? off[1] + (float)(-dy - 1) : 0.f);
        gy *= R.hf[1];
        cy = c[1] + dy;
        cy += cy < 0 ? ny : 0;
        cy -= cy >= ny ? ny : 0;
      }
      float dxy2 = gx * gx + gy * gy;
      if (dxy2 >= rcc2) continue;
      float zr = sqrtf(rcc2 - dxy2) / R.hf[2];
      float zc = (float)c[2] + off[2];
      int zlo = (int)floorf(zc - zr), zhi = (int)floorf(zc + zr);
      int colbase = R.cell_off + (cx * ny + cy) * nz;
      int segs[2][2];
      int nseg;
      if (zhi - zlo + 1 >= nz) {
        segs[0][0] = 0;
        segs[0][1] = nz - 1;
        nseg = 1;
      } else {
        int a = zlo < 0 ? zlo + nz : zlo;
        int b = zhi >= nz ? zhi - nz : zhi;
        if (a <= b) {
          segs[0][0] = a;
          segs[0][1] = b;
          nseg = 1;
        } else {
          segs[0][0] = a;
          segs[0][1] = nz - 1;
          segs[1][0] = 0;
          segs[1][1] = b;
          nseg = 2;
        }
      }
      for (int sgi = 0; sgi < nseg; ++sgi) {
        int jlo = start[colbase + segs[sgi][0]];
        int jhi = start[colbase + segs[sgi][1] + 1];
        for (int j = jlo + sub; j < jhi; j += TPA) f(j);
      }
    }
  }
}

// Per-lane accumulators.
template <typename T>
struct Lane {
  T fx, fy, fz;
  double e, w0, w1, w2, w3, w4, w5;  // energy and virial summed in FP64
  T eA[MAXT], dj[MAXT], di;          // adjoint sums of the current bead i
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

// Separation of a staged pair in physical units; returns false if r >= rc
// or j is the bead itself.
template <typename T>
struct PairGeom;
template <>
struct PairGeom<float> {
  float unit, unit2, rc2u;
  __device__ inline bool sep(const StageRec<float>& me, const StageRec<float>& o, float& dx, float& dy, float& dz,
                             float& r2) const {
    const float fx = (float)(me.x - o.x), fy = (float)(me.y - o.y), fz = (float)(me.z - o.z);
    const float r2u = fx * fx + fy * fy + fz * fz;
    if (!(r2u < rc2u)) return false;
    dx = fx * unit;
    dy = fy * unit;
    dz = fz * unit;
    r2 = r2u * unit2;
    return true;
  }
  __device__ inline float coord(int v) const { return (float)v * unit; }
};
template <>
struct PairGeom<double> {
  double unit, unit2, rc2u;
  __device__ inline bool sep(const StageRec<double>& me, const StageRec<double>& o, double& dx, double& dy,
                             double& dz, double& r2) const {
    dx = me.x - o.x;
    dy = me.y - o.y;
    dz = me.z - o.z;
    r2 = dx * dx + dy * dy + dz * dz;
    return r2 < rc2u;
  }
  __device__ inline float coord(double v) const { return (float)v; }
};

constexpr int MAX_HOME_COLS = 64;
constexpr int QN = 8;          // per-lane hit queue entries (power of two)
constexpr int SCAN_BATCH = 4;  // candidates tested per lane between drains
constexpr int DRAIN_MIN = 48;  // lanes with a queued hit needed to drain

template <typename T, int TPA, bool ELEC, bool EV, bool ADJ, bool COUNT>
__global__ __launch_bounds__(1024) void k_pair(PairLaunch a) {
  extern __shared__ unsigned char smem[];
  __shared__ double red[16];
  __shared__ int scan_sh[16];
  __shared__ int s_hstart[MAX_HOME_COLS + 1];
  __shared__ int s_fallback;

  const Brick B = a.bricks[blockIdx.x];
  const RepDesc& R = a.rep[B.rep];
  const int rx = R.nreach[0], ry = R.nreach[1], rz = R.nreach[2];
  const int bx = B.nb[0], by = B.nb[1], bz = B.nb[2];
  const int nxn = bx + 2 * rx, nyn = by + 2 * ry, nzn = bz + 2 * rz;
  const int ncn = nxn * nyn * nzn;
  const int ncol = (2 * rx + 1) * (2 * ry + 1);
  int* tab = reinterpret_cast<int*>(smem);
  StageRec<T>* st = reinterpret_cast<StageRec<T>*>(smem + a.lds_tab_bytes);
  uint32_t* colr = reinterpret_cast<uint32_t*>(st + a.lds_cap);
  unsigned short* qbuf = reinterpret_cast<unsigned short*>(smem + a.lds_q_off);
  const int* __restrict__ start = a.start;
  const int nx = R.nc[0], ny = R.nc[1], nz = R.nc[2];

  // 1. bead counts of the neighbourhood cells -> exclusive prefix in LDS
  for (int k = threadIdx.x; k < ncn; k += blockDim.x) {
    int ic = k % nzn, t = k / nzn, ib = t % nyn, ia = t / nyn, s0, s1, s2;
    int cx = wrap_cell(B.c0[0] - rx + ia, nx, s0);
    int cy = wrap_cell(B.c0[1] - ry + ib, ny, s1);
    int cz = wrap_cell(B.c0[2] - rz + ic, nz, s2);
    int g = R.cell_off + (cx * ny + cy) * nz + cz;
    tab[k] = start[g + 1] - start[g];
  }
  __syncthreads();
  {
    const int per = (ncn + blockDim.x - 1) / blockDim.x;
    const int lo = threadIdx.x * per, hi = min(lo + per, ncn);
    int s = 0;
    for (int k = lo; k < hi; ++k) s += tab[k];
    int inc = block_inclusive_scan(s, scan_sh);
    int run = inc - s;
    for (int k = lo; k < hi; ++k) {
      int v = tab[k];
      tab[k] = run;
      run += v;
    }
    if (threadIdx.x == blockDim.x - 1) tab[ncn] = inc;
  }
  __syncthreads();
  const int total = tab[ncn];
  if (threadIdx.x == 0) {
    s_fallback = total > a.lds_cap ? 1 : 0;
    int acc = 0;
    for (int hc = 0; hc < bx * by; ++hc) {
      int hx = hc / by, hy = hc % by;
      int col = ((hx + rx) * nyn + (hy + ry)) * nzn;
      s_hstart[hc] = acc;
      acc += tab[col + rz + bz] - tab[col + rz];
    }
    s_hstart[bx * by] = acc;
  }
  __syncthreads();
  const bool fallback = s_fallback != 0;
  const int ni = s_hstart[bx * by];
  const double h0 = R.L[0] / nx, h1 = R.L[1] / ny, h2 = R.L[2] / nz;
  const double hmax = fmax(h0, fmax(h1, h2));
  PairGeom<T> geo;
  if (sizeof(T) == 4) {
    geo.unit = (T)(hmax / STAGE_FRAC);
    geo.unit2 = geo.unit * geo.unit;
    geo.rc2u = (T)(R.rc2 / ((hmax / STAGE_FRAC) * (hmax / STAGE_FRAC)));
  } else {
    geo.unit = (T)1;
    geo.unit2 = (T)1;
    geo.rc2u = (T)R.rc2;
  }

  // 2. stage positions relative to the brick corner, images applied
  if (!fallback) {
    const double ox = B.c0[0] * h0, oy = B.c0[1] * h1, oz = B.c0[2] * h2;
    const double inv_unit = STAGE_FRAC / hmax;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      int lo = 0, hi = ncn - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tab[mid] <= e)
          lo = mid;
        else
          hi = mid - 1;
      }
      const int k = lo;
      int ic = k % nzn, t = k / nzn, ib = t % nyn, ia = t / nyn, s0, s1, s2;
      int cx = wrap_cell(B.c0[0] - rx + ia, nx, s0);
      int cy = wrap_cell(B.c0[1] - ry + ib, ny, s1);
      int cz = wrap_cell(B.c0[2] - rz + ic, nz, s2);
      int g = R.cell_off + (cx * ny + cy) * nz + cz;
      int j = start[g] + (e - tab[k]);
      const double xr = (double)a.pos[0][j] * R.scaled[0] + s0 * R.L[0] - ox;
      const double yr = (double)a.pos[1][j] * R.scaled[1] + s1 * R.L[1] - oy;
      const double zr = (double)a.pos[2][j] * R.scaled[2] + s2 * R.L[2] - oz;
      StageRec<T> r;
      if constexpr (sizeof(T) == 4) {
        r.x = (int)llrint(xr * inv_unit);
        r.y = (int)llrint(yr * inv_unit);
        r.z = (int)llrint(zr * inv_unit);
      } else {
        r.x = xr;
        r.y = yr;
        r.z = zr;
      }
      r.p = a.param[j];
      st[e] = r;
    }
  }
  __syncthreads();

  const GcmPar<T>* gtab = reinterpret_cast<const GcmPar<T>*>(a.gcm);
  const ElecPar<T>* etab = reinterpret_cast<const ElecPar<T>*>(a.elec);
  const AdjPar<T>* atab = reinterpret_cast<const AdjPar<T>*>(a.adj);
  const T sx = (T)R.scaled[0], sy = (T)R.scaled[1], sz = (T)R.scaled[2];
  const T rc2 = (T)R.rc2;
  const T beta = (T)R.beta, beta2 = (T)(R.beta * R.beta), lB = (T)R.lB;
  const float rcc = sqrtf(R.rc2f) * 1.0001f + 1e-6f;
  const float rcc2 = rcc * rcc;
  const float hf0 = (float)h0, hf1 = (float)h1, hf2 = (float)h2;
  const int ncy = 2 * ry + 1;

  Lane<T> L;
  lane_zero(L);
  const int per_pass = blockDim.x / TPA;
  const int sub = threadIdx.x % TPA;
  const int lb = threadIdx.x / TPA;  // bead slot of this lane group within the pass
  // this workgroup's slice of the brick's home beads
  const int i_lo = B.h0, i_hi = min(ni, B.h0 + B.hn);
  for (int base = i_lo; base < i_hi; base += per_pass) {
    const int ibd = base + lb;
    const bool active = ibd < i_hi;
    int gi = 0, ti = 0;
    L.fx = L.fy = L.fz = 0;
    int hx = 0, hy = 0, hz = 0, slot = 0, col = 0;
    if (active) {
      int hc = 0;
      while (hc + 1 < bx * by && s_hstart[hc + 1] <= ibd) ++hc;
      hx = hc / by;
      hy = hc % by;
      col = ((hx + rx) * nyn + (hy + ry)) * nzn;
      slot = tab[col + rz] + (ibd - s_hstart[hc]);
      while (hz + 1 < bz && tab[col + rz + hz + 1] <= slot) ++hz;
    }
    if (!fallback) {
      StageRec<T> me{};
      float xf = 0.f, yf = 0.f, zf = 0.f;
      if (active) {
        me = st[slot];
        xf = geo.coord(me.x);
        yf = geo.coord(me.y);
        zf = geo.coord(me.z);
      }
      // LDS range [lo, hi) of column k of this bead's culled neighbourhood,
      // packed lo | hi << 16 (empty if the column is beyond rc)
      auto col_range = [&](int k) -> uint32_t {
        const int dxc = k / ncy - rx, dyc = k % ncy - ry;
        const int cxn = hx + dxc, cyn = hy + dyc;
        const float gx = fmaxf(0.f, fmaxf((float)cxn * hf0 - xf, xf - (float)(cxn + 1) * hf0));
        const float gy = fmaxf(0.f, fmaxf((float)cyn * hf1 - yf, yf - (float)(cyn + 1) * hf1));
        const float d2 = gx * gx + gy * gy;
        if (!(d2 < rcc2)) return 0u;
        const float zr = sqrtf(rcc2 - d2);
        int zlo = (int)floorf((zf - zr) / hf2), zhi = (int)floorf((zf + zr) / hf2);
        zlo = max(zlo, hz - rz);
        zhi = min(zhi, hz + rz);
        const int cb = ((cxn + rx) * nyn + (cyn + ry)) * nzn + rz;
        return (uint32_t)tab[cb + zlo] | ((uint32_t)tab[cb + zhi + 1] << 16);
      };
      // with several lanes per bead the ranges are computed once, by the
      // bead's lanes together, into an LDS list
      uint32_t* myr = colr + (size_t)lb * a.ncol_max;
      if (TPA > 1) {
        if (active)
          for (int k = sub; k < ncol; k += TPA) myr[k] = col_range(k);
        __syncthreads();
      }
      {
        if (active) {
          ti = param_type(me.p);
          // sorted index of the home bead: its cell's start + rank in the cell
          const int kc = col + rz + hz;
          int s0, s1, s2;
          const int gx = wrap_cell(B.c0[0] + hx, nx, s0), gy = wrap_cell(B.c0[1] + hy, ny, s1);
          const int gz = wrap_cell(B.c0[2] + hz, nz, s2);
          gi = start[R.cell_off + (gx * ny + gy) * nz + gz] + (slot - tab[kc]);
        }
        const T zi = (T)param_z(me.p);
        const GcmPar<T>* grow = gtab + ((size_t)B.rep * MAXT + ti) * MAXT;
        const ElecPar<T>* erow = etab + ((size_t)B.rep * MAXT + ti) * MAXT;
        const AdjPar<T>* arow = atab + ((size_t)B.rep * MAXT + ti) * MAXT;
        // Walk the concatenated column ranges: candidate c (c = sub, sub +
        // TPA, ...) of the bead lies in column k at LDS slot jlo + c - P.
        // Hits go to this lane's LDS queue; queued hits are evaluated only
        // while at least 3/4 of the wave has one, so the costly interaction
        // runs with dense lanes.  Each lane keeps its own hits in order, so
        // every force is still a fixed-order private sum.
        unsigned short* q = qbuf + (size_t)threadIdx.x * QN;
        int qh = 0, qt = 0;
        int k = -1, P = 0, jlo = 0, n = 0;
        int c = sub;
        bool more = active;
        auto advance = [&]() {
          while (more && c >= P + n) {
            P += n;
            ++k;
            if (k >= ncol) {
              more = false;
              break;
            }
            const uint32_t v = TPA > 1 ? myr[k] : col_range(k);
            jlo = (int)(v & 0xffffu);
            n = (int)(v >> 16) - jlo;
          }
        };
        auto drain_one = [&]() {
          const int j = q[qh & (QN - 1)];
          ++qh;
          T ddx, ddy, ddz, r2;
          const StageRec<T> o = st[j];
          geo.sep(me, o, ddx, ddy, ddz, r2);
          interact<T, ELEC, EV, ADJ, COUNT>(L, ddx, ddy, ddz, r2, o.p, grow, erow, arow, zi, beta, beta2, lB);
        };
        advance();
        while (__any(more)) {
#pragma unroll
          for (int s = 0; s < SCAN_BATCH; ++s) {
            if (more && qt - qh < QN) {
              const int j = jlo + (c - P);
              T ddx, ddy, ddz, r2;
              if (geo.sep(me, st[j], ddx, ddy, ddz, r2) && j != slot) {
                q[qt & (QN - 1)] = (unsigned short)j;
                ++qt;
              }
              c += TPA;
              advance();
            }
          }
          while (true) {
            const bool blocked = more && qt - qh == QN;
            if (__popcll(__ballot(qt > qh)) < DRAIN_MIN && !__any(blocked)) break;
            if (qt > qh) drain_one();
          }
        }
        while (__any(qt > qh)) {
          if (qt > qh) drain_one();
        }
      }
      if (TPA > 1) __syncthreads();
    } else if (active) {
      // global-memory walk for a neighbourhood too large for LDS
      const int kc = col + rz + hz;
      int ic = kc % nzn, t = kc / nzn, ib = t % nyn, ia = t / nyn, s0, s1, s2;
      int cx = wrap_cell(B.c0[0] - rx + ia, nx, s0);
      int cy = wrap_cell(B.c0[1] - ry + ib, ny, s1);
      int cz = wrap_cell(B.c0[2] - rz + ic, nz, s2);
      int g = R.cell_off + (cx * ny + cy) * nz + cz;
      gi = start[g] + (slot - tab[kc]);
      const uint32_t u[3] = {a.pos[0][gi], a.pos[1][gi], a.pos[2][gi]};
      const uint32_t pi = a.param[gi];
      ti = param_type(pi);
      const T zi = (T)param_z(pi);
      const GcmPar<T>* grow = gtab + ((size_t)B.rep * MAXT + ti) * MAXT;
      const ElecPar<T>* erow = etab + ((size_t)B.rep * MAXT + ti) * MAXT;
      const AdjPar<T>* arow = atab + ((size_t)B.rep * MAXT + ti) * MAXT;
      const int me = gi;
      for_each_candidate<TPA>(R, u, start, sub, [&](int j) {
        T ddx = (T)(int)(u[0] - a.pos[0][j]) * sx;
        T ddy = (T)(int)(u[1] - a.pos[1][j]) * sy;
        T ddz = (T)(int)(u[2] - a.pos[2][j]) * sz;
        T r2 = ddx * ddx + ddy * ddy + ddz * ddz;
        if (r2 < rc2 && j != me)
          interact<T, ELEC, EV, ADJ, COUNT>(L, ddx, ddy, ddz, r2, a.param[j], grow, erow, arow, zi, beta, beta2, lB);
      });
    }
    if (ADJ && active) flush_adj<T, ELEC>(L, ti);
    T fx = L.fx, fy = L.fy, fz = L.fz;
    if (TPA > 1) {
      fx = lane_reduce(fx, TPA);
      fy = lane_reduce(fy, TPA);
      fz = lane_reduce(fz, TPA);
    }
    if (active && sub == 0) {
      const int fi = ELEC ? a.qidx[gi] : gi;
      atomicAdd((unsigned long long*)&a.F[0][fi], (unsigned long long)to_fixed((double)fx, a.fscale, a.status));
      atomicAdd((unsigned long long*)&a.F[1][fi], (unsigned long long)to_fixed((double)fy, a.fscale, a.status));
      atomicAdd((unsigned long long*)&a.F[2][fi], (unsigned long long)to_fixed((double)fz, a.fscale, a.status));
    }
  }

  if (COUNT) {
    unsigned long long c = L.cnt;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(a.pair_count, c);
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

// Workgroups may use more than 64 KiB of dynamic LDS (gfx950 has 160 KiB per
// CU): raise each kernel's limit once to what it is launched with.
void allow_lds(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  if (bytes <= 65536) return;
  std::lock_guard<std::mutex> lk(mu);
  size_t& d = done[fn];
  if (d >= bytes) return;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess) d = bytes;
}

template <typename T, int TPA, bool ELEC, bool EV, bool ADJ, bool COUNT>
void launch_one(hipStream_t s, const PairLaunch& a) {
  auto fn = k_pair<T, TPA, ELEC, EV, ADJ, COUNT>;
  allow_lds((const void*)fn, a.lds_bytes);
  hipLaunchKernelGGL(fn, dim3(a.nbricks), dim3(a.threads), a.lds_bytes, s, a);
}

template <typename T, int TPA, bool ELEC>
void dispatch_mode(hipStream_t s, const PairLaunch& a, bool ev, bool adj, bool count) {
  if (count)
    launch_one<T, TPA, ELEC, false, false, true>(s, a);
  else if (adj)
    launch_one<T, TPA, ELEC, true, true, false>(s, a);
  else if (ev)
    launch_one<T, TPA, ELEC, true, false, false>(s, a);
  else
    launch_one<T, TPA, ELEC, false, false, false>(s, a);
}

template <typename T, bool ELEC>
void dispatch_tpa(hipStream_t s, const PairLaunch& a, int tpa, bool ev, bool adj, bool count) {
  switch (tpa) {
    case 1: dispatch_mode<T, 1, ELEC>(s, a, ev, adj, count); break;
    case 2: dispatch_mode<T, 2, ELEC>(s, a, ev, adj, count); break;
    case 4: dispatch_mode<T, 4, ELEC>(s, a, ev, adj, count); break;
    case 8: dispatch_mode<T, 8, ELEC>(s, a, ev, adj, count); break;
    default: dispatch_mode<T, 16, ELEC>(s, a, ev, adj, count); break;
  }
}

}  // namespace

void launch_pair_gcm(hipStream_t s, const PairLaunch& a, bool fp64, int tpa, bool ev, bool adjoint) {
  if (a.nbricks <= 0) return;
  bool count = a.pair_count != nullptr;
  if (fp64)
    dispatch_tpa<double, false>(s, a, tpa, ev, adjoint, count);
  else
    dispatch_tpa<float, false>(s, a, tpa, ev, adjoint, count);
}

void launch_pair_elec(hipStream_t s, const PairLaunch& a, bool fp64, int tpa, bool ev, bool adjoint) {
  if (a.nbricks <= 0) return;
  if (fp64)
    dispatch_tpa<double, true>(s, a, tpa, ev, adjoint, false);
  else
    dispatch_tpa<float, true>(s, a, tpa, ev, adjoint, false);
}

size_t pair_stage_bytes(bool fp64) { return fp64 ? sizeof(StageRec<double>) : sizeof(StageRec<float>); }

int pair_queue_bytes(int threads) { return threads * QN * 2; }

}  // namespace gcme
