// Cutoff pair kernels.
//
//  * k_pair_gcm: eq. u_ex for every pair within rc (all beads).
//  * k_pair_elec: the real-space bracket of eq. ewald,
//    lB z_i z_j [erf(alpha_ij r) - erf(beta r)]/r, over the charged beads only
//    (a separate cell list of charged beads), so the transcendental-heavy
//    term costs nothing for neutral beads and the two kernels never diverge
//    on charge.
//
// Mapping: TPA lanes of a wavefront share one bead i and split its neighbour
// scan; their partial forces are combined with xor shuffles in a fixed order.
// The scan walks columns of cells around i (cells are z-major within a
// column, so a run of z cells is one contiguous range of sorted beads) and,
// per lane, culls columns by the exact distance from i to the column and
// clips the z run to the cutoff sphere.  Every pair is visited from both
// ends (no force scatter to j), so each force is a private sum in a fixed
// order; it is added once to the 64-bit fixed-point accumulator.
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

template <typename T>
__device__ inline T lane_reduce(T v, int tpa) {
  for (int o = tpa >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum over a 256-thread block; result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0) t = ((sh[0] + sh[1]) + (sh[2] + sh[3]));
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

// Walk the cutoff neighbourhood of bead i (fixed-point position u) in replica
// R, calling f(j) for every candidate bead j of the cell ranges (j may be i).
// `start` is the cell-start array of the bead set being scanned.
template <int TPA, typename F>
__device__ inline void for_each_candidate(const RepDesc& R, const uint32_t u[3], const int* __restrict__ start,
                                          int sub, F&& f) {
  int c[3];
  float off[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    unsigned long long p = (unsigned long long)u[k] * (unsigned)R.nc[k];
    c[k] = (int)(p >> 32);
    off[k] = (float)(uint32_t)(p & 0xffffffffu) * 2.3283064365386963e-10f;  // in cell units
  }
  // slack so that rounding in the culling never drops a pair; the exact
  // r < rc test is done per pair
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

template <typename T, int TPA, bool EV, bool ADJ, bool COUNT>
__global__ __launch_bounds__(256) void k_pair_gcm(PairLaunch a) {
  __shared__ double sh[4];
  const Tile tile = a.tiles[blockIdx.x];
  const RepDesc& R = a.rep[tile.rep];
  const int local = threadIdx.x / TPA;
  const int sub = threadIdx.x % TPA;
  const bool active = local < tile.count;
  const int i = tile.first + (active ? local : 0);
  const GcmPar<T>* gtab = reinterpret_cast<const GcmPar<T>*>(a.gcm);
  const AdjPar<T>* atab = reinterpret_cast<const AdjPar<T>*>(a.adj);

  T fx = 0, fy = 0, fz = 0;
  T e = 0, w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0;
  T eA[MAXT] = {}, dsj[MAXT] = {};
  T dsi = 0;
  unsigned long long cnt = 0;
  int ti = 0;
  if (active) {
    const uint32_t u[3] = {a.pos[0][i], a.pos[1][i], a.pos[2][i]};
    ti = param_type(a.param[i]);
    const GcmPar<T>* row = gtab + ((size_t)tile.rep * MAXT + ti) * MAXT;
    const AdjPar<T>* arow = atab + ((size_t)tile.rep * MAXT + ti) * MAXT;
    const T sx = (T)R.scaled[0], sy = (T)R.scaled[1], sz = (T)R.scaled[2];
    const T rc2 = (T)R.rc2;
    for_each_candidate<TPA>(R, u, a.start, sub, [&](int j) {
      T dx = (T)(int)(u[0] - a.pos[0][j]) * sx;
      T dy = (T)(int)(u[1] - a.pos[1][j]) * sy;
      T dz = (T)(int)(u[2] - a.pos[2][j]) * sz;
      T r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < rc2 && j != i) {
        int tj = param_type(a.param[j]);
        GcmPar<T> g = row[tj];
        T uu = g.C * gexp2(-g.bl * r2);
        T fs = g.twob * uu;
        fx += fs * dx;
        fy += fs * dy;
        fz += fs * dz;
        if (EV) {
          e += uu;
          w0 += fs * dx * dx;
          w1 += fs * dy * dy;
          w2 += fs * dz * dz;
          w3 += fs * dx * dy;
          w4 += fs * dx * dz;
          w5 += fs * dy * dz;
        }
        if (ADJ) {
          AdjPar<T> ap = arow[tj];
          // du/ds = u (3 r^2/s^3 - 3/s)
          T duds = uu * ((T)3 * r2 * ap.inv_s2 - (T)3) * ap.s_inv;
          dsi += duds * ap.dsig_i;
#pragma unroll
          for (int t = 0; t < MAXT; ++t) {
            if (t == tj) {
              eA[t] += uu;
              dsj[t] += duds * ap.dsig_j;
            }
          }
        }
        if (COUNT) ++cnt;
      }
    });
  }
  if (TPA > 1) {
    fx = lane_reduce(fx, TPA);
    fy = lane_reduce(fy, TPA);
    fz = lane_reduce(fz, TPA);
  }
  if (active && sub == 0) {
    atomicAdd((unsigned long long*)&a.F[0][i], (unsigned long long)to_fixed((double)fx, a.fscale, a.status));
    atomicAdd((unsigned long long*)&a.F[1][i], (unsigned long long)to_fixed((double)fy, a.fscale, a.status));
    atomicAdd((unsigned long long*)&a.F[2][i], (unsigned long long)to_fixed((double)fz, a.fscale, a.status));
  }
  if (COUNT) {
    // each pair is seen from both ends
    unsigned long long c = cnt;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(a.pair_count, c);
  }
  if (EV) {
    double v[7] = {(double)e, (double)w0, (double)w1, (double)w2, (double)w3, (double)w4, (double)w5};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      double t = block_sum(v[k], sh);
      if (threadIdx.x == 0) a.part[(size_t)blockIdx.x * PART_W + k] = 0.5 * t;
    }
  }
  if (ADJ) {
    // [ti*MAXT + tj] type-pair energies, then dE/dsigma per type
    for (int q = 0; q < MAXT * MAXT; ++q) {
      int qt = q / MAXT, qu = q % MAXT;
      double v = (active && qt == ti) ? (double)eA[qu] : 0.0;
      double t = block_sum(v, sh);
      if (threadIdx.x == 0) a.adj_part[(size_t)blockIdx.x * (MAXT * MAXT + 2 * MAXT) + q] = 0.5 * t;
    }
    for (int t = 0; t < MAXT; ++t) {
      double v = active ? (double)dsj[t] + (t == ti ? (double)dsi : 0.0) : 0.0;
      double s = block_sum(v, sh);
      if (threadIdx.x == 0) a.adj_part[(size_t)blockIdx.x * (MAXT * MAXT + 2 * MAXT) + MAXT * MAXT + t] = 0.5 * s;
    }
  }
}

template <typename T, int TPA, bool EV, bool ADJ>
__global__ __launch_bounds__(256) void k_pair_elec(PairLaunch a) {
  __shared__ double sh[4];
  const Tile tile = a.tiles[blockIdx.x];
  const RepDesc& R = a.rep[tile.rep];
  const int local = threadIdx.x / TPA;
  const int sub = threadIdx.x % TPA;
  const bool active = local < tile.count;
  const int i = tile.first + (active ? local : 0);
  const ElecPar<T>* etab = reinterpret_cast<const ElecPar<T>*>(a.elec);
  const AdjPar<T>* atab = reinterpret_cast<const AdjPar<T>*>(a.adj);
  constexpr T TSP = (T)1.1283791670955126;  // 2/sqrt(pi)

  T fx = 0, fy = 0, fz = 0;
  T e = 0, w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0;
  T daj[MAXT] = {};
  T dai = 0;
  int ti = 0;
  if (active) {
    const uint32_t u[3] = {a.pos[0][i], a.pos[1][i], a.pos[2][i]};
    const uint32_t pi = a.param[i];
    ti = param_type(pi);
    const T zi = (T)param_z(pi);
    const ElecPar<T>* row = etab + ((size_t)tile.rep * MAXT + ti) * MAXT;
    const AdjPar<T>* arow = atab + ((size_t)tile.rep * MAXT + ti) * MAXT;
    const T sx = (T)R.scaled[0], sy = (T)R.scaled[1], sz = (T)R.scaled[2];
    const T rc2 = (T)R.rc2;
    const T beta = (T)R.beta, beta2 = (T)(R.beta * R.beta), lB = (T)R.lB;
    for_each_candidate<TPA>(R, u, a.start, sub, [&](int j) {
      T dx = (T)(int)(u[0] - a.pos[0][j]) * sx;
      T dy = (T)(int)(u[1] - a.pos[1][j]) * sy;
      T dz = (T)(int)(u[2] - a.pos[2][j]) * sz;
      T r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < rc2 && j != i) {
        const uint32_t pj = a.param[j];
        const int tj = param_type(pj);
        const ElecPar<T>& p = row[tj];
        const T zz = zi * (T)param_z(pj);
        T phi, g;
        if (r2 < p.rs2) {
          // series in r^2 (cancellation-free near contact)
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
        T fs = lB * zz * g;
        fx += fs * dx;
        fy += fs * dy;
        fz += fs * dz;
        if (EV) {
          e += lB * zz * phi;
          w0 += fs * dx * dx;
          w1 += fs * dy * dy;
          w2 += fs * dz * dz;
          w3 += fs * dx * dy;
          w4 += fs * dx * dz;
          w5 += fs * dy * dz;
        }
        if (ADJ) {
          const AdjPar<T> ap = arow[tj];
          // d/da_ij of lB zz erf(alpha r)/r = -lB zz (2/sqrt(pi)) (alpha/a_ij) exp(-alpha^2 r^2)
          T dd = -lB * zz * ap.ea * gexp(-p.alpha2 * r2);
          dai += dd * ap.daij_i;
#pragma unroll
          for (int t = 0; t < MAXT; ++t)
            if (t == tj) daj[t] += dd * ap.daij_j;
        }
      }
    });
  }
  if (TPA > 1) {
    fx = lane_reduce(fx, TPA);
    fy = lane_reduce(fy, TPA);
    fz = lane_reduce(fz, TPA);
  }
  if (active && sub == 0) {
    int bi = a.qidx[i];
    atomicAdd((unsigned long long*)&a.F[0][bi], (unsigned long long)to_fixed((double)fx, a.fscale, a.status));
    atomicAdd((unsigned long long*)&a.F[1][bi], (unsigned long long)to_fixed((double)fy, a.fscale, a.status));
    atomicAdd((unsigned long long*)&a.F[2][bi], (unsigned long long)to_fixed((double)fz, a.fscale, a.status));
  }
  if (EV) {
    double v[7] = {(double)e, (double)w0, (double)w1, (double)w2, (double)w3, (double)w4, (double)w5};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      double t = block_sum(v[k], sh);
      if (threadIdx.x == 0) a.part[(size_t)blockIdx.x * PART_W + k] = 0.5 * t;
    }
  }
  if (ADJ) {
    for (int t = 0; t < MAXT; ++t) {
      double v = active ? (double)daj[t] + (t == ti ? (double)dai : 0.0) : 0.0;
      double s = block_sum(v, sh);
      if (threadIdx.x == 0) a.adj_part[(size_t)blockIdx.x * (MAXT * MAXT + 2 * MAXT) + MAXT * MAXT + MAXT + t] = 0.5 * s;
    }
  }
}

template <typename T, int TPA>
void gcm_dispatch(hipStream_t s, const PairLaunch& a, bool ev, bool adj, bool count) {
  dim3 g(a.ntiles), b(256);
  if (count)
    hipLaunchKernelGGL((k_pair_gcm<T, TPA, false, false, true>), g, b, 0, s, a);
  else if (adj)
    hipLaunchKernelGGL((k_pair_gcm<T, TPA, true, true, false>), g, b, 0, s, a);
  else if (ev)
    hipLaunchKernelGGL((k_pair_gcm<T, TPA, true, false, false>), g, b, 0, s, a);
  else
    hipLaunchKernelGGL((k_pair_gcm<T, TPA, false, false, false>), g, b, 0, s, a);
}

template <typename T, int TPA>
void elec_dispatch(hipStream_t s, const PairLaunch& a, bool ev, bool adj) {
  dim3 g(a.ntiles), b(256);
  if (adj)
    hipLaunchKernelGGL((k_pair_elec<T, TPA, true, true>), g, b, 0, s, a);
  else if (ev)
    hipLaunchKernelGGL((k_pair_elec<T, TPA, true, false>), g, b, 0, s, a);
  else
    hipLaunchKernelGGL((k_pair_elec<T, TPA, false, false>), g, b, 0, s, a);
}

template <typename T>
void gcm_tpa(hipStream_t s, const PairLaunch& a, int tpa, bool ev, bool adj, bool count) {
  switch (tpa) {
    case 1: gcm_dispatch<T, 1>(s, a, ev, adj, count); break;
    case 2: gcm_dispatch<T, 2>(s, a, ev, adj, count); break;
    case 4: gcm_dispatch<T, 4>(s, a, ev, adj, count); break;
    case 8: gcm_dispatch<T, 8>(s, a, ev, adj, count); break;
    default: gcm_dispatch<T, 16>(s, a, ev, adj, count); break;
  }
}

template <typename T>
void elec_tpa(hipStream_t s, const PairLaunch& a, int tpa, bool ev, bool adj) {
  switch (tpa) {
    case 1: elec_dispatch<T, 1>(s, a, ev, adj); break;
    case 2: elec_dispatch<T, 2>(s, a, ev, adj); break;
    case 4: elec_dispatch<T, 4>(s, a, ev, adj); break;
    case 8: elec_dispatch<T, 8>(s, a, ev, adj); break;
    default: elec_dispatch<T, 16>(s, a, ev, adj); break;
  }
}

}  // namespace

void launch_pair_gcm(hipStream_t s, const PairLaunch& a, bool fp64, int tpa, bool ev, bool adjoint) {
  if (a.ntiles <= 0) return;
  bool count = a.pair_count != nullptr;
  if (fp64)
    gcm_tpa<double>(s, a, tpa, ev, adjoint, count);
  else
    gcm_tpa<float>(s, a, tpa, ev, adjoint, count);
}

void launch_pair_elec(hipStream_t s, const PairLaunch& a, bool fp64, int tpa, bool ev, bool adjoint) {
  if (a.ntiles <= 0) return;
  if (fp64)
    elec_tpa<double>(s, a, tpa, ev, adjoint);
  else
    elec_tpa<float>(s, a, tpa, ev, adjoint);
}

}  // namespace gcme
