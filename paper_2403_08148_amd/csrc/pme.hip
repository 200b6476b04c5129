// Smooth particle-mesh Ewald for U_recip of eq. ewald (the paper evaluates
// the reciprocal sum with the particle-mesh Ewald method it cites):
//
//   spread   Q(k) = sum_i z_i prod_a M_p(u_ia - k_a)   (fixed-point atomics)
//   z pass   real-to-complex transform of each z line (and clears Q)
//   y pass   complex transform of each y line
//   x pass   transform x lines, multiply by G(m) = B(m) exp(-pi^2 m^2/beta^2)
//            / (pi V m^2) while summing E = lB/2 sum G |Q^|^2 and the virial,
//            inverse-transform the lines (one kernel, lines stay in LDS)
//   y pass   inverse
//   z pass   complex-to-real inverse -> potential phi(k)
//   gather   F_i = -lB z_i sum_k grad W_i(k) phi(k)
//
// The mesh transforms are Stockham radix-4/2/3 FFTs on batches of lines held
// in LDS; batches of strided lines are loaded so that consecutive threads
// touch consecutive addresses.
#include "gcme_internal.h"

namespace gcme {

namespace {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Cardinal B-spline weights w[j] = M_P(t + j) and derivatives dw[j] =
// M_P'(t + j), j = 0..P-1, t in [0, 1), from the two-term recursion of
// M_n in n; the derivative is M_{P-1}(x) - M_{P-1}(x - 1).
template <typename T, int P>
__device__ inline void bspline(T t, T* w, T* dw) {
  T m[P];
#pragma unroll
  for (int j = 0; j < P; ++j) m[j] = j == 0 ? (T)1 : (T)0;
#pragma unroll
  for (int n = 2; n <= P; ++n) {
    if (n == P) {
#pragma unroll
      for (int j = 0; j < P; ++j) dw[j] = (j < P - 1 ? m[j] : (T)0) - (j > 0 ? m[j - 1] : (T)0);
    }
    const T inv = (T)1 / (T)(n - 1);
#pragma unroll
    for (int j = n - 1; j >= 0; --j) {
      T a = j < n - 1 ? m[j] : (T)0;
      T b = j > 0 ? m[j - 1] : (T)0;
      m[j] = ((t + (T)j) * a + ((T)n - t - (T)j) * b) * inv;
    }
  }
#pragma unroll
  for (int j = 0; j < P; ++j) w[j] = m[j];
}

// Mesh coordinate of a fixed-point fractional position: integer cell and
// fractional offset, exact up to the final rounding of the offset.
template <typename T>
__device__ inline void mesh_coord(uint32_t u, int K, int& k, T& t) {
  unsigned long long p = (unsigned long long)u * (unsigned)K;
  k = (int)(p >> 32);
  t = (T)((double)(uint32_t)(p & 0xffffffffu) * 2.3283064365386963e-10);
}

// Eight lanes per charged bead: lane j0 < P of the group handles the
// x-slab j0 of the P^3 stencil (the others idle), which gives the small
// charged sets enough lanes to hide the atomics' latency.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_spread(PmeLaunch a, int nq) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = t >> 3, j0 = t & 7;
  if (q >= nq || j0 >= P) return;
  uint32_t prm = a.qparam[q];
  const RepDesc& R = a.rep[param_rep(prm)];
  T w[3][P], dw[P];
  int k0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T t;
    mesh_coord<T>(a.qpos[d][q], R.K[d], k0[d], t);
    bspline<T, P>(t, w[d], dw);
  }
  const T z = (T)param_z(prm);
  const int K0 = R.K[0], K1 = R.K[1], K2 = R.K[2];
  long long* Q = a.Qint + R.grid_off;
  int g2s[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    int g = k0[2] - j;
    g2s[j] = g < 0 ? g + K2 : g;
  }
  {
    int g0 = k0[0] - j0;
    g0 += g0 < 0 ? K0 : 0;
    T a0 = z * w[0][j0];
    for (int j1 = 0; j1 < P; ++j1) {
      int g1 = k0[1] - j1;
      g1 += g1 < 0 ? K1 : 0;
      T a01 = a0 * w[1][j1];
      long long* row = Q + ((long long)g0 * K1 + g1) * K2;
#pragma unroll
      for (int j2 = 0; j2 < P; ++j2) {
        double v = (double)(a01 * w[2][j2]) * a.qscale;
        atomicAdd((unsigned long long*)&row[g2s[j2]], (unsigned long long)(long long)llrint(v));
      }
    }
  }
}

// In-LDS Stockham FFT of nl lines of length K (element (k, l) at k*LBP + l).
// Returns the buffer holding the result (A or B).
template <typename T>
__device__ cplx<T>* fft_lines(cplx<T>* A, cplx<T>* B, int K, int LBP, int nl, const cplx<T>* __restrict__ tw,
                              const int* __restrict__ rad, int nrad, bool inverse) {
  const T sgn = inverse ? (T)1 : (T)-1;
  int Ns = 1;
  for (int s = 0; s < nrad; ++s) {
    const int Rr = rad[s];
    const int nb = K / Rr;
    const int tstride = K / (Ns * Rr);
    for (int b = threadIdx.x; b < nb * nl; b += blockDim.x) {
      const int l = b % nl;
      const int j = b / nl;
      const int k = j % Ns;
      cplx<T> v[4];
      for (int r = 0; r < Rr; ++r) v[r] = A[(j + r * nb) * LBP + l];
      for (int r = 1; r < Rr; ++r) {
        cplx<T> w = tw[k * r * tstride];
        if (inverse) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
      cplx<T> o[4];
      if (Rr == 2) {
        o[0] = {v[0].x + v[1].x, v[0].y + v[1].y};
        o[1] = {v[0].x - v[1].x, v[0].y - v[1].y};
      } else if (Rr == 4) {
        // X_q = sum_s v_s exp(sgn 2 pi i s q / 4); exp(sgn pi i/2) = sgn i
        cplx<T> a0 = {v[0].x + v[2].x, v[0].y + v[2].y};
        cplx<T> a1 = {v[0].x - v[2].x, v[0].y - v[2].y};
        cplx<T> b0 = {v[1].x + v[3].x, v[1].y + v[3].y};
        cplx<T> b1 = {v[1].x - v[3].x, v[1].y - v[3].y};
        // sgn i * b1
        cplx<T> ib1 = {-sgn * b1.y, sgn * b1.x};
        o[0] = {a0.x + b0.x, a0.y + b0.y};
        o[2] = {a0.x - b0.x, a0.y - b0.y};
        o[1] = {a1.x + ib1.x, a1.y + ib1.y};
        o[3] = {a1.x - ib1.x, a1.y - ib1.y};
      } else {
        // radix 3: w = exp(sgn 2 pi i / 3) = -1/2 + sgn i sqrt(3)/2
        const T h = (T)0.86602540378443864676;
        cplx<T> s = {v[1].x + v[2].x, v[1].y + v[2].y};
        cplx<T> d = {v[1].x - v[2].x, v[1].y - v[2].y};
        o[0] = {v[0].x + s.x, v[0].y + s.y};
        cplx<T> m = {v[0].x - (T)0.5 * s.x, v[0].y - (T)0.5 * s.y};
        // sgn i h d
        cplx<T> id = {-sgn * h * d.y, sgn * h * d.x};
        o[1] = {m.x + id.x, m.y + id.y};
        o[2] = {m.x - id.x, m.y - id.y};
      }
      const int idxD = (j / Ns) * Ns * Rr + k;
      for (int r = 0; r < Rr; ++r) B[(idxD + r * Ns) * LBP + l] = o[r];
    }
    __syncthreads();
    cplx<T>* t = A;
    A = B;
    B = t;
    Ns *= Rr;
  }
  return A;
}

template <typename T>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_z_r2c(PmeLaunch a) {
  extern __shared__ unsigned char smem[];
  const LineItem it = a.items[0][blockIdx.x];
  const RepDesc& R = a.rep[it.rep];
  const int K = R.K[2], K2h = R.K2h, nl = it.count, LBP = a.lb[0] + 1;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + (size_t)a.maxK[0] * LBP;
  long long* Q = a.Qint + R.grid_off + (long long)it.first * K;
  const double inv_qs = 1.0 / a.qscale;
  for (int e = threadIdx.x; e < nl * K; e += blockDim.x) {
    int l = e / K, k = e % K;
    long long v = Q[(long long)l * K + k];
    Q[(long long)l * K + k] = 0;  // leave the mesh cleared for the next spread
    A[k * LBP + l] = {(T)((double)v * inv_qs), (T)0};
  }
  __syncthreads();
  const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(a.tw) + R.tw_off[2];
  cplx<T>* res = fft_lines<T>(A, B, K, LBP, nl, tw, a.radix + R.rad_off[2], R.nrad[2], false);
  cplx<T>* out = reinterpret_cast<cplx<T>*>(a.Qc) + R.cgrid_off + (long long)it.first * K2h;
  for (int e = threadIdx.x; e < nl * K2h; e += blockDim.x) {
    int l = e / K2h, m = e % K2h;
    out[(long long)l * K2h + m] = res[m * LBP + l];
  }
}

template <typename T>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_y(PmeLaunch a, int inverse) {
  extern __shared__ unsigned char smem[];
  const LineItem it = a.items[1][blockIdx.x];
  const RepDesc& R = a.rep[it.rep];
  const int K = R.K[1], K2h = R.K2h, nl = it.count, LBP = a.lb[1] + 1;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + (size_t)a.maxK[1] * LBP;
  const int x = it.first / K2h, kz0 = it.first % K2h;
  cplx<T>* base = reinterpret_cast<cplx<T>*>(a.Qc) + R.cgrid_off + (long long)x * R.K[1] * K2h + kz0;
  for (int e = threadIdx.x; e < nl * K; e += blockDim.x) {
    int k = e / nl, l = e % nl;
    A[k * LBP + l] = base[(long long)k * K2h + l];
  }
  __syncthreads();
  const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(a.tw) + R.tw_off[1];
  cplx<T>* res = fft_lines<T>(A, B, K, LBP, nl, tw, a.radix + R.rad_off[1], R.nrad[1], inverse != 0);
  for (int e = threadIdx.x; e < nl * K; e += blockDim.x) {
    int k = e / nl, l = e % nl;
    base[(long long)k * K2h + l] = res[k * LBP + l];
  }
}

__device__ inline double block_sum_fft(double v, double* sh) {
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

template <typename T, bool EV>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_x_conv(PmeLaunch a) {
  extern __shared__ unsigned char smem[];
  __shared__ double sh[4];
  const LineItem it = a.items[2][blockIdx.x];
  const RepDesc& R = a.rep[it.rep];
  const int K = R.K[0], K1 = R.K[1], K2 = R.K[2], K2h = R.K2h, nl = it.count, LBP = a.lb[2] + 1;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + (size_t)a.maxK[2] * LBP;
  const int y = it.first / K2h, kz0 = it.first % K2h;
  const long long xstride = (long long)K1 * K2h;
  cplx<T>* base = reinterpret_cast<cplx<T>*>(a.Qc) + R.cgrid_off + (long long)y * K2h + kz0;
  for (int e = threadIdx.x; e < nl * K; e += blockDim.x) {
    int k = e / nl, l = e % nl;
    A[k * LBP + l] = base[(long long)k * xstride + l];
  }
  __syncthreads();
  const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(a.tw) + R.tw_off[0];
  cplx<T>* res = fft_lines<T>(A, B, K, LBP, nl, tw, a.radix + R.rad_off[0], R.nrad[0], false);
  cplx<T>* other = res == A ? B : A;
  // Green's function, energy and virial
  const T* bsp = reinterpret_cast<const T*>(a.bsp);
  const T* frq = reinterpret_cast<const T*>(a.freq);
  const T b0y = bsp[R.bsp_off[1] + y], f1 = frq[R.bsp_off[1] + y];
  const double pi2b2 = 9.869604401089358 / (R.beta * R.beta);
  const double piV = 3.141592653589793 * R.V;
  double e = 0, w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0;
  for (int q = threadIdx.x; q < nl * K; q += blockDim.x) {
    int k = q / nl, l = q % nl;
    int m2 = kz0 + l;
    T f0 = frq[R.bsp_off[0] + k];
    T f2 = frq[R.bsp_off[2] + m2];
    T mm = f0 * f0 + f1 * f1 + f2 * f2;
    cplx<T> v = res[k * LBP + l];
    T G = 0;
    if (mm > (T)0) {
      G = (T)(exp(-pi2b2 * (double)mm) / (piV * (double)mm)) * bsp[R.bsp_off[0] + k] * b0y * bsp[R.bsp_off[2] + m2];
      if (EV) {
        double wgt = (m2 == 0 || 2 * m2 == K2) ? 1.0 : 2.0;
        double em = 0.5 * R.lB * wgt * (double)G * ((double)v.x * v.x + (double)v.y * v.y);
        double c = 2.0 * (1.0 + pi2b2 * (double)mm) / (double)mm;
        double m0 = f0, m1 = f1, m2d = f2;
        e += em;
        w0 += em * (1.0 - c * m0 * m0);
        w1 += em * (1.0 - c * m1 * m1);
        w2 += em * (1.0 - c * m2d * m2d);
        w3 -= em * c * m0 * m1;
        w4 -= em * c * m0 * m2d;
        w5 -= em * c * m1 * m2d;
      }
    }
    res[k * LBP + l] = {v.x * G, v.y * G};
  }
  __syncthreads();
  cplx<T>* fin = fft_lines<T>(res, other, K, LBP, nl, tw, a.radix + R.rad_off[0], R.nrad[0], true);
  for (int e2 = threadIdx.x; e2 < nl * K; e2 += blockDim.x) {
    int k = e2 / nl, l = e2 % nl;
    base[(long long)k * xstride + l] = fin[k * LBP + l];
  }
  if (EV) {
    double v[7] = {e, w0, w1, w2, w3, w4, w5};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      double t = block_sum_fft(v[k], sh);
      if (threadIdx.x == 0) a.part[(size_t)blockIdx.x * PART_W + k] = t;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_z_c2r(PmeLaunch a) {
  extern __shared__ unsigned char smem[];
  const LineItem it = a.items[0][blockIdx.x];
  const RepDesc& R = a.rep[it.rep];
  const int K = R.K[2], K2h = R.K2h, nl = it.count, LBP = a.lb[0] + 1;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + (size_t)a.maxK[0] * LBP;
  const cplx<T>* in = reinterpret_cast<const cplx<T>*>(a.Qc) + R.cgrid_off + (long long)it.first * K2h;
  for (int e = threadIdx.x; e < nl * K2h; e += blockDim.x) {
    int l = e / K2h, m = e % K2h;
    cplx<T> v = in[(long long)l * K2h + m];
    A[m * LBP + l] = v;
    // Hermitian partner of a real field
    int mc = K - m;
    if (m > 0 && mc > m && mc < K) A[mc * LBP + l] = {v.x, -v.y};
  }
  __syncthreads();
  const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(a.tw) + R.tw_off[2];
  cplx<T>* res = fft_lines<T>(A, B, K, LBP, nl, tw, a.radix + R.rad_off[2], R.nrad[2], true);
  T* phi = reinterpret_cast<T*>(a.phi) + R.grid_off + (long long)it.first * K;
  for (int e = threadIdx.x; e < nl * K; e += blockDim.x) {
    int l = e / K, k = e % K;
    phi[(long long)l * K + k] = res[k * LBP + l].x;
  }
}

// Eight lanes per charged bead (x-slab j0 per lane), partial gradients
// combined with xor shuffles in a fixed order.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_gather(PmeLaunch a, int nq) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int q0 = t >> 3, j0 = t & 7;
  const bool active = q0 < nq && j0 < P;
  const int q = q0 < nq ? q0 : nq - 1;
  uint32_t prm = a.qparam[q];
  const RepDesc& R = a.rep[param_rep(prm)];
  T w[3][P], dw[3][P];
  int k0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T t;
    mesh_coord<T>(a.qpos[d][q], R.K[d], k0[d], t);
    bspline<T, P>(t, w[d], dw[d]);
  }
  const int K0 = R.K[0], K1 = R.K[1], K2 = R.K[2];
  const T* phi = reinterpret_cast<const T*>(a.phi) + R.grid_off;
  int g2s[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    int g = k0[2] - j;
    g2s[j] = g < 0 ? g + K2 : g;
  }
  T gx = 0, gy = 0, gz = 0;
  if (active) {
    int g0 = k0[0] - j0;
    g0 += g0 < 0 ? K0 : 0;
    for (int j1 = 0; j1 < P; ++j1) {
      int g1 = k0[1] - j1;
      g1 += g1 < 0 ? K1 : 0;
      const T* row = phi + ((long long)g0 * K1 + g1) * K2;
      T s0 = 0, s2 = 0;
#pragma unroll
      for (int j2 = 0; j2 < P; ++j2) {
        T ph = row[g2s[j2]];
        s0 += w[2][j2] * ph;
        s2 += dw[2][j2] * ph;
      }
      gx += dw[0][j0] * w[1][j1] * s0;
      gy += w[0][j0] * dw[1][j1] * s0;
      gz += w[0][j0] * w[1][j1] * s2;
    }
  }
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) {
    gx += __shfl_xor(gx, o, 64);
    gy += __shfl_xor(gy, o, 64);
    gz += __shfl_xor(gz, o, 64);
  }
  if (q0 >= nq || j0 != 0) return;
  const double c = -R.lB * (double)param_z(prm);
  const int bi = a.qidx[q];
  double f[3] = {c * (double)gx * K0 / R.L[0], c * (double)gy * K1 / R.L[1], c * (double)gz * K2 / R.L[2]};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double v = f[d] * a.fscale;
    long long iv = 0;
    if (fabs(v) < 4.0e18)
      iv = (long long)llrint(v);
    else
      atomicOr(a.status, (unsigned)STATUS_FORCE_OVERFLOW);
    atomicAdd((unsigned long long*)&a.F[d][bi], (unsigned long long)iv);
  }
}

template <typename T>
void spread_p(hipStream_t s, const PmeLaunch& a, int p, int nq) {
  dim3 g((8 * nq + 255) / 256), b(256);
  switch (p) {
    case 3: hipLaunchKernelGGL((k_spread<T, 3>), g, b, 0, s, a, nq); break;
    case 4: hipLaunchKernelGGL((k_spread<T, 4>), g, b, 0, s, a, nq); break;
    case 5: hipLaunchKernelGGL((k_spread<T, 5>), g, b, 0, s, a, nq); break;
    case 6: hipLaunchKernelGGL((k_spread<T, 6>), g, b, 0, s, a, nq); break;
    case 7: hipLaunchKernelGGL((k_spread<T, 7>), g, b, 0, s, a, nq); break;
    default: hipLaunchKernelGGL((k_spread<T, 8>), g, b, 0, s, a, nq); break;
  }
}

template <typename T>
void gather_p(hipStream_t s, const PmeLaunch& a, int p, int nq) {
  dim3 g((8 * nq + 255) / 256), b(256);
  switch (p) {
    case 3: hipLaunchKernelGGL((k_gather<T, 3>), g, b, 0, s, a, nq); break;
    case 4: hipLaunchKernelGGL((k_gather<T, 4>), g, b, 0, s, a, nq); break;
    case 5: hipLaunchKernelGGL((k_gather<T, 5>), g, b, 0, s, a, nq); break;
    case 6: hipLaunchKernelGGL((k_gather<T, 6>), g, b, 0, s, a, nq); break;
    case 7: hipLaunchKernelGGL((k_gather<T, 7>), g, b, 0, s, a, nq); break;
    default: hipLaunchKernelGGL((k_gather<T, 8>), g, b, 0, s, a, nq); break;
  }
}

inline size_t lds_bytes(const PmeLaunch& a, int pass, bool fp64) {
  return 2 * (size_t)a.maxK[pass] * (size_t)(a.lb[pass] + 1) * (fp64 ? 16 : 8);
}

}  // namespace

void launch_spread(hipStream_t s, const PmeLaunch& a, bool fp64) {
  int nq = a.nq, p = a.order;
  if (nq <= 0) return;
  if (fp64)
    spread_p<double>(s, a, p, nq);
  else
    spread_p<float>(s, a, p, nq);
}

void launch_gather(hipStream_t s, const PmeLaunch& a, bool fp64) {
  int nq = a.nq, p = a.order;
  if (nq <= 0) return;
  if (fp64)
    gather_p<double>(s, a, p, nq);
  else
    gather_p<float>(s, a, p, nq);
}

void launch_fft_z_r2c(hipStream_t s, const PmeLaunch& a, bool fp64) {
  if (a.nitems[0] <= 0) return;
  size_t sh = lds_bytes(a, 0, fp64);
  if (fp64)
    hipLaunchKernelGGL(k_fft_z_r2c<double>, dim3(a.nitems[0]), dim3(FFT_THREADS), sh, s, a);
  else
    hipLaunchKernelGGL(k_fft_z_r2c<float>, dim3(a.nitems[0]), dim3(FFT_THREADS), sh, s, a);
}

void launch_fft_y(hipStream_t s, const PmeLaunch& a, bool fp64, bool inverse) {
  if (a.nitems[1] <= 0) return;
  size_t sh = lds_bytes(a, 1, fp64);
  if (fp64)
    hipLaunchKernelGGL(k_fft_y<double>, dim3(a.nitems[1]), dim3(FFT_THREADS), sh, s, a, (int)inverse);
  else
    hipLaunchKernelGGL(k_fft_y<float>, dim3(a.nitems[1]), dim3(FFT_THREADS), sh, s, a, (int)inverse);
}

void launch_fft_x_conv(hipStream_t s, const PmeLaunch& a, bool fp64, bool ev) {
  if (a.nitems[2] <= 0) return;
  size_t sh = lds_bytes(a, 2, fp64);
  dim3 g(a.nitems[2]), b(FFT_THREADS);
  if (fp64) {
    if (ev)
      hipLaunchKernelGGL((k_fft_x_conv<double, true>), g, b, sh, s, a);
    else
      hipLaunchKernelGGL((k_fft_x_conv<double, false>), g, b, sh, s, a);
  } else {
    if (ev)
      hipLaunchKernelGGL((k_fft_x_conv<float, true>), g, b, sh, s, a);
    else
      hipLaunchKernelGGL((k_fft_x_conv<float, false>), g, b, sh, s, a);
  }
}

void launch_fft_z_c2r(hipStream_t s, const PmeLaunch& a, bool fp64) {
  if (a.nitems[0] <= 0) return;
  size_t sh = lds_bytes(a, 0, fp64);
  if (fp64)
    hipLaunchKernelGGL(k_fft_z_c2r<double>, dim3(a.nitems[0]), dim3(FFT_THREADS), sh, s, a);
  else
    hipLaunchKernelGGL(k_fft_z_c2r<float>, dim3(a.nitems[0]), dim3(FFT_THREADS), sh, s, a);
}

}  // namespace gcme
