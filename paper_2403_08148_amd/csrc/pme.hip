// Smooth particle-mesh Ewald for U_recip of eq. ewald (the paper evaluates
// the reciprocal sum with the particle-mesh Ewald method it cites):
//
//   spread+z  per tile of TX x TY z lines: every charged bead whose B-spline
//             stencil meets the tile adds z_i prod_a M_p(u_ia - k_a) to the
//             tile's points (64-bit fixed-point LDS atomics, so the sum is
//             exact and order-free), then the real-to-complex transform of
//             the tile's lines; the charge mesh never goes to HBM
//   y pass    complex transform of each y line
//   x pass    transform x lines, multiply by G(m) = B(m) exp(-pi^2 m^2/beta^2)
//             / (pi V m^2) while summing E = lB/2 sum G |Q^|^2 and the virial,
//             inverse-transform the lines (one kernel, lines stay in LDS)
//   y pass    inverse
//   z+gather  per tile: complex-to-real inverse of the tile's lines, then
//             every bead whose stencil meets the tile adds its share of
//             F_i = -lB z_i sum_k grad W_i(k) phi(k) (64-bit fixed point)
//
// The mesh transforms are Stockham radix-4/2/3 FFTs on batches of lines held
// in LDS; batches of strided lines are loaded so that consecutive threads
// touch consecutive addresses.  The beads of a tile are found through the
// charged beads' cell list (whole cell columns along z).
#include <algorithm>
#include <type_traits>

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

// Integer form of the charge mesh while a tile is spread.  Single precision:
// 32-bit integers at 2^-24 of a unit charge, so a point holds up to 128 unit
// charges' worth (one bead adds z w_x w_y w_z, at most 0.42 |z|); 32-bit LDS
// atomics and no double arithmetic, at a rounding of 3e-8 per contribution.
// Double precision: 64-bit integers at the launch's qscale.
template <typename T>
struct MeshInt;
template <>
struct MeshInt<float> {
  using U = unsigned int;
  static constexpr float scale = 16777216.0f;  // 2^24
};
template <>
struct MeshInt<double> {
  using U = unsigned long long;
};

// Mesh coordinate of a fixed-point fractional position: integer cell and
// fractional offset, exact up to the final rounding of the offset.
template <typename T>
__device__ inline void mesh_coord(uint32_t u, int K, int& k, T& t) {
  unsigned long long p = (unsigned long long)u * (unsigned)K;
  k = (int)(p >> 32);
  t = (T)((double)(uint32_t)(p & 0xffffffffu) * 2.3283064365386963e-10);
}

// Quotient of n / d for 0 <= n < 2^22, d >= 1: float reciprocal estimate
// (off by at most one in that range) and one exact integer correction --
// a handful of instructions instead of a full integer division.
struct FDiv {
  int d;
  float r;
  __device__ explicit FDiv(int dd) : d(dd), r(1.0f / (float)dd) {}
  __device__ inline int div(int n) const {
    int q = (int)((float)n * r);
    const int rem = n - q * d;
    q += (rem >= d) - (rem < 0);
    return q;
  }
};

// Quotient by a divisor fixed at compile time (D > 0: a shift or a
// multiply) or at run time (D == 0: FDiv).
template <int D>
struct QDiv {
  FDiv f;
  __device__ explicit QDiv(int d) : f(D > 0 ? D : d) {}
  __device__ inline int div(int n) const {
    if constexpr (D > 0)
      return (int)((unsigned)n / (unsigned)D);
    else
      return f.div(n);
  }
};

// Offset of half-complex mesh point (x, y, m) within a replica's mesh, in
// the layout the launch uses.
__device__ inline long long mesh_index(const PmeLaunch& a, const RepDesc& R, int x, int y, int m) {
  return a.plane_major ? ((long long)m * R.K[0] + x) * R.K[1] + y : ((long long)x * R.K[1] + y) * R.K2s + m;
}

// Radix-RR DFT of v (twiddles already applied): o_q = sum_s v_s
// exp(sgn 2 pi i s q / RR), sgn = -1 forward, +1 inverse.
template <typename T, int RR>
__device__ inline void butterfly(const cplx<T>* v, cplx<T>* o, T sgn) {
  if constexpr (RR == 2) {
    o[0] = {v[0].x + v[1].x, v[0].y + v[1].y};
    o[1] = {v[0].x - v[1].x, v[0].y - v[1].y};
  } else if constexpr (RR == 4) {
    // exp(sgn pi i/2) = sgn i
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
}

// One radix-RR Stockham stage over nl lines of length K held in LDS
// (element (k, l) at k*SK + l*SL), A -> B.  The radix is a template
// parameter so the butterfly operands stay in registers.  Consecutive
// threads take consecutive lines when the lines are interleaved (SL = 1) and
// consecutive butterflies of one line when its points are (SK = 1), so LDS
// accesses stay on consecutive banks.  NT is the block's thread count (a
// compile-time stride: blockDim would be reloaded from the dispatch packet
// with a memory round trip in every stage).
template <typename T, int RR, int NT>
__device__ inline void fft_stage(const cplx<T>* A, cplx<T>* B, int K, int SK, int SL, int nl, int Ns,
                                 const cplx<T>* __restrict__ tw, bool inverse) {
  const T sgn = inverse ? (T)1 : (T)-1;
  const int nb = K / RR;
  const int tstride = K / (Ns * RR);
  const FDiv dnl(nl), dnb(nb), dns(Ns);
  const bool kfast = SK == 1 && SL != 1;
  for (int b = threadIdx.x; b < nb * nl; b += NT) {
    int j, l;
    if (kfast) {
      l = dnb.div(b);
      j = b - l * nb;
    } else {
      j = dnl.div(b);
      l = b - j * nl;
    }
    const int jn = dns.div(j);
    const int k = j - jn * Ns;
    cplx<T> v[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) v[r] = A[(j + r * nb) * SK + l * SL];
#pragma unroll
    for (int r = 1; r < RR; ++r) {
      cplx<T> w = tw[k * r * tstride];
      if (inverse) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    cplx<T> o[RR];
    butterfly<T, RR>(v, o, sgn);
    const int idxD = jn * Ns * RR + k;
#pragma unroll
    for (int r = 0; r < RR; ++r) B[(idxD + r * Ns) * SK + l * SL] = o[r];
  }
}

// The host's radix plan of a K-point transform (radix-4 stages, then 2,
// then 3) at compile time: its length and its stage s.
constexpr int plan_len(int K) {
  int n = 0;
  while (K % 4 == 0) K /= 4, ++n;
  while (K % 2 == 0) K /= 2, ++n;
  while (K % 3 == 0) K /= 3, ++n;
  return n;
}
constexpr int plan_radix(int K, int s) {
  while (K % 4 == 0) {
    if (s-- == 0) return 4;
    K /= 4;
  }
  while (K % 2 == 0) {
    if (s-- == 0) return 2;
    K /= 2;
  }
  return 3;
}

// fft_stage with the line length, layout, line count and stage (NS = product
// of the earlier radices) known at compile time: the butterfly's indices
// are shifts and its LDS offsets immediates.
template <typename T, int K, int NT, int SK, int SL, int NL, int RR, int NS>
__device__ inline void fft_stage_c(const cplx<T>* A, cplx<T>* B, const cplx<T>* __restrict__ tw, bool inverse) {
  constexpr int NB = K / RR, TS = K / (NS * RR), NBUT = NB * NL;
  constexpr bool kfast = SK == 1 && SL != 1;
  const T sgn = inverse ? (T)1 : (T)-1;
#pragma unroll
  for (int b0 = 0; b0 < NBUT; b0 += NT) {
    const unsigned b = b0 + threadIdx.x;
    if (NBUT % NT == 0 || b < (unsigned)NBUT) {
      unsigned j, l;
      if constexpr (kfast) {
        l = b / NB;
        j = b % NB;
      } else {
        j = b / NL;
        l = b % NL;
      }
      const unsigned jn = j / NS, k = j % NS;
      const cplx<T>* src = A + j * SK + l * SL;
      cplx<T> v[RR];
#pragma unroll
      for (int r = 0; r < RR; ++r) v[r] = src[r * NB * SK];
#pragma unroll
      for (int r = 1; r < RR; ++r) {
        cplx<T> w = tw[k * r * TS];
        if (inverse) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
      cplx<T> o[RR];
      butterfly<T, RR>(v, o, sgn);
      cplx<T>* dst = B + (jn * NS * RR + k) * SK + l * SL;
#pragma unroll
      for (int r = 0; r < RR; ++r) dst[r * NS * SK] = o[r];
    }
  }
}

// All stages of fft_stage_c from stage S on, A -> B -> A ...; returns the
// buffer holding the result.
template <typename T, int K, int NT, int SK, int SL, int NL, int S = 0, int NS = 1>
__device__ inline cplx<T>* fft_lines_c(cplx<T>* A, cplx<T>* B, const cplx<T>* __restrict__ tw, bool inverse) {
  if constexpr (S == plan_len(K)) {
    return A;
  } else {
    constexpr int RR = plan_radix(K, S);
    fft_stage_c<T, K, NT, SK, SL, NL, RR, NS>(A, B, tw, inverse);
    __syncthreads();
    return fft_lines_c<T, K, NT, SK, SL, NL, S + 1, NS * RR>(B, A, tw, inverse);
  }
}

// In-LDS Stockham FFT of nl lines of length K (element (k, l) at
// k*SK + l*SL).  Returns the buffer holding the result (A or B).
template <typename T, int NT>
__device__ cplx<T>* fft_lines_s(cplx<T>* A, cplx<T>* B, int K, int SK, int SL, int nl,
                                const cplx<T>* __restrict__ tw, const int* __restrict__ rad, int nrad,
                                bool inverse) {
  int Ns = 1;
  for (int s = 0; s < nrad; ++s) {
    const int Rr = rad[s];
    if (Rr == 4)
      fft_stage<T, 4, NT>(A, B, K, SK, SL, nl, Ns, tw, inverse);
    else if (Rr == 2)
      fft_stage<T, 2, NT>(A, B, K, SK, SL, nl, Ns, tw, inverse);
    else
      fft_stage<T, 3, NT>(A, B, K, SK, SL, nl, Ns, tw, inverse);
    __syncthreads();
    cplx<T>* t = A;
    A = B;
    B = t;
    Ns *= Rr;
  }
  return A;
}

// Lines interleaved: element (k, l) at k*LBP + l.
template <typename T, int NT>
__device__ cplx<T>* fft_lines(cplx<T>* A, cplx<T>* B, int K, int LBP, int nl, const cplx<T>* __restrict__ tw,
                              const int* __restrict__ rad, int nrad, bool inverse) {
  return fft_lines_s<T, NT>(A, B, K, LBP, 1, nl, tw, rad, nrad, inverse);
}

// Copies the K twiddles of one axis into LDS (whole block; the caller's
// next __syncthreads publishes them).  The FFT stages then read twiddles at
// LDS latency instead of waiting on global loads once per stage.
template <typename T, int NT>
__device__ inline const cplx<T>* stage_twiddles(cplx<T>* dst, const PmeLaunch& a, int off, int K) {
  const cplx<T>* src = reinterpret_cast<const cplx<T>*>(a.tw) + off;
  for (int e = threadIdx.x; e < K; e += NT) dst[e] = src[e];
  return dst;
}

// Loads nl lines of K points, point k of line l at src[k * stride + l],
// into LDS at A[k * LBP + l]: consecutive threads take consecutive lines of
// one point (consecutive addresses), and each thread issues U loads before
// it stores any, so their latencies overlap.
template <typename T, int U>
__device__ inline void load_lines(cplx<T>* A, const cplx<T>* src, long long stride, int K, int nl, int LBP) {
  const FDiv dnl(nl);
  const int n = nl * K;
  for (int e0 = threadIdx.x; e0 < n; e0 += U * FFT_THREADS) {
    cplx<T> v[U];
    int k[U], l[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = min(e0 + u * FFT_THREADS, n - 1);
      k[u] = dnl.div(e);
      l[u] = e - k[u] * nl;
      v[u] = src[(long long)k[u] * stride + l[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * FFT_THREADS < n) A[k[u] * LBP + l[u]] = v[u];
  }
}

// load_lines with the line count NL of the LDS layout known at compile
// time (LDS line stride NL + 1); lines count .. NL - 1 are zero.
template <typename T, int U, int NL>
__device__ inline void load_lines_c(cplx<T>* A, const cplx<T>* src, long long stride, int K, int count) {
  const int n = NL * K;
  for (int e0 = threadIdx.x; e0 < n; e0 += U * FFT_THREADS) {
    cplx<T> v[U];
    int k[U], l[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned e = min(e0 + u * FFT_THREADS, n - 1);
      k[u] = (int)(e / NL);
      l[u] = (int)(e % NL);
      v[u] = l[u] < count ? src[(long long)k[u] * stride + l[u]] : cplx<T>{};
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * FFT_THREADS < n) A[k[u] * (NL + 1) + l[u]] = v[u];
  }
}

// y lines of a batch of kz lines at one x.  KC > 0: every replica's K1 is
// KC and the batch holds LB lines (the plan's lines per item), so the
// transform's stages, indices and LDS offsets are compile-time constants.
template <typename T, int KC, int LB>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_y(PmeLaunch a, int inverse) {
  wave_stamp(a.stamps, 0);
  extern __shared__ __align__(16) unsigned char smem[];
  const LineItem it = a.items[1][xcd_item(blockIdx.x, gridDim.x)];
  const RepDesc& R = a.rep[it.rep];
  const int K = KC > 0 ? KC : R.K[1], K2h = R.K2h, K2s = R.K2s, nl = it.count;
  const int LBP = KC > 0 ? LB + 1 : a.lb[1] + 1;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + (size_t)a.maxK[1] * LBP;
  const cplx<T>* tw = stage_twiddles<T, FFT_THREADS>(B + (size_t)a.maxK[1] * LBP, a, R.tw_off[1], K);
  const int x = it.first / K2h, kz0 = it.first % K2h;
  cplx<T>* base = reinterpret_cast<cplx<T>*>(a.Qc) + R.cgrid_off + (long long)x * R.K[1] * K2s + kz0;
  if constexpr (KC > 0) {
    load_lines_c<T, 8, LB>(A, base, K2s, KC, nl);
    __syncthreads();
    const cplx<T>* res = fft_lines_c<T, KC, FFT_THREADS, LB + 1, 1, LB>(A, B, tw, inverse != 0);
    for (int e = threadIdx.x; e < LB * KC; e += FFT_THREADS) {
      const int k = (unsigned)e / LB, l = (unsigned)e % LB;
      if (l < nl) base[(long long)k * K2s + l] = res[k * (LB + 1) + l];
    }
  } else {
    const FDiv dnl(nl);
    load_lines<T, 8>(A, base, K2s, K, nl, LBP);
    __syncthreads();
    cplx<T>* res = fft_lines<T, FFT_THREADS>(A, B, K, LBP, nl, tw, a.radix + R.rad_off[1], R.nrad[1], inverse != 0);
    for (int e = threadIdx.x; e < nl * K; e += FFT_THREADS) {
      const int k = dnl.div(e), l = e - k * nl;
      base[(long long)k * K2s + l] = res[k * LBP + l];
    }
  }
  wave_stamp(a.stamps, 1);
}

template <int NT>
__device__ inline double block_sum_fft(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0) {
    const int nw = NT >> 6;
    for (int w = 0; w < nw; ++w) t += sh[w];
  }
  return t;
}

struct RecipSums {
  double e;
  double w[6];
};

// Multiply the transformed charge at mesh frequency (mx, my, mz) (mz of the
// half-complex axis) by G(m) = B(m) exp(-pi^2 m^2/beta^2) / (pi V m^2) of
// eq. ewald, and add its energy lB/2 G |Q^|^2 (doubled for the mz lines
// that stand for their conjugates) and virial to the sums.  The Gaussian
// factorises over the axes, so gf_a(m) = exp(-pi^2 (m/L_a)^2/beta^2)/|b_a(m)|^2
// comes from per-axis tables and fr_a(m) = m/L_a is the signed frequency.
template <typename T, bool EV>
__device__ inline cplx<T> green_apply(const RepDesc& R, const T* gf0, const T* gf1, const T* gf2, const T* fr0,
                                      const T* fr1, const T* fr2, int mx, int my, int mz, cplx<T> v, RecipSums& acc) {
  const T f0 = fr0[mx], f1 = fr1[my], f2 = fr2[mz];
  const T mm = f0 * f0 + f1 * f1 + f2 * f2;
  T G = 0;
  if (mm > (T)0) {
    G = gf0[mx] * gf1[my] * gf2[mz] / ((T)(3.141592653589793 * R.V) * mm);
    if (EV) {
      const double pi2b2 = 9.869604401089358 / (R.beta * R.beta);
      const double wgt = (mz == 0 || 2 * mz == R.K[2]) ? 1.0 : 2.0;
      const double em = 0.5 * R.lB * wgt * (double)G * ((double)v.x * v.x + (double)v.y * v.y);
      const double c = 2.0 * (1.0 + pi2b2 * (double)mm) / (double)mm;
      const double m0 = f0, m1 = f1, m2 = f2;
      acc.e += em;
      acc.w[0] += em * (1.0 - c * m0 * m0);
      acc.w[1] += em * (1.0 - c * m1 * m1);
      acc.w[2] += em * (1.0 - c * m2 * m2);
      // The sum runs over every m with each component in (-K/2, K/2]; an
      // interior kz plane stands for itself and its conjugate partner
      // (-m0, -m1, -m2), except that on a Nyquist line (m0 = K0/2 or
      // m1 = K1/2) the partner keeps +K/2 there.  A term odd in such a
      // component then cancels between the two instead of doubling.
      const bool interior = wgt == 2.0;
      const bool nyx = 2 * mx == R.K[0], nyy = 2 * my == R.K[1];
      const double sxy = interior && nyx != nyy ? 0.0 : 1.0;
      const double sxz = interior && nyx ? 0.0 : 1.0;
      const double syz = interior && nyy ? 0.0 : 1.0;
      acc.w[3] -= sxy * em * c * m0 * m1;
      acc.w[4] -= sxz * em * c * m0 * m2;
      acc.w[5] -= syz * em * c * m1 * m2;
    }
  }
  return {v.x * G, v.y * G};
}

// x lines of a batch of kz lines at one y: transform, Green's function
// (energy, virial), inverse transform.  KC, LB as for k_fft_y (K0 = KC).
template <typename T, bool EV, int KC, int LB>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_x_conv(PmeLaunch a) {
  wave_stamp(a.stamps, 0);
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sh[4];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const LineItem it = a.items[2][item];
  const RepDesc& R = a.rep[it.rep];
  const int K = KC > 0 ? KC : R.K[0], K1 = R.K[1], K2h = R.K2h, K2s = R.K2s, nl = it.count;
  const int LBP = KC > 0 ? LB + 1 : a.lb[2] + 1;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + (size_t)a.maxK[2] * LBP;
  const cplx<T>* tw = stage_twiddles<T, FFT_THREADS>(B + (size_t)a.maxK[2] * LBP, a, R.tw_off[0], K);
  const int y = it.first / K2h, kz0 = it.first % K2h;
  const long long xstride = (long long)K1 * K2s;
  cplx<T>* base = reinterpret_cast<cplx<T>*>(a.Qc) + R.cgrid_off + (long long)y * K2s + kz0;
  const T* gf = reinterpret_cast<const T*>(a.bsp);
  const T* fr = reinterpret_cast<const T*>(a.freq);
  RecipSums acc{};
  if constexpr (KC > 0) {
    load_lines_c<T, 8, LB>(A, base, xstride, KC, nl);
    __syncthreads();
    cplx<T>* res = fft_lines_c<T, KC, FFT_THREADS, LB + 1, 1, LB>(A, B, tw, false);
    cplx<T>* other = res == A ? B : A;
    for (int q = threadIdx.x; q < LB * KC; q += FFT_THREADS) {
      const int k = (unsigned)q / LB, l = (unsigned)q % LB;
      if (l < nl)
        res[k * (LB + 1) + l] = green_apply<T, EV>(R, gf + R.bsp_off[0], gf + R.bsp_off[1], gf + R.bsp_off[2],
                                                   fr + R.bsp_off[0], fr + R.bsp_off[1], fr + R.bsp_off[2], k, y,
                                                   kz0 + l, res[k * (LB + 1) + l], acc);
    }
    __syncthreads();
    const cplx<T>* fin = fft_lines_c<T, KC, FFT_THREADS, LB + 1, 1, LB>(res, other, tw, true);
    for (int e2 = threadIdx.x; e2 < LB * KC; e2 += FFT_THREADS) {
      const int k = (unsigned)e2 / LB, l = (unsigned)e2 % LB;
      if (l < nl) base[(long long)k * xstride + l] = fin[k * (LB + 1) + l];
    }
  } else {
    const FDiv dnl(nl);
    load_lines<T, 8>(A, base, xstride, K, nl, LBP);
    __syncthreads();
    cplx<T>* res = fft_lines<T, FFT_THREADS>(A, B, K, LBP, nl, tw, a.radix + R.rad_off[0], R.nrad[0], false);
    cplx<T>* other = res == A ? B : A;
    for (int q = threadIdx.x; q < nl * K; q += FFT_THREADS) {
      const int k = dnl.div(q), l = q - k * nl;
      res[k * LBP + l] = green_apply<T, EV>(R, gf + R.bsp_off[0], gf + R.bsp_off[1], gf + R.bsp_off[2],
                                            fr + R.bsp_off[0], fr + R.bsp_off[1], fr + R.bsp_off[2], k, y, kz0 + l,
                                            res[k * LBP + l], acc);
    }
    __syncthreads();
    cplx<T>* fin = fft_lines<T, FFT_THREADS>(res, other, K, LBP, nl, tw, a.radix + R.rad_off[0], R.nrad[0], true);
    for (int e2 = threadIdx.x; e2 < nl * K; e2 += FFT_THREADS) {
      const int k = dnl.div(e2), l = e2 - k * nl;
      base[(long long)k * xstride + l] = fin[k * LBP + l];
    }
  }
  if (EV) {
    double v[7] = {acc.e, acc.w[0], acc.w[1], acc.w[2], acc.w[3], acc.w[4], acc.w[5]};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      double t = block_sum_fft<FFT_THREADS>(v[k], sh);
      if (threadIdx.x == 0) a.part[(size_t)item * PART_W + k] = t;
    }
  }
  wave_stamp(a.stamps, 1);
}

// y transform, x transform, Green's function (energy, virial), inverse x,
// inverse y of one kz plane of the half-complex mesh, all in LDS (for meshes
// whose K0 x K1 plane fits twice in a workgroup's LDS).  The plane stays in
// one layout, (y, x) at y*LY + x (LY = K0 + 1): the y lines are transformed
// with x interleaved, the x lines with their points consecutive.
template <typename T, bool EV, int KC, int NT>
__device__ __attribute__((always_inline)) inline void yx_plane(const PmeLaunch& a, const LineItem& it,
                                                                const RepDesc& R, int item) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sh[NT / 64];
  // KC > 0: this plane is KC x KC (compile-time transforms)
  const int K0 = KC > 0 ? KC : R.K[0], K1 = KC > 0 ? KC : R.K[1], K2h = R.K2h;
  const int kz = it.first;
  const int LY = K0 + 1;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + (size_t)a.plane_elems;
  cplx<T>* twx = B + (size_t)a.plane_elems;
  cplx<T>* twy = twx + a.maxK[2];
  // per-axis Green's function factors and frequencies of this replica
  T* tabs = reinterpret_cast<T*>(twy + a.maxK[1]);
  T* gf0 = tabs;
  T* gf1 = gf0 + K0;
  T* gf2 = gf1 + K1;
  T* fr0 = gf2 + K2h;
  T* fr1 = fr0 + K0;
  T* fr2 = fr1 + K1;
  // the plane is contiguous in the plane-major mesh layout
  const int n = K0 * K1;
  cplx<T>* Q = reinterpret_cast<cplx<T>*>(a.Qc) + R.cgrid_off + (long long)kz * n;
  const QDiv<KC> dk0(K0), dk1(K1);
  {
    // Every load of the first NT table entries and PL plane points per
    // thread is issued before the first LDS store, so the block waits for
    // one memory latency rather than one per table and per plane row.
    const int t = threadIdx.x;
    const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(a.tw);
    const T* gf = reinterpret_cast<const T*>(a.bsp);
    const T* fr = reinterpret_cast<const T*>(a.freq);
    constexpr int PL = 4;
    cplx<T> v[PL], wx = {}, wy = {};
    T g[3] = {}, f[3] = {};
#pragma unroll
    for (int u = 0; u < PL; ++u) v[u] = t + u * NT < n ? Q[t + u * NT] : cplx<T>{};
    if (t < K0) {
      wx = tw[R.tw_off[0] + t];
      g[0] = gf[R.bsp_off[0] + t];
      f[0] = fr[R.bsp_off[0] + t];
    }
    if (t < K1) {
      wy = tw[R.tw_off[1] + t];
      g[1] = gf[R.bsp_off[1] + t];
      f[1] = fr[R.bsp_off[1] + t];
    }
    if (t < K2h) {
      g[2] = gf[R.bsp_off[2] + t];
      f[2] = fr[R.bsp_off[2] + t];
    }
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int e = t + u * NT;
      if (e < n) {
        const int x = dk1.div(e), y = e - x * K1;
        A[y * LY + x] = v[u];
      }
    }
    if (t < K0) {
      twx[t] = wx;
      gf0[t] = g[0];
      fr0[t] = f[0];
    }
    if (t < K1) {
      twy[t] = wy;
      gf1[t] = g[1];
      fr1[t] = f[1];
    }
    if (t < K2h) {
      gf2[t] = g[2];
      fr2[t] = f[2];
    }
    // the rest, for meshes with more points than that
    for (int e = t + NT; e < K0; e += NT) {
      twx[e] = tw[R.tw_off[0] + e];
      gf0[e] = gf[R.bsp_off[0] + e];
      fr0[e] = fr[R.bsp_off[0] + e];
    }
    for (int e = t + NT; e < K1; e += NT) {
      twy[e] = tw[R.tw_off[1] + e];
      gf1[e] = gf[R.bsp_off[1] + e];
      fr1[e] = fr[R.bsp_off[1] + e];
    }
    for (int e = t + NT; e < K2h; e += NT) {
      gf2[e] = gf[R.bsp_off[2] + e];
      fr2[e] = fr[R.bsp_off[2] + e];
    }
    for (int e = t + PL * NT; e < n; e += NT) {
      const int x = dk1.div(e), y = e - x * K1;
      A[y * LY + x] = Q[e];
    }
  }
  __syncthreads();
  const int* radx = a.radix + R.rad_off[0];
  const int* rady = a.radix + R.rad_off[1];
  // y lines (x interleaved), then x lines in place in the same layout
  // (points of a line consecutive, lines LY apart): no transposes
  cplx<T>* r1;
  if constexpr (KC > 0)
    r1 = fft_lines_c<T, KC, NT, KC + 1, 1, KC>(A, B, twy, false);
  else
    r1 = fft_lines_s<T, NT>(A, B, K1, LY, 1, K0, twy, rady, R.nrad[1], false);
  cplx<T>* o1 = r1 == A ? B : A;
  cplx<T>* r2;
  if constexpr (KC > 0)
    r2 = fft_lines_c<T, KC, NT, 1, KC + 1, KC>(r1, o1, twx, false);
  else
    r2 = fft_lines_s<T, NT>(r1, o1, K0, 1, LY, K1, twx, radx, R.nrad[0], false);
  cplx<T>* o2 = r2 == r1 ? o1 : r1;
  RecipSums acc{};
  for (int e = threadIdx.x; e < n; e += NT) {
    const int y = dk0.div(e), x = e - y * K0;
    r2[y * LY + x] = green_apply<T, EV>(R, gf0, gf1, gf2, fr0, fr1, fr2, x, y, kz, r2[y * LY + x], acc);
  }
  __syncthreads();
  cplx<T>* r3;
  if constexpr (KC > 0)
    r3 = fft_lines_c<T, KC, NT, 1, KC + 1, KC>(r2, o2, twx, true);
  else
    r3 = fft_lines_s<T, NT>(r2, o2, K0, 1, LY, K1, twx, radx, R.nrad[0], true);
  cplx<T>* o3 = r3 == r2 ? o2 : r2;
  cplx<T>* r4;
  if constexpr (KC > 0)
    r4 = fft_lines_c<T, KC, NT, KC + 1, 1, KC>(r3, o3, twy, true);
  else
    r4 = fft_lines_s<T, NT>(r3, o3, K1, LY, 1, K0, twy, rady, R.nrad[1], true);
  for (int e = threadIdx.x; e < n; e += NT) {
    const int x = dk1.div(e), y = e - x * K1;
    Q[e] = r4[y * LY + x];
  }
  if (EV) {
    double v[7] = {acc.e, acc.w[0], acc.w[1], acc.w[2], acc.w[3], acc.w[4], acc.w[5]};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      double t = block_sum_fft<NT>(v[k], sh);
      if (threadIdx.x == 0) a.part[(size_t)item * PART_W + k] = t;
    }
  }
}

// KC > 0: every replica's plane is KC x KC.  KC == 0: each workgroup takes
// the compile-time transforms of its replica's plane when that is square
// with one of the sides the batched workloads use, else the run-time plan.
template <typename T, bool EV, int KC, int NT>
__global__ __launch_bounds__(NT) void k_fft_yx_conv(PmeLaunch a) {
  wave_stamp(a.stamps, 0);
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const LineItem it = a.items[0][item];
  const RepDesc& R = a.rep[it.rep];
  if constexpr (KC > 0) {
    yx_plane<T, EV, KC, NT>(a, it, R, item);
  } else {
    switch (R.K[0] == R.K[1] ? R.K[0] : 0) {
      case 16: yx_plane<T, EV, 16, NT>(a, it, R, item); break;
      case 18: yx_plane<T, EV, 18, NT>(a, it, R, item); break;
      case 24: yx_plane<T, EV, 24, NT>(a, it, R, item); break;
      case 27: yx_plane<T, EV, 27, NT>(a, it, R, item); break;
      case 32: yx_plane<T, EV, 32, NT>(a, it, R, item); break;
      case 36: yx_plane<T, EV, 36, NT>(a, it, R, item); break;
      case 48: yx_plane<T, EV, 48, NT>(a, it, R, item); break;
      default: yx_plane<T, EV, 0, NT>(a, it, R, item); break;
    }
  }
  wave_stamp(a.stamps, 1);
}

// Inclusive scan of one int per thread over the block (FFT_THREADS).
__device__ inline int block_scan_incl(int v, int* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
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

// Charged beads whose order-P stencil can meet a mesh tile: whole cell
// columns (all z) of the charged cell list over the cell range that holds
// the stencil base points k0 in [t0, t0 + n + P - 2] (mod K) on x and y.
struct TileCols {
  int lo[2], n[2];
};
__device__ inline TileCols tile_columns(const RepDesc& R, const MeshTile& mt, int P) {
  TileCols tc;
  const int t0[2] = {mt.x0, mt.y0};
  const int nt[2] = {mt.nxy & 0xffff, mt.nxy >> 16};
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const long long nc = R.nc[d], K = R.K[d];
    const int lo = (int)((t0[d] * nc) / K);
    const int hi = (int)(((long long)(t0[d] + nt[d] + P - 1) * nc) / K);
    if (hi - lo + 1 >= nc) {
      tc.lo[d] = 0;
      tc.n[d] = (int)nc;
    } else {
      tc.lo[d] = lo;
      tc.n[d] = hi - lo + 1;
    }
  }
  return tc;
}

// Start and count of this thread's column of the tile's columns cb.. (zero
// past the last column).
struct ColRun {
  int st, n;
};
template <int NT>
__device__ inline ColRun tile_column(const RepDesc& R, const TileCols& tc, const int* __restrict__ qstart, int cb) {
  const int c = cb + threadIdx.x;
  ColRun r{0, 0};
  if (c < tc.n[0] * tc.n[1]) {
    const int nx = R.nc[0], ny = R.nc[1], nz = R.nc[2];
    int cx = tc.lo[0] + c / tc.n[1], cy = tc.lo[1] + c % tc.n[1];
    cx -= cx >= nx ? nx : 0;
    cy -= cy >= ny ? ny : 0;
    const int base = R.cell_off + (cx * ny + cy) * nz;
    r.st = qstart[base];
    r.n = qstart[base + nz] - r.st;
  }
  return r;
}

// Calls f(q) for every charged bead q in the tile's columns for which
// keep(q) holds.  The kept beads are queued per wavefront and handed to f 64
// at a time, so every lane of a call but those of the last has a bead (the
// test alone rejects about half the candidates of a small tile).  Every
// thread of the block must call this; f runs on one lane per bead and uses
// no cross-lane operation.  work is 4 NT ints of LDS (the column table and
// the queues); first is tile_column(.., 0), which callers load early so that
// its latency overlaps other work.  The order in which beads reach f depends
// on timing: the callers only add integers.
template <int NT, typename Keep, typename F>
__device__ inline void for_tile_beads(const RepDesc& R, const TileCols& tc, const int* __restrict__ qstart,
                                      ColRun first, int* work, int* s_tot, int* scan_sh, Keep&& keep, F&& f) {
  int* s_cs = work;
  int* s_cp = work + NT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int* que = work + 2 * NT + wv * 128;
  int qn = 0;  // wavefront-uniform: queued beads
  const int ncol = tc.n[0] * tc.n[1];
  for (int cb = 0; cb < ncol; cb += NT) {
    const ColRun cr = cb == 0 ? first : tile_column<NT>(R, tc, qstart, cb);
    const int inc = block_scan_incl(cr.n, scan_sh);
    s_cs[threadIdx.x] = cr.st;
    s_cp[threadIdx.x] = inc - cr.n;
    if (threadIdx.x == NT - 1) *s_tot = inc;
    __syncthreads();
    const int tot = *s_tot, last = min(NT, ncol - cb) - 1;
    for (int e0 = wv * 64; e0 < tot; e0 += NT) {
      const int e = e0 + lane;
      int q = -1;
      if (e < tot) {
        // the last column whose prefix is <= e holds candidate e
        int lo = 0, hi = last;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_cp[mid] <= e)
            lo = mid;
          else
            hi = mid - 1;
        }
        q = s_cs[lo] + (e - s_cp[lo]);
        if (!keep(q)) q = -1;
      }
      const unsigned long long m = __ballot(q >= 0);
      if (q >= 0) que[qn + __popcll(m & ((1ull << lane) - 1ull))] = q;
      qn += __popcll(m);
      __builtin_amdgcn_wave_barrier();
      if (qn >= 64) {
        f(que[lane]);
        const int rest = qn - 64;
        const int v = lane < rest ? que[64 + lane] : 0;
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) que[lane] = v;
        __builtin_amdgcn_wave_barrier();
        qn = rest;
      }
    }
    // the column table is rewritten by the next column block
    __syncthreads();
  }
  if (lane < qn) f(que[lane]);
  __syncthreads();
}

// Complex entries of each of the two LDS line buffers of a tile pass: the
// packed lines (nl + 1) / 2 (+1 padding) of the longest z line; at least the
// spread's integer accumulators (nl lines of maxK2 + order - 1 entries, half
// a complex each) and the 4 FFT_THREADS ints of the bead enumeration, which
// use a buffer while it is free.
__host__ __device__ inline int tile_buf_elems(int maxK2, int nl, int order, int cplx_bytes) {
  int e = maxK2 * ((nl + 1) / 2 + 1);
  const int acc = (nl * (maxK2 + order - 1) + 1) / 2;
  const int work = (4 * FFT_THREADS * 4 + cplx_bytes - 1) / cplx_bytes;
  e = e > acc ? e : acc;
  return e > work ? e : work;
}

// w[i] <- w[i + s] for i < P - s (s in [0, P); the rest is not used).
template <typename T, int P>
__device__ inline void shift_down(T* w, int s) {
#pragma unroll
  for (int b = 1; b < P; b <<= 1) {
    const bool on = (s & b) != 0;
#pragma unroll
    for (int i = 0; i + b < P; ++i) w[i] = on ? w[i + b] : w[i];
  }
}

// The stencil offsets j of one axis whose mesh line (o - j mod K) lies in
// the tile's n lines, o the stencil base's offset from the tile origin (at
// most n + P - 2).  When the axis is longer than n + P - 2 no stencil point
// wraps into the tile, and they are the run j0 .. j0 + nv - 1 with
// line o - j0 - i; else every j is tried (j0 = 0, nv = P) and the caller
// tests each line.
struct StencilRun {
  int j0, nv;
  bool wrap;
};
template <int P>
__device__ inline StencilRun stencil_run(int o, int n, int K) {
  if (K >= n + P - 1) return {max(0, o - n + 1), min(P - 1, o) - max(0, o - n + 1) + 1, false};
  return {0, P, true};
}

// The packed z lines of a tile pass (np lines of K2 points, line stride
// LBP = np + 1): compile-time transforms for the z lengths and tile shapes
// of the bulk workloads (64-point lines in 4 x 4 tiles, 256-point lines in
// 4 x 4 and 8 x 4 tiles), the run-time plan otherwise.
template <typename T>
__device__ __attribute__((always_inline)) inline cplx<T>* z_lines(cplx<T>* A, cplx<T>* B, int K2, int np,
                                                                  const cplx<T>* tw, const int* rad, int nrad,
                                                                  bool inverse) {
  if (K2 == 64 && np == 8) return fft_lines_c<T, 64, FFT_THREADS, 9, 1, 8>(A, B, tw, inverse);
  if (K2 == 256 && np == 8) return fft_lines_c<T, 256, FFT_THREADS, 9, 1, 8>(A, B, tw, inverse);
  if (K2 == 256 && np == 16) return fft_lines_c<T, 256, FFT_THREADS, 17, 1, 16>(A, B, tw, inverse);
  return fft_lines<T, FFT_THREADS>(A, B, K2, np + 1, np, tw, rad, nrad, inverse);
}

// Offset of a stencil base point from the tile origin (mod K); the bead
// meets the tile iff it is at most n + P - 2.
__device__ inline int tile_off(int k0, int t0, int K) {
  int o = k0 - t0;
  return o < 0 ? o + K : o;
}

template <typename T, int P>
__global__ __launch_bounds__(FFT_THREADS) void k_spread_z(PmeLaunch a) {
  wave_stamp(a.stamps, 0);
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_tot, scan_sh[FFT_THREADS / 64];
  const MeshTile mt = a.tiles[xcd_item(blockIdx.x, gridDim.x)];
  const RepDesc& R = a.rep[mt.rep];
  const int K0 = R.K[0], K1 = R.K[1], K2 = R.K[2], K2h = R.K2h;
  // the tile's real z lines are transformed two to a complex line: line l
  // is the real (l even) or imaginary (l odd) part of packed line l / 2
  const int TY = a.ty, NL = a.tx * a.ty, NP = (NL + 1) >> 1, LBP = NP + 1;
  const int nxt = mt.nxy & 0xffff, nyt = mt.nxy >> 16;
  const int SB = tile_buf_elems(a.maxK[0], NL, P, (int)sizeof(cplx<T>));
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + SB;
  // the tile's first column run and this thread's twiddle are loaded first;
  // the twiddles go to LDS after the spread, so neither latency is waited
  // for on its own
  const TileCols tc = tile_columns(R, mt, P);
  const ColRun first = tile_column<FFT_THREADS>(R, tc, a.qstart, 0);
  cplx<T>* tw = B + SB;
  const cplx<T>* tws = reinterpret_cast<const cplx<T>*>(a.tw) + R.tw_off[2];
  const cplx<T> tw0 = threadIdx.x < K2 ? tws[threadIdx.x] : cplx<T>{};
  // integer accumulators of the tile in B (which the transform first writes
  // after they are read): line l = lx * TY + ly at l * KP, mesh point z at
  // z + P - 1, so that a stencil's P points are consecutive (those below
  // z = 0 are folded onto z + K2 afterwards)
  using U = typename MeshInt<T>::U;
  U* acc = reinterpret_cast<U*>(B);
  const int KP = K2 + P - 1;
  for (int e = threadIdx.x; e < NL * KP; e += FFT_THREADS) acc[e] = 0;
  __syncthreads();
  const double qs = a.qscale;
  auto keep = [&](int q) {
    const uint4 rec = a.qpk[q];
    const int ox = tile_off((int)(((unsigned long long)rec.x * (unsigned)K0) >> 32), mt.x0, K0);
    const int oy = tile_off((int)(((unsigned long long)rec.y * (unsigned)K1) >> 32), mt.y0, K1);
    return ox <= nxt + P - 2 && oy <= nyt + P - 2;
  };
  // A is free until the transform: the enumeration's tables go there
  for_tile_beads<FFT_THREADS>(R, tc, a.qstart, first, reinterpret_cast<int*>(A), &s_tot, scan_sh, keep, [&](int q) {
    const uint4 rec = a.qpk[q];
    int k0[3];
    T t[3];
    mesh_coord<T>(rec.x, K0, k0[0], t[0]);
    mesh_coord<T>(rec.y, K1, k0[1], t[1]);
    mesh_coord<T>(rec.z, K2, k0[2], t[2]);
    const int ox = tile_off(k0[0], mt.x0, K0), oy = tile_off(k0[1], mt.y0, K1);
    T w[3][P], dw[P];
#pragma unroll
    for (int d = 0; d < 3; ++d) bspline<T, P>(t[d], w[d], dw);
    const T z = (T)param_z(rec.w);
    // only the stencil rows and columns inside the tile: w[0][i], w[1][k]
    // become the weights of offsets jx0 + i, jy0 + k
    const StencilRun rx = stencil_run<P>(ox, nxt, K0), ry = stencil_run<P>(oy, nyt, K1);
    shift_down<T, P>(w[0], rx.j0);
    shift_down<T, P>(w[1], ry.j0);
    // the stencil's lowest z point (jz = P - 1) at accumulator offset k0z,
    // point jz at k0z + P - 1 - jz
    const int lx0 = ox - rx.j0, ly0 = oy - ry.j0;
    // at most min(P, n) offsets per axis can be inside (uniform bounds)
    const int mx = rx.wrap ? P : min(P, nxt), my = ry.wrap ? P : min(P, nyt);
    int rowy[P];
    bool oky[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      int ly = ly0 - k;
      ly += ly < 0 ? K1 : 0;
      oky[k] = k < my && k < ry.nv && ly < nyt;
      rowy[k] = ly * KP + k0[2];
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      int lx = lx0 - i;
      lx += lx < 0 ? K0 : 0;
      if (i >= mx || i >= rx.nv || lx >= nxt) continue;
      const T ax = z * w[0][i];
      U* const row = acc + lx * TY * KP;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        if (oky[k]) {
          const T axy = ax * w[1][k];
          U* pt = row + rowy[k];
          if constexpr (std::is_same<T, float>::value) {
            const float axs = axy * MeshInt<float>::scale;  // exact: a power of two
#pragma unroll
            for (int jz = 0; jz < P; ++jz) atomicAdd(&pt[P - 1 - jz], (unsigned)(int)rintf(axs * w[2][jz]));
          } else {
#pragma unroll
            for (int jz = 0; jz < P; ++jz) {
              const double v = (double)(axy * w[2][jz]) * qs;
              atomicAdd(&pt[P - 1 - jz], (unsigned long long)(long long)llrint(v));
            }
          }
        }
      }
    }
  });
  // fold the points below z = 0 onto z + K2 (K2 >= 2P: no double wrap)
  for (int e = threadIdx.x; e < NL * (P - 1); e += FFT_THREADS) {
    const int l = e / (P - 1), j = e - l * (P - 1);
    acc[l * KP + K2 + j] += acc[l * KP + j];
  }
  __syncthreads();
  if (threadIdx.x < K2) tw[threadIdx.x] = tw0;
  for (int e = threadIdx.x + FFT_THREADS; e < K2; e += FFT_THREADS) tw[e] = tws[e];
  // integer mesh -> packed lines: real point k of line l at AT[k * 2 LBP + l]
  // (a line past the tile's last is zero)
  const double inv_qs = 1.0 / qs;
  T* AT = reinterpret_cast<T*>(A);
  const FDiv dk2(K2), dk2h(K2h);
  for (int e = threadIdx.x; e < 2 * NP * K2; e += FFT_THREADS) {
    const int l = dk2.div(e), k = e - l * K2;
    T v = 0;
    if (l < NL) {
      const U c = acc[l * KP + P - 1 + k];
      if constexpr (std::is_same<T, float>::value)
        v = (float)(int)c * (1.0f / MeshInt<float>::scale);
      else
        v = (T)((double)(long long)c * inv_qs);
    }
    AT[k * 2 * LBP + l] = v;
  }
  __syncthreads();
  const cplx<T>* res = z_lines<T>(A, B, K2, NP, tw, a.radix + R.rad_off[2], R.nrad[2], false);
  cplx<T>* out = reinterpret_cast<cplx<T>*>(a.Qc) + R.cgrid_off;
  const FDiv dnl(NL), dty(TY);
  for (int e = threadIdx.x; e < NL * K2h; e += FFT_THREADS) {
    // consecutive threads take consecutive addresses of either layout
    int l, m;
    if (a.plane_major) {
      m = dnl.div(e);
      l = e - m * NL;
    } else {
      l = dk2h.div(e);
      m = e - l * K2h;
    }
    const int lx = dty.div(l), ly = l - lx * TY;
    if (lx < nxt && ly < nyt) {
      // packed transform Z = X + i Y of real lines x, y: X_m = (Z_m +
      // conj Z_-m) / 2, Y_m = (Z_m - conj Z_-m) / 2i
      const int p = l >> 1;
      const cplx<T> zm = res[m * LBP + p], zc = res[(m == 0 ? 0 : K2 - m) * LBP + p];
      const cplx<T> v = (l & 1) ? cplx<T>{(zm.y + zc.y) * (T)0.5, (zc.x - zm.x) * (T)0.5}
                                : cplx<T>{(zm.x + zc.x) * (T)0.5, (zm.y - zc.y) * (T)0.5};
      out[mesh_index(a, R, mt.x0 + lx, mt.y0 + ly, m)] = v;
    }
  }
  wave_stamp(a.stamps, 1);
}

template <typename T, int P>
__global__ __launch_bounds__(FFT_THREADS) void k_z_gather(PmeLaunch a) {
  wave_stamp(a.stamps, 0);
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_tot, scan_sh[FFT_THREADS / 64];
  const MeshTile mt = a.tiles[xcd_item(blockIdx.x, gridDim.x)];
  const RepDesc& R = a.rep[mt.rep];
  const int K0 = R.K[0], K1 = R.K[1], K2 = R.K[2], K2h = R.K2h;
  // the tile's real z lines come out of the inverse transform two to a
  // complex line: line l is the real (l even) or imaginary (l odd) part of
  // packed line l / 2
  const int TY = a.ty, NL = a.tx * a.ty, NP = (NL + 1) >> 1, LBP = NP + 1;
  const int nxt = mt.nxy & 0xffff, nyt = mt.nxy >> 16;
  const int SB = tile_buf_elems(a.maxK[0], NL, P, (int)sizeof(cplx<T>));
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + SB;
  const TileCols tc = tile_columns(R, mt, P);
  const ColRun first = tile_column<FFT_THREADS>(R, tc, a.qstart, 0);
  const cplx<T>* in = reinterpret_cast<const cplx<T>*>(a.Qc) + R.cgrid_off;
  const FDiv dk2h(K2h), dnp(NP), dty(TY);
  // mesh offset of frequency m of tile line l (negative outside the tile)
  auto offset = [&](int l, int m) -> long long {
    const int lx = dty.div(l), ly = l - lx * TY;
    return l < NL && lx < nxt && ly < nyt ? mesh_index(a, R, mt.x0 + lx, mt.y0 + ly, m) : -1;
  };
  // point e of the packed half-complex lines: packed line p, frequency m;
  // consecutive e take consecutive addresses of either layout
  auto point = [&](int e, int& p, int& m) {
    if (a.plane_major) {
      m = dnp.div(e);
      p = e - m * NP;
    } else {
      p = dk2h.div(e);
      m = e - p * K2h;
    }
  };
  // Z = X + i Y over the whole line from the half-complex X, Y of two real
  // lines (X_-m = conj X_m); at m = 0 and K2 / 2 only the real parts count
  auto put = [&](int p, int m, cplx<T> x, cplx<T> y) {
    const int mc = K2 - m;
    if (m == 0 || mc == m) {
      A[m * LBP + p] = {x.x, y.x};
    } else {
      A[m * LBP + p] = {x.x - y.y, x.y + y.x};
      A[mc * LBP + p] = {x.x + y.y, y.x - x.y};
    }
  };
  const int ne = NP * K2h;
  // the first PL points per thread are loaded together (one memory latency)
  constexpr int PL = 4;
  cplx<T> v[PL][2];
  int vp[PL], vm[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int e = threadIdx.x + u * FFT_THREADS;
    v[u][0] = v[u][1] = cplx<T>{};
    vp[u] = vm[u] = 0;
    if (e < ne) {
      point(e, vp[u], vm[u]);
      const long long o0 = offset(2 * vp[u], vm[u]), o1 = offset(2 * vp[u] + 1, vm[u]);
      if (o0 >= 0) v[u][0] = in[o0];
      if (o1 >= 0) v[u][1] = in[o1];
    }
  }
  const cplx<T>* tw = stage_twiddles<T, FFT_THREADS>(B + SB, a, R.tw_off[2], K2);
#pragma unroll
  for (int u = 0; u < PL; ++u)
    if (threadIdx.x + u * FFT_THREADS < ne) put(vp[u], vm[u], v[u][0], v[u][1]);
  for (int e = threadIdx.x + PL * FFT_THREADS; e < ne; e += FFT_THREADS) {
    int p, m;
    point(e, p, m);
    const long long o0 = offset(2 * p, m), o1 = offset(2 * p + 1, m);
    put(p, m, o0 >= 0 ? in[o0] : cplx<T>{}, o1 >= 0 ? in[o1] : cplx<T>{});
  }
  __syncthreads();
  // real point g of line l at phi[g * 2 LBP + l]
  const cplx<T>* res = z_lines<T>(A, B, K2, NP, tw, a.radix + R.rad_off[2], R.nrad[2], true);
  const T* phi = reinterpret_cast<const T*>(res);
  const double fx = -R.lB * K0 / R.L[0], fy = -R.lB * K1 / R.L[1], fz = -R.lB * K2 / R.L[2];
  auto keep = [&](int q) {
    const uint4 rec = a.qpk[q];
    const int ox = tile_off((int)(((unsigned long long)rec.x * (unsigned)K0) >> 32), mt.x0, K0);
    const int oy = tile_off((int)(((unsigned long long)rec.y * (unsigned)K1) >> 32), mt.y0, K1);
    return ox <= nxt + P - 2 && oy <= nyt + P - 2;
  };
  // the buffer the transform did not end in holds the enumeration's tables
  int* work = reinterpret_cast<int*>(res == A ? B : A);
  for_tile_beads<FFT_THREADS>(R, tc, a.qstart, first, work, &s_tot, scan_sh, keep, [&](int q) {
    const uint4 rec = a.qpk[q];
    const int bi = a.qidx[q];
    int k0[3];
    T t[3];
    mesh_coord<T>(rec.x, K0, k0[0], t[0]);
    mesh_coord<T>(rec.y, K1, k0[1], t[1]);
    mesh_coord<T>(rec.z, K2, k0[2], t[2]);
    const int ox = tile_off(k0[0], mt.x0, K0), oy = tile_off(k0[1], mt.y0, K1);
    T w[3][P], dw[3][P];
#pragma unroll
    for (int d = 0; d < 3; ++d) bspline<T, P>(t[d], w[d], dw[d]);
    // only the stencil rows and columns inside the tile: index i, k stands
    // for offset jx0 + i, jy0 + k
    const StencilRun rx = stencil_run<P>(ox, nxt, K0), ry = stencil_run<P>(oy, nyt, K1);
    shift_down<T, P>(w[0], rx.j0);
    shift_down<T, P>(dw[0], rx.j0);
    shift_down<T, P>(w[1], ry.j0);
    shift_down<T, P>(dw[1], ry.j0);
    int zo[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int g = k0[2] - j;
      zo[j] = (g < 0 ? g + K2 : g) * 2 * LBP;
    }
    const int lx0 = ox - rx.j0, ly0 = oy - ry.j0;
    const int mx = rx.wrap ? P : min(P, nxt), my = ry.wrap ? P : min(P, nyt);
    T gx = 0, gy = 0, gz = 0;
    // stencil loops unrolled so the weights stay in registers
    int rowy[P];
    bool oky[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      int ly = ly0 - k;
      ly += ly < 0 ? K1 : 0;
      oky[k] = k < my && k < ry.nv && ly < nyt;
      rowy[k] = ly;
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      int lx = lx0 - i;
      lx += lx < 0 ? K0 : 0;
      if (i >= mx || i >= rx.nv || lx >= nxt) continue;
      const int rowx = lx * TY;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        if (oky[k]) {
          const int l = rowx + rowy[k];
          T s0 = 0, s2 = 0;
#pragma unroll
          for (int jz = 0; jz < P; ++jz) {
            const T ph = phi[zo[jz] + l];
            s0 += w[2][jz] * ph;
            s2 += dw[2][jz] * ph;
          }
          gx += dw[0][i] * w[1][k] * s0;
          gy += w[0][i] * dw[1][k] * s0;
          gz += w[0][i] * w[1][k] * s2;
        }
      }
    }
    const double z = (double)param_z(rec.w);
    const double f[3] = {z * fx * (double)gx, z * fy * (double)gy, z * fz * (double)gz};
    long long iv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double v = f[d] * a.fscale;
      iv[d] = 0;
      if (fabs(v) < 4.0e18)
        iv[d] = (long long)llrint(v);
      else
        atomicOr(a.status, (unsigned)STATUS_FORCE_OVERFLOW);
    }
    atomicAdd((unsigned long long*)&a.F[0][bi], (unsigned long long)iv[0]);
    atomicAdd((unsigned long long*)&a.F[1][bi], (unsigned long long)iv[1]);
    atomicAdd((unsigned long long*)&a.F[2][bi], (unsigned long long)iv[2]);
  });
  wave_stamp(a.stamps, 1);
}

template <typename T>
void spread_z_p(hipStream_t s, const PmeLaunch& a, size_t sh) {
  dim3 g(a.ntiles), b(FFT_THREADS);
  switch (a.order) {
    case 3: hipLaunchKernelGGL((k_spread_z<T, 3>), g, b, sh, s, a); break;
    case 4: hipLaunchKernelGGL((k_spread_z<T, 4>), g, b, sh, s, a); break;
    case 5: hipLaunchKernelGGL((k_spread_z<T, 5>), g, b, sh, s, a); break;
    case 6: hipLaunchKernelGGL((k_spread_z<T, 6>), g, b, sh, s, a); break;
    case 7: hipLaunchKernelGGL((k_spread_z<T, 7>), g, b, sh, s, a); break;
    default: hipLaunchKernelGGL((k_spread_z<T, 8>), g, b, sh, s, a); break;
  }
}

template <typename T>
void z_gather_p(hipStream_t s, const PmeLaunch& a, size_t sh) {
  dim3 g(a.ntiles), b(FFT_THREADS);
  switch (a.order) {
    case 3: hipLaunchKernelGGL((k_z_gather<T, 3>), g, b, sh, s, a); break;
    case 4: hipLaunchKernelGGL((k_z_gather<T, 4>), g, b, sh, s, a); break;
    case 5: hipLaunchKernelGGL((k_z_gather<T, 5>), g, b, sh, s, a); break;
    case 6: hipLaunchKernelGGL((k_z_gather<T, 6>), g, b, sh, s, a); break;
    case 7: hipLaunchKernelGGL((k_z_gather<T, 7>), g, b, sh, s, a); break;
    default: hipLaunchKernelGGL((k_z_gather<T, 8>), g, b, sh, s, a); break;
  }
}

// Workgroups may use more than 64 KiB of dynamic LDS: raise a kernel's
// limit to what it is launched with.
void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

inline size_t lds_bytes(const PmeLaunch& a, int pass, bool fp64) {
  return (2 * (size_t)a.maxK[pass] * (size_t)(a.lb[pass] + 1) + a.maxK[pass]) * (fp64 ? 16 : 8);
}

}  // namespace

size_t pme_tile_lds_bytes(int maxK2, int tx, int ty, int order, bool fp64) {
  // two line buffers and the twiddles
  const int cs = fp64 ? 16 : 8;
  return (2 * (size_t)tile_buf_elems(maxK2, tx * ty, order, cs) + maxK2) * cs;
}

void launch_spread_z(hipStream_t s, const PmeLaunch& a, bool fp64) {
  if (a.ntiles <= 0) return;
  const size_t sh = pme_tile_lds_bytes(a.maxK[0], a.tx, a.ty, a.order, fp64);
  const int o = std::min(std::max(a.order, 3), 8) - 3;
  if (fp64) {
    static const void* fns[6] = {(const void*)k_spread_z<double, 3>, (const void*)k_spread_z<double, 4>,
                                 (const void*)k_spread_z<double, 5>, (const void*)k_spread_z<double, 6>,
                                 (const void*)k_spread_z<double, 7>, (const void*)k_spread_z<double, 8>};
    allow_lds(fns[o], sh);
    spread_z_p<double>(s, a, sh);
  } else {
    static const void* fns[6] = {(const void*)k_spread_z<float, 3>, (const void*)k_spread_z<float, 4>,
                                 (const void*)k_spread_z<float, 5>, (const void*)k_spread_z<float, 6>,
                                 (const void*)k_spread_z<float, 7>, (const void*)k_spread_z<float, 8>};
    allow_lds(fns[o], sh);
    spread_z_p<float>(s, a, sh);
  }
}

void launch_z_gather(hipStream_t s, const PmeLaunch& a, bool fp64) {
  if (a.ntiles <= 0) return;
  const size_t sh = pme_tile_lds_bytes(a.maxK[0], a.tx, a.ty, a.order, fp64);
  const int o = std::min(std::max(a.order, 3), 8) - 3;
  if (fp64) {
    static const void* fns[6] = {(const void*)k_z_gather<double, 3>, (const void*)k_z_gather<double, 4>,
                                 (const void*)k_z_gather<double, 5>, (const void*)k_z_gather<double, 6>,
                                 (const void*)k_z_gather<double, 7>, (const void*)k_z_gather<double, 8>};
    allow_lds(fns[o], sh);
    z_gather_p<double>(s, a, sh);
  } else {
    static const void* fns[6] = {(const void*)k_z_gather<float, 3>, (const void*)k_z_gather<float, 4>,
                                 (const void*)k_z_gather<float, 5>, (const void*)k_z_gather<float, 6>,
                                 (const void*)k_z_gather<float, 7>, (const void*)k_z_gather<float, 8>};
    allow_lds(fns[o], sh);
    z_gather_p<float>(s, a, sh);
  }
}

// the compile-time line passes: every replica's K0 = K1 = KC (plane_k) and
// the plan's lines per item equal LINE_LB
constexpr int LINE_LB = 8;

template <typename T, int KC>
void fft_y_k(hipStream_t s, const PmeLaunch& a, size_t sh, bool inverse) {
  allow_lds((const void*)k_fft_y<T, KC, LINE_LB>, sh);
  hipLaunchKernelGGL((k_fft_y<T, KC, LINE_LB>), dim3(a.nitems[1]), dim3(FFT_THREADS), sh, s, a, (int)inverse);
}

template <typename T>
void fft_y_t(hipStream_t s, const PmeLaunch& a, size_t sh, bool inverse) {
  const bool c = a.lb[1] == LINE_LB && a.maxK[1] == a.plane_k;
  if (c && a.plane_k == 256)
    fft_y_k<T, 256>(s, a, sh, inverse);
  else if (c && a.plane_k == 128)
    fft_y_k<T, 128>(s, a, sh, inverse);
  else
    fft_y_k<T, 0>(s, a, sh, inverse);
}

void launch_fft_y(hipStream_t s, const PmeLaunch& a, bool fp64, bool inverse) {
  if (a.nitems[1] <= 0) return;
  const size_t sh = lds_bytes(a, 1, fp64);
  if (fp64)
    fft_y_t<double>(s, a, sh, inverse);
  else
    fft_y_t<float>(s, a, sh, inverse);
}

int pme_plane_threads(int plane_elems) {
  // planes up to 48 x 48 (49 x 49 with padding; the small meshes of batched
  // replicas) have few butterflies per stage: four wavefronts per plane, so
  // that four planes share a compute unit instead of one plane's sixteen
  // mostly idle wavefronts
  return plane_elems <= 49 * 49 ? YX_SMALL_THREADS : YX_THREADS;
}

size_t pme_plane_lds_bytes(int plane_elems, int maxK0, int maxK1, int maxK2, bool fp64) {
  // two plane buffers, x and y twiddles, then six per-axis real tables
  return (2 * (size_t)plane_elems + maxK0 + maxK1) * (fp64 ? 16 : 8) + 2 * (size_t)(maxK0 + maxK1 + maxK2) * (fp64 ? 8 : 4);
}

template <typename T, bool EV, int KC, int NT>
void fft_yx_conv_k(hipStream_t s, const PmeLaunch& a, size_t sh) {
  allow_lds((const void*)k_fft_yx_conv<T, EV, KC, NT>, sh);
  hipLaunchKernelGGL((k_fft_yx_conv<T, EV, KC, NT>), dim3(a.nitems[0]), dim3(NT), sh, s, a);
}

template <typename T, bool EV>
void fft_yx_conv_t(hipStream_t s, const PmeLaunch& a, size_t sh) {
  if (a.plane_k == 64)
    fft_yx_conv_k<T, EV, 64, YX_THREADS>(s, a, sh);
  else if (a.plane_k == 32)
    fft_yx_conv_k<T, EV, 32, YX_SMALL_THREADS>(s, a, sh);
  else if (pme_plane_threads(a.plane_elems) == YX_SMALL_THREADS)
    fft_yx_conv_k<T, EV, 0, YX_SMALL_THREADS>(s, a, sh);
  else
    fft_yx_conv_k<T, EV, 0, YX_THREADS>(s, a, sh);
}

void launch_fft_yx_conv(hipStream_t s, const PmeLaunch& a, bool fp64, bool ev) {
  if (a.nitems[0] <= 0) return;
  const size_t sh = pme_plane_lds_bytes(a.plane_elems, a.maxK[2], a.maxK[1], a.maxK[0], fp64);
  if (fp64) {
    if (ev)
      fft_yx_conv_t<double, true>(s, a, sh);
    else
      fft_yx_conv_t<double, false>(s, a, sh);
  } else {
    if (ev)
      fft_yx_conv_t<float, true>(s, a, sh);
    else
      fft_yx_conv_t<float, false>(s, a, sh);
  }
}

template <typename T, bool EV, int KC>
void fft_x_conv_k(hipStream_t s, const PmeLaunch& a, size_t sh) {
  allow_lds((const void*)k_fft_x_conv<T, EV, KC, LINE_LB>, sh);
  hipLaunchKernelGGL((k_fft_x_conv<T, EV, KC, LINE_LB>), dim3(a.nitems[2]), dim3(FFT_THREADS), sh, s, a);
}

template <typename T, bool EV>
void fft_x_conv_t(hipStream_t s, const PmeLaunch& a, size_t sh) {
  const bool c = a.lb[2] == LINE_LB && a.maxK[2] == a.plane_k;
  if (c && a.plane_k == 256)
    fft_x_conv_k<T, EV, 256>(s, a, sh);
  else if (c && a.plane_k == 128)
    fft_x_conv_k<T, EV, 128>(s, a, sh);
  else
    fft_x_conv_k<T, EV, 0>(s, a, sh);
}

void launch_fft_x_conv(hipStream_t s, const PmeLaunch& a, bool fp64, bool ev) {
  if (a.nitems[2] <= 0) return;
  const size_t sh = lds_bytes(a, 2, fp64);
  if (fp64) {
    if (ev)
      fft_x_conv_t<double, true>(s, a, sh);
    else
      fft_x_conv_t<double, false>(s, a, sh);
  } else {
    if (ev)
      fft_x_conv_t<float, true>(s, a, sh);
    else
      fft_x_conv_t<float, false>(s, a, sh);
  }
}

}  // namespace gcme
