// The reciprocal term of eq. ewald summed exactly, for replicas that ask for
// it (gcme_params.kmax > 0) instead of the particle-mesh approximation:
//
//   U_recip = (2 pi lB / V) sum_{k != 0, |k| <= kmax} exp(-k^2/(4 beta^2)) / k^2 |S(k)|^2,
//   S(k)    = sum_j z_j exp(i k.r_j),   k = 2 pi (n0/L0, n1/L1, n2/L2),
//
// over the half space of integer vectors n, each standing for itself and -n
// (S(-k) is the conjugate of S(k)); the factor 2 is folded into ek.  The force
// is minus the gradient of that sum:
//
//   F_i = 2 z_i sum_{half space} ek k Im(S(k)* exp(i k.r_i)),
//
// and the virial of each k is ek |S|^2 (delta_ab - c k_a k_b) with
// c = 2 (1 + k^2/(4 beta^2)) / k^2.
//
// The phase is exact: with the fractional fixed-point position u = x/L 2^32,
// k.r / (2 pi) = sum_a n_a u_a / 2^32, and its fraction is the wrapping 32-bit
// integer sum n0 u0 + n1 u1 + n2 u2; read as a signed integer it is the phase
// in units of pi 2^-31, so sin and cos come from sincospi of a value in
// [-1, 1) with no large-argument reduction.
//
// Two passes, both tiled so that small replicas still fill many workgroups:
//   k_ewald_sk     64 wave vectors x 256 charged beads per workgroup (a
//                  wavefront per 64 beads, whose records are broadcast with
//                  readlane); partial S(k) per 256-bead chunk, each summed in
//                  a fixed order;
//   k_ewald_force  64 charged beads x 256 wave vectors per workgroup (a
//                  wavefront per 64 vectors): S(k) is completed from the
//                  chunks in a fixed order, every lane takes one bead, the
//                  four wavefronts' sums are combined in a fixed order and
//                  added to the 64-bit fixed-point forces; the tiles holding
//                  the first beads of a replica also sum the energy and
//                  virial of their vectors.
#include <type_traits>

#include "gcme_internal.h"

namespace gcme {

namespace {

constexpr int EW_THREADS = 256;

__device__ inline void sincos_pi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ inline void sincos_pi(double x, double* s, double* c) { sincospi(x, s, c); }

// lane j's value of v (j wave-uniform)
__device__ inline int lane_i(int v, int j) { return __builtin_amdgcn_readlane(v, j); }
__device__ inline float lane_t(float v, int j) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j)); }
__device__ inline double lane_t(double v, int j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Phase of wave vector n at fixed-point position u, in units of pi.
template <typename T>
__device__ inline T phase_pi(int n0, int n1, int n2, uint32_t ux, uint32_t uy, uint32_t uz) {
  const uint32_t ph = (uint32_t)n0 * ux + (uint32_t)n1 * uy + (uint32_t)n2 * uz;
  return (T)(int)ph * (T)4.656612873077392578125e-10;  // 2^-31
}

template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_ewald_sk(EwaldLaunch a) {
  static_assert(EW_SK_K == 64 && EW_SK_Q == 4 * 64, "one lane per vector, one wavefront per 64 beads");
  __shared__ double sre[4][64], sim[4][64];
  const EwaldItem it = a.items_s[blockIdx.x];
  const RepDesc& R = a.rep[it.rep];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = it.k0 + lane;
  const bool vk = k < R.ek_n;
  int n0 = 0, n1 = 0, n2 = 0;
  if (vk) {
    const EwaldK& e = a.kv[R.ek_off + k];
    n0 = e.n[0];
    n1 = e.n[1];
    n2 = e.n[2];
  }
  // this wavefront's beads: one record per lane, read back by every lane
  const int qb = it.q0 + wave * 64;
  const int nq = min(64, R.nq - qb);  // wave-uniform, may be <= 0
  uint4 rec = make_uint4(0u, 0u, 0u, 0u);
  if (lane < nq) rec = a.qpk[R.q_off + qb + lane];
  double sr = 0.0, si = 0.0;
  for (int j = 0; j < nq; ++j) {
    const uint32_t ux = (uint32_t)lane_i((int)rec.x, j), uy = (uint32_t)lane_i((int)rec.y, j),
                   uz = (uint32_t)lane_i((int)rec.z, j);
    const T z = (T)param_z((uint32_t)lane_i((int)rec.w, j));
    T s, c;
    sincos_pi(phase_pi<T>(n0, n1, n2, ux, uy, uz), &s, &c);
    sr += (double)(z * c);
    si += (double)(z * s);
  }
  sre[wave][lane] = sr;
  sim[wave][lane] = si;
  __syncthreads();
  if (wave == 0 && vk) {
    double* out = a.sp + 2 * (R.sp_off + (long long)(it.q0 / EW_SK_Q) * R.ek_n + k);
    out[0] = ((sre[0][lane] + sre[1][lane]) + sre[2][lane]) + sre[3][lane];
    out[1] = ((sim[0][lane] + sim[1][lane]) + sim[2][lane]) + sim[3][lane];
  }
}

__device__ inline long long to_fixed_ew(double f, double scale, unsigned int* status) {
  const double v = f * scale;
  if (!(fabs(v) < 4.0e18)) {
    atomicOr(status, (unsigned)STATUS_FORCE_OVERFLOW);
    return 0;
  }
  return (long long)llrint(v);
}

// Fixed-order sum over the workgroup; result valid in thread 0.
__device__ inline double block_sum_ew(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  return threadIdx.x == 0 ? ((sh[0] + sh[1]) + (sh[2] + sh[3])) : 0.0;
}

template <typename T, bool EV>
__global__ __launch_bounds__(EW_THREADS) void k_ewald_force(EwaldLaunch a) {
  static_assert(EW_F_Q == 64 && EW_F_K == 4 * 64, "one lane per bead, one wavefront per 64 vectors");
  __shared__ double fsh[3][4][64];
  __shared__ double red[4];
  const EwaldItem it = a.items_f[blockIdx.x];
  const RepDesc& R = a.rep[it.rep];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // this lane's wave vector: S(k) completed from the chunk partials in a
  // fixed order, and the force coefficients 2 ek Re S, 2 ek Im S
  const int kw = it.k0 + wave * 64;
  const int k = kw + lane;
  const bool vk = k < R.ek_n;
  int kn0 = 0, kn1 = 0, kn2 = 0;
  T cA = 0, cB = 0, kx = 0, ky = 0, kz = 0;
  double e = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
  if (vk) {
    const EwaldK& E = a.kv[R.ek_off + k];
    const int nch = (R.nq + EW_SK_Q - 1) / EW_SK_Q;
    double Sr = 0.0, Si = 0.0;
    for (int c = 0; c < nch; ++c) {
      const double* p = a.sp + 2 * (R.sp_off + (long long)c * R.ek_n + k);
      Sr += p[0];
      Si += p[1];
    }
    kn0 = E.n[0];
    kn1 = E.n[1];
    kn2 = E.n[2];
    cA = (T)(2.0 * E.ek * Sr);
    cB = (T)(2.0 * E.ek * Si);
    kx = (T)E.k[0];
    ky = (T)E.k[1];
    kz = (T)E.k[2];
    if (EV && it.q0 == 0) {
      e = E.ek * (Sr * Sr + Si * Si);
      w[0] = e * (1.0 - E.c * E.k[0] * E.k[0]);
      w[1] = e * (1.0 - E.c * E.k[1] * E.k[1]);
      w[2] = e * (1.0 - E.c * E.k[2] * E.k[2]);
      w[3] = -e * E.c * E.k[0] * E.k[1];
      w[4] = -e * E.c * E.k[0] * E.k[2];
      w[5] = -e * E.c * E.k[1] * E.k[2];
    }
  }
  // this lane's charged bead against the wavefront's vectors
  const int q = it.q0 + lane;
  const bool vq = q < R.nq;
  uint4 rec = make_uint4(0u, 0u, 0u, 0u);
  if (vq) rec = a.qpk[R.q_off + q];
  double fx = 0.0, fy = 0.0, fz = 0.0;
  const int nk = min(64, R.ek_n - kw);  // wave-uniform, may be <= 0
  for (int j = 0; j < nk; ++j) {
    const int m0 = lane_i(kn0, j), m1 = lane_i(kn1, j), m2 = lane_i(kn2, j);
    const T A = lane_t(cA, j), B = lane_t(cB, j);
    T s, c;
    sincos_pi(phase_pi<T>(m0, m1, m2, rec.x, rec.y, rec.z), &s, &c);
    // Im(S* e^{i phi}) = Re S sin phi - Im S cos phi
    const T g = A * s - B * c;
    fx += (double)(g * lane_t(kx, j));
    fy += (double)(g * lane_t(ky, j));
    fz += (double)(g * lane_t(kz, j));
  }
  fsh[0][wave][lane] = fx;
  fsh[1][wave][lane] = fy;
  fsh[2][wave][lane] = fz;
  __syncthreads();
  if (wave == 0 && vq) {
    const double z = (double)param_z(rec.w);
    const int bi = a.qidx[R.q_off + q];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double f = z * (((fsh[d][0][lane] + fsh[d][1][lane]) + fsh[d][2][lane]) + fsh[d][3][lane]);
      atomicAdd((unsigned long long*)&a.F[d][bi], (unsigned long long)to_fixed_ew(f, a.fscale, a.status));
    }
  }
  if (EV) {
    // energy and virial of the tile's vectors (carried by the tiles of the
    // first 64 beads only, so each vector counts once)
    double v[7] = {e, w[0], w[1], w[2], w[3], w[4], w[5]};
#pragma unroll
    for (int t = 0; t < 7; ++t) {
      const double s = block_sum_ew(v[t], red);
      if (threadIdx.x == 0) a.part[(size_t)blockIdx.x * PART_W + t] = s;
    }
  }
}

}  // namespace

void launch_ewald(hipStream_t s, const EwaldLaunch& a, bool fp64, bool ev) {
  if (a.nitems_s <= 0 || a.nitems_f <= 0) return;
  dim3 b(EW_THREADS);
  if (fp64) {
    hipLaunchKernelGGL(k_ewald_sk<double>, dim3(a.nitems_s), b, 0, s, a);
    if (ev)
      hipLaunchKernelGGL((k_ewald_force<double, true>), dim3(a.nitems_f), b, 0, s, a);
    else
      hipLaunchKernelGGL((k_ewald_force<double, false>), dim3(a.nitems_f), b, 0, s, a);
  } else {
    hipLaunchKernelGGL(k_ewald_sk<float>, dim3(a.nitems_s), b, 0, s, a);
    if (ev)
      hipLaunchKernelGGL((k_ewald_force<float, true>), dim3(a.nitems_f), b, 0, s, a);
    else
      hipLaunchKernelGGL((k_ewald_force<float, false>), dim3(a.nitems_f), b, 0, s, a);
  }
}

}  // namespace gcme
