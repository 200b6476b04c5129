// Integrators (velocity Verlet, BAOAB Langevin), output conversion and the
// fixed-order final reductions.
//
// Langevin noise: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
// counter (step, bead id, replica, 0) and key (seed, 0x67636d65); uniforms
// ((x >> 11) + 1/2) 2^-53; Box-Muller on (u0, u1) and (u2, u3).  Keying by
// the original bead id makes the noise independent of the cell ordering.
#include "gcme_internal.h"

namespace gcme {

namespace {

__device__ inline void philox4x64_10(unsigned long long x[4], unsigned long long k0, unsigned long long k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B97F4A7C15ULL;
      k1 += 0xBB67AE8584CAA73BULL;
    }
    const unsigned long long m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
    unsigned long long hi0 = __umul64hi(m0, x[0]), lo0 = m0 * x[0];
    unsigned long long hi1 = __umul64hi(m1, x[2]), lo1 = m1 * x[2];
    unsigned long long y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
  }
}

__device__ inline void gauss3(unsigned long long seed, unsigned long long step, unsigned long long id,
                              unsigned long long rep, double g[3]) {
  unsigned long long x[4] = {step, id, rep, 0ULL};
  philox4x64_10(x, seed, 0x67636d65ULL);
  double u[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = ((double)(x[k] >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
  double s1, c1, s3, c3;
  sincospi(2.0 * u[1], &s1, &c1);
  sincospi(2.0 * u[3], &s3, &c3);
  g[0] = r0 * c1;
  g[1] = r0 * s1;
  g[2] = r1 * c3;
}

__device__ inline uint32_t drift(uint32_t u, double dx, double L) {
  long long du = llrint(dx / L * 4294967296.0);
  return u + (uint32_t)du;
}

// First half of a step for one bead, from velocity v, position u and force
// f (already in force units): kick, then drift (velocity Verlet) or drift,
// Ornstein-Uhlenbeck noise, drift (BAOAB), with the noise of `step`.  A type
// of infinite mass (inverse mass 0, no noise amplitude) is held at rest.
__device__ inline void first_half(const IntLaunch& a, const RepDesc& R, int r, int t, unsigned long long step,
                                  int id, const double f[3], double v[3], uint32_t u[3]) {
  const double im = a.inv_mass[r * MAXT + t];
  const double dt = a.dt[r];
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = im == 0.0 ? 0.0 : v[k] + 0.5 * dt * f[k] * im;
  if (a.langevin[r]) {
    double g[3];
    gauss3(a.seed, step, (unsigned long long)id, (unsigned long long)r, g);
    const double c1 = a.c1[r], c2 = a.c2s[r * MAXT + t];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      u[k] = drift(u[k], 0.5 * dt * v[k], R.L[k]);
      v[k] = c1 * v[k] + c2 * g[k];
      u[k] = drift(u[k], 0.5 * dt * v[k], R.L[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = drift(u[k], dt * v[k], R.L[k]);
  }
}

template <bool BIN>
__global__ void k_int_first(IntLaunch a, StateView A, long long* F0, long long* F1, long long* F2, CellView c,
                            int N) {
  wave_stamp(a.stamps, 0);
  const int s0 = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = s0 < N;
  if (!BIN && !active) return;
  const int s = active ? s0 : 0;  // inactive lanes of the last wavefront only take part in the binning
  const uint32_t prm = A.param[s];
  const int r = param_rep(prm), t = param_type(prm);
  const RepDesc& R = a.rep[r];
  long long* Fk[3] = {F0, F1, F2};
  double f[3], v[3];
  uint32_t u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f[k] = (double)Fk[k][s] * a.fscale_inv;
    if (active) Fk[k][s] = 0;
    v[k] = A.vel[k][s];
    u[k] = A.pos[k][s];
  }
  const int id = A.id[s];
  first_half(a, R, r, t, *a.step, id, f, v, u);
  if (active) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      A.pos[k][s] = u[k];
      A.vel[k][s] = v[k];
    }
  }
  if (BIN) bin_bead(c, R, u[0], u[1], u[2], prm, s, id, active);
  wave_stamp(a.stamps, 1);
}

// The second half kick of the step just completed (as k_int_last, on the
// sorted copy B), then the first half of the next step (as k_int_first) and
// its binning, written to A.  The step counter already names the next step:
// the scan of the step's sort advanced it (one thread, where a count of the
// finished blocks would take one same-address atomic per block: 340 us per
// step at N = 2,097,152).
__global__ __launch_bounds__(BEAD_THREADS) void k_int_between(IntLaunch a, StateView B, StateView A, long long* F0,
                                                     long long* F1, long long* F2, CellView c, int N) {
  wave_stamp(a.stamps, 0);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long step = *a.step;
  const bool active = s < N;
  int cid = 0;
  uint32_t prm = 0;
  if (active) {
    prm = B.param[s];
    const int r = param_rep(prm), t = param_type(prm);
    const RepDesc& R = a.rep[r];
    const double im = a.inv_mass[r * MAXT + t];
    const double dt = a.dt[r];
    long long* Fk[3] = {F0, F1, F2};
    double f[3], v[3];
    uint32_t u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const long long fi = Fk[k][s];
      v[k] = B.vel[k][s] + 0.5 * dt * (double)fi * a.fscale_inv * im;
      f[k] = (double)fi * a.fscale_inv;
      Fk[k][s] = 0;
      u[k] = B.pos[k][s];
    }
    const int id = B.id[s];
    first_half(a, R, r, t, step, id, f, v, u);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      A.pos[k][s] = u[k];
      A.vel[k][s] = v[k];
    }
    A.param[s] = prm;
    A.id[s] = id;
    cid = cell_of(R, u[0], u[1], u[2]);
    c.cell[s] = cid;
    if (c.slot_a) c.slot_a[id] = s;
  }
  // the binning's counts, one atomic per run of equal cells in the wavefront
  (void)run_atomic_add(c.counts, cid, active);
  (void)run_atomic_add(c.qcounts, cid, active && param_z(prm) != 0);
  wave_stamp(a.stamps, 1);
}

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

// Second half kick on the sorted copy B, written back to A (so the state is
// left in the order the forces are indexed in).  One tile per block.
template <bool KIN>
__global__ __launch_bounds__(256) void k_int_last(IntLaunch a, StateView B, StateView A, long long* F0,
                                                  long long* F1, long long* F2) {
  wave_stamp(a.stamps, 0);
  __shared__ double sh[4];
  const Tile tile = a.tiles[blockIdx.x];
  const bool active = (int)threadIdx.x < tile.count;
  const int n = tile.first + (active ? (int)threadIdx.x : 0);
  double ke = 0;
  if (active) {
    const uint32_t prm = B.param[n];
    const int r = tile.rep, t = param_type(prm);
    const double im = a.inv_mass[r * MAXT + t];
    const double dt = a.dt[r];
    long long* Fk[3] = {F0, F1, F2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double v = B.vel[k][n] + 0.5 * dt * (double)Fk[k][n] * a.fscale_inv * im;
      A.vel[k][n] = v;
      A.pos[k][n] = B.pos[k][n];
      ke += im == 0.0 ? 0.0 : 0.5 * v * v / im;
    }
    A.param[n] = prm;
    A.id[n] = B.id[n];
  }
  if (KIN) {
    double t = block_sum(ke, sh);
    if (threadIdx.x == 0) {
      a.part[(size_t)blockIdx.x * PART_W + 0] = t;
      for (int k = 1; k < PART_W; ++k) a.part[(size_t)blockIdx.x * PART_W + k] = 0.0;
    }
  }
  wave_stamp(a.stamps, 1);
}

__global__ void k_forces_out(StateView B, long long* F0, long long* F1, long long* F2, double* out, long long ld,
                             int N, double sc) {
  int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  int id = B.id[n];
  out[id] = (double)F0[n] * sc;
  out[ld + id] = (double)F1[n] * sc;
  out[2 * ld + id] = (double)F2[n] * sc;
}

__global__ void k_gather_vjp(StateView B, const double* v, double* vs, int N) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int id = B.id[n];
#pragma unroll
  for (int k = 0; k < 3; ++k) vs[(size_t)k * N + n] = v[(size_t)k * N + id];
}

__global__ void k_bead_adj_out(StateView B, const double* dg, const double* dq, const double* self_a,
                               double* out_s, double* out_a, int N) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int id = B.id[n];
  const uint32_t prm = B.param[n];
  const int z = param_z(prm);
  if (out_s) out_s[id] = dg[n];
  if (out_a) out_a[id] = dq[n] + self_a[param_rep(prm) * MAXT + param_type(prm)] * (double)(z * z);
}

__global__ void k_state_out(StateView A, const RepDesc* rep, double* pos, double* vel, long long ld, int N) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  int id = A.id[s];
  const RepDesc& R = rep[param_rep(A.param[s])];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (pos) pos[k * ld + id] = (double)A.pos[k][s] * R.scaled[k];
    if (vel) vel[k * ld + id] = A.vel[k][s];
  }
}

// Fixed-order sum of the partial-sum rows [lo, hi) of one slot: thread t
// takes rows lo + t, lo + t + 256, ... in order, then a fixed tree.
__device__ inline double slot_sum(const double* part, int lo, int hi, int col, double* sh) {
  double v = 0;
  for (int r = lo + (int)threadIdx.x; r < hi; r += blockDim.x) v += part[(size_t)r * PART_W + col];
  return block_sum(v, sh);
}

__device__ inline double adj_sum(const double* part, int lo, int hi, int col, double* sh) {
  constexpr int W = MAXT * MAXT + 2 * MAXT;
  double v = 0;
  for (int r = lo + (int)threadIdx.x; r < hi; r += blockDim.x) v += part[(size_t)r * W + col];
  return block_sum(v, sh);
}

__global__ __launch_bounds__(256) void k_finalize(FinalLaunch a) {
  __shared__ double sh[4];
  __shared__ double res[N_SLOTS][7];
  const int r = blockIdx.x;
  for (int sl = 0; sl < N_SLOTS; ++sl) {
    for (int col = 0; col < 7; ++col) {
      double t = 0;
      if (a.part[sl] && (sl != SLOT_KIN || a.have_kin)) {
        t = slot_sum(a.part[sl], a.slot_off[sl][r], a.slot_off[sl][r + 1], col, sh);
      } else {
        __syncthreads();
        __syncthreads();
      }
      if (threadIdx.x == 0) res[sl][col] = t;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double ec = a.consts[2 * r], es = a.consts[2 * r + 1];
    if (a.energy) {
      double* E = a.energy + (size_t)r * N_TERMS;
      E[0] = res[SLOT_GCM][0];
      E[1] = res[SLOT_REAL][0];
      E[2] = res[SLOT_RECIP][0] + res[SLOT_EWALD][0];  // a replica has one of the two
      E[3] = ec;
      E[4] = es;
      E[7] = res[SLOT_SLAB][0];
      E[8] = res[SLOT_BOND][0];
      E[5] = (((E[0] + E[1]) + (E[2] + E[3])) + E[4]) + (E[7] + E[8]);
      E[6] = a.have_kin ? res[SLOT_KIN][0] : 0.0;
    }
    if (a.virial) {
      for (int k = 0; k < 6; ++k)
        a.virial[(size_t)r * 6 + k] =
            ((res[SLOT_GCM][1 + k] + res[SLOT_REAL][1 + k]) + (res[SLOT_RECIP][1 + k] + res[SLOT_EWALD][1 + k])) +
            (res[SLOT_SLAB][1 + k] + res[SLOT_BOND][1 + k]);
    }
  }
  if (a.dE_dA || a.dE_dsigma || a.dE_da) {
    __shared__ double ett[MAXT * MAXT], dsg[MAXT], dea[MAXT];
    for (int q = 0; q < MAXT * MAXT; ++q) {
      double t = adj_sum(a.adj_part[0], a.adj_off[0][r], a.adj_off[0][r + 1], q, sh);
      if (threadIdx.x == 0) ett[q] = t;
    }
    for (int t2 = 0; t2 < MAXT; ++t2) {
      double t = adj_sum(a.adj_part[0], a.adj_off[0][r], a.adj_off[0][r + 1], MAXT * MAXT + t2, sh);
      if (threadIdx.x == 0) dsg[t2] = t;
    }
    for (int t2 = 0; t2 < MAXT; ++t2) {
      double t = 0;
      if (a.adj_part[1])
        t = adj_sum(a.adj_part[1], a.adj_off[1][r], a.adj_off[1][r + 1], MAXT * MAXT + MAXT + t2, sh);
      else {
        __syncthreads();
        __syncthreads();
      }
      if (threadIdx.x == 0) dea[t2] = t;
    }
    if (threadIdx.x == 0) {
      for (int t = 0; t < MAXT; ++t) {
        for (int u = 0; u < MAXT; ++u) {
          // unordered type-pair energy: both visiting orders
          double E = t == u ? ett[t * MAXT + t] : ett[t * MAXT + u] + ett[u * MAXT + t];
          double A = a.Avals[(size_t)r * MAXT * MAXT + t * MAXT + u];
          if (a.dE_dA) a.dE_dA[(size_t)r * MAXT * MAXT + t * MAXT + u] = A != 0.0 ? a.adj_scale * E / A : 0.0;
        }
        if (a.dE_dsigma) a.dE_dsigma[(size_t)r * MAXT + t] = a.adj_scale * dsg[t];
        if (a.dE_da)
          a.dE_da[(size_t)r * MAXT + t] = a.adj_scale * dea[t] + (a.vjp ? 0.0 : a.dself[(size_t)r * MAXT + t]);
      }
    }
  }
}

inline int nblk(long long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_int_first(hipStream_t s, const IntLaunch& a, StateView A, long long* const F[3], const CellView* bin) {
  if (bin)
    hipLaunchKernelGGL(k_int_first<true>, dim3(nblk(a.nbeads, BEAD_THREADS)), dim3(BEAD_THREADS), 0, s, a, A, F[0], F[1], F[2], *bin,
                       a.nbeads);
  else
    hipLaunchKernelGGL(k_int_first<false>, dim3(nblk(a.nbeads, BEAD_THREADS)), dim3(BEAD_THREADS), 0, s, a, A, F[0], F[1], F[2],
                       CellView{}, a.nbeads);
}

void launch_int_between(hipStream_t s, const IntLaunch& a, StateView B, StateView A, long long* const F[3],
                        const CellView& bin) {
  hipLaunchKernelGGL(k_int_between, dim3(nblk(a.nbeads, BEAD_THREADS)), dim3(BEAD_THREADS), 0, s, a, B, A, F[0], F[1], F[2], bin,
                     a.nbeads);
}

void launch_int_last(hipStream_t s, const IntLaunch& a, StateView B, StateView A, long long* const F[3], bool kin) {
  if (kin)
    hipLaunchKernelGGL(k_int_last<true>, dim3(a.ntiles), dim3(256), 0, s, a, B, A, F[0], F[1], F[2]);
  else
    hipLaunchKernelGGL(k_int_last<false>, dim3(a.ntiles), dim3(256), 0, s, a, B, A, F[0], F[1], F[2]);
}

void launch_forces_out(hipStream_t s, StateView B, long long* const F[3], double* out, long long ld, int N,
                       double fscale_inv) {
  hipLaunchKernelGGL(k_forces_out, dim3(nblk(N, 256)), dim3(256), 0, s, B, F[0], F[1], F[2], out, ld, N,
                     fscale_inv);
}

void launch_gather_vjp(hipStream_t s, StateView B, const double* v, double* vs, int N) {
  hipLaunchKernelGGL(k_gather_vjp, dim3(nblk(N, 256)), dim3(256), 0, s, B, v, vs, N);
}

void launch_bead_adj_out(hipStream_t s, StateView B, const double* dg, const double* dq, const double* self_a,
                         double* out_sigma, double* out_a, int N) {
  hipLaunchKernelGGL(k_bead_adj_out, dim3(nblk(N, 256)), dim3(256), 0, s, B, dg, dq, self_a, out_sigma, out_a, N);
}

void launch_state_out(hipStream_t s, StateView A, const RepDesc* rep, double* pos, double* vel, long long ld,
                      int N) {
  hipLaunchKernelGGL(k_state_out, dim3(nblk(N, 256)), dim3(256), 0, s, A, rep, pos, vel, ld, N);
}

void launch_finalize(hipStream_t s, const FinalLaunch& a) {
  hipLaunchKernelGGL(k_finalize, dim3(a.nrep), dim3(256), 0, s, a);
}

}  // namespace gcme
