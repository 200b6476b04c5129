// Terms of the slab systems (section "Image charge effects on
// polyelectrolyte adsorption"): the slab correction for a slab with a vacuum
// gap along z (the nonmetal-electrode boxes, tripled along z for it, with
// the correction of Yeh and Berkowitz that the paper cites) and the harmonic
// bonds of the polyanion backbones.
//
// Slab correction, per replica with it switched on:
//   E = 2 pi lB M_z^2 / V,  M_z = sum_i z_i zeta_i  (zeta in [0, Lz)),
//   F_iz = -4 pi lB z_i M_z / V,  virial diag(E, E, -E).
// With fixed-point positions z_i u_iz is an integer (|z| < 2^7, u < 2^32),
// so M_z 2^32 / Lz is summed exactly in 64 bits: one pass writes a partial
// per 256-bead tile, the next sums the replica's partials (any order gives
// the same integer) and adds the force.
//
// Bonds, u = k/2 (r - b)^2 over the minimum image: the fractional
// fixed-point difference of two positions, read as a signed 32-bit integer,
// is the minimum-image separation exactly.  The bond list holds original
// bead indices; the permute of each step's sort records the sorted slot of
// every bead index, through which a bond finds its two beads.
#include "gcme_internal.h"

namespace gcme {

namespace {

constexpr int EX_THREADS = 256;

__device__ inline long long block_sum_i64(long long v, long long* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Fixed-order sum over the workgroup; valid in thread 0.
__device__ inline double block_sum_ex(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  return threadIdx.x == 0 ? ((sh[0] + sh[1]) + (sh[2] + sh[3])) : 0.0;
}

__device__ inline long long to_fixed_ex(double f, double scale, unsigned int* status) {
  const double v = f * scale;
  if (!(fabs(v) < 4.0e18)) {
    atomicOr(status, (unsigned)STATUS_FORCE_OVERFLOW);
    return 0;
  }
  return (long long)llrint(v);
}

__global__ __launch_bounds__(EX_THREADS) void k_slab_moment(SlabLaunch a, StateView B) {
  static_assert(EX_THREADS == 256, "four wavefronts");
  __shared__ long long sh[4];
  const Tile tile = a.tiles[blockIdx.x];
  long long v = 0;
  if (a.on[tile.rep] && (int)threadIdx.x < tile.count) {
    const int n = tile.first + threadIdx.x;
    v = (long long)param_z(B.param[n]) * (long long)B.pos[2][n];
  }
  const long long t = block_sum_i64(v, sh);
  if (threadIdx.x == 0) a.mz[blockIdx.x] = t;
}

__global__ __launch_bounds__(EX_THREADS) void k_slab_force(SlabLaunch a, StateView B) {
  __shared__ long long sh[4];
  const Tile tile = a.tiles[blockIdx.x];
  const int r = tile.rep;
  double* out = a.part + (size_t)blockIdx.x * PART_W;
  if (!a.on[r]) {
    if (threadIdx.x < PART_W) out[threadIdx.x] = 0.0;
    return;
  }
  const RepDesc& R = a.rep[r];
  // the replica's moment, exactly
  long long v = 0;
  for (int k = a.tile_off[r] + (int)threadIdx.x; k < a.tile_off[r + 1]; k += EX_THREADS) v += a.mz[k];
  const long long m = block_sum_i64(v, sh);
  const double Mz = (double)m * R.scaled[2];
  const double c = -4.0 * M_PI * R.lB * Mz / R.V;
  if ((int)threadIdx.x < tile.count) {
    const int n = tile.first + threadIdx.x;
    const int z = param_z(B.param[n]);
    if (z != 0)
      atomicAdd((unsigned long long*)&a.F[2][n], (unsigned long long)to_fixed_ex(c * (double)z, a.fscale, a.status));
  }
  if (threadIdx.x == 0) {
    const double E = tile.first == R.bead_off ? 2.0 * M_PI * R.lB * Mz * Mz / R.V : 0.0;
    out[0] = E;
    out[1] = E;
    out[2] = E;
    out[3] = -E;
    for (int k = 4; k < PART_W; ++k) out[k] = 0.0;
  }
}

__global__ __launch_bounds__(EX_THREADS) void k_bond(BondLaunch a, StateView B) {
  __shared__ double sh[4];
  const Tile tile = a.tiles[blockIdx.x];
  const RepDesc& R = a.rep[tile.rep];
  double e = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
  if ((int)threadIdx.x < tile.count) {
    const int2 bd = a.bonds[tile.first + threadIdx.x];
    int si = a.slot_of[bd.x], sj = a.slot_of[bd.y];
    if ((unsigned)si >= (unsigned)a.nbeads || (unsigned)sj >= (unsigned)a.nbeads) {
      // a bead the sort did not place (inconsistent counts): flagged, skipped
      atomicOr(a.status, (unsigned)STATUS_SLOT_MAP);
      si = sj = 0;
    }
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = (double)(int)(B.pos[k][si] - B.pos[k][sj]) * R.scaled[k];
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double kb = a.k[tile.rep], b = a.b[tile.rep];
    e = 0.5 * kb * (r - b) * (r - b);
    // force on bead i: -k (r - b) d / r
    const double g = r > 0.0 ? -kb * (r - b) / r : 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const long long f = to_fixed_ex(g * d[k], a.fscale, a.status);
      atomicAdd((unsigned long long*)&a.F[k][si], (unsigned long long)f);
      atomicAdd((unsigned long long*)&a.F[k][sj], (unsigned long long)(-f));
    }
    w[0] = d[0] * g * d[0];
    w[1] = d[1] * g * d[1];
    w[2] = d[2] * g * d[2];
    w[3] = d[0] * g * d[1];
    w[4] = d[0] * g * d[2];
    w[5] = d[1] * g * d[2];
  }
  double v[7] = {e, w[0], w[1], w[2], w[3], w[4], w[5]};
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    const double s = block_sum_ex(v[t], sh);
    if (threadIdx.x == 0) a.part[(size_t)blockIdx.x * PART_W + t] = s;
  }
}

// Method of image charges (metal electrodes at z = 0 and z = Lz of the real
// system, box 2 Lz long): the reflection (x, y, -z) of the source is, in
// fractional fixed point, (ux, uy, 2^32 - uz) exactly.  Sources are never
// images, so the reads and writes of one launch do not overlap.
__global__ __launch_bounds__(EX_THREADS) void k_images(ImageLaunch a, StateView A, CellView c) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.n) return;
  const int2 pr = a.pairs[m];
  const int si = c.slot_a[pr.x], ss = c.slot_a[pr.y];
  if ((unsigned)si >= (unsigned)a.nbeads || (unsigned)ss >= (unsigned)a.nbeads) {
    atomicOr(a.status, (unsigned)STATUS_SLOT_MAP);
    return;
  }
  const uint32_t ux = A.pos[0][ss], uy = A.pos[1][ss], uz = 0u - A.pos[2][ss];
  A.pos[0][si] = ux;
  A.pos[1][si] = uy;
  A.pos[2][si] = uz;
  const uint32_t prm = A.param[si];
  const int cid = cell_of(a.rep[param_rep(prm)], ux, uy, uz);
  const int old = c.cell[si];
  if (cid != old) {
    c.cell[si] = cid;
    atomicAdd(&c.counts[old], -1);
    atomicAdd(&c.counts[cid], 1);
    if (param_z(prm) != 0) {
      atomicAdd(&c.qcounts[old], -1);
      atomicAdd(&c.qcounts[cid], 1);
    }
  }
}

}  // namespace

void launch_images(hipStream_t s, const ImageLaunch& a, StateView A, CellView c) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(k_images, dim3((a.n + EX_THREADS - 1) / EX_THREADS), dim3(EX_THREADS), 0, s, a, A, c);
}

void launch_slab(hipStream_t s, const SlabLaunch& a, StateView B) {
  if (a.ntiles <= 0) return;
  hipLaunchKernelGGL(k_slab_moment, dim3(a.ntiles), dim3(EX_THREADS), 0, s, a, B);
  hipLaunchKernelGGL(k_slab_force, dim3(a.ntiles), dim3(EX_THREADS), 0, s, a, B);
}

void launch_bonds(hipStream_t s, const BondLaunch& a, StateView B) {
  if (a.ntiles <= 0) return;
  hipLaunchKernelGGL(k_bond, dim3(a.ntiles), dim3(EX_THREADS), 0, s, a, B);
}

}  // namespace gcme
