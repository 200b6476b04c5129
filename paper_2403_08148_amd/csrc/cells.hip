// Cell list: wrap into fixed point, bin, scan, scatter and a deterministic
// permutation of the state into (cell, previous order) order.
//
// Positions are stored as 32-bit fractions of the box edge (u = x/L * 2^32),
// so the minimum-image separation of two beads is the wrapped 32-bit
// difference, and drift never leaves the box.  Beads of one cell are kept in
// their previous relative order (a stable counting sort), which makes every
// later sum over neighbours run in the same order on every rerun.
#include "gcme_internal.h"

namespace gcme {

namespace {

__global__ void k_ingest(const double* __restrict__ pos, long long ld, int N, const RepDesc* __restrict__ rep,
                         StateView A, long long* F0, long long* F1, long long* F2, int nF) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nF) {
    F0[s] = 0;
    F1[s] = 0;
    F2[s] = 0;
  }
  if (s >= N) return;
  int id = A.id[s];
  const RepDesc& R = rep[param_rep(A.param[s])];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double f = pos[k * ld + id] / R.L[k];
    f -= floor(f);
    // round to the nearest 2^-32 fraction; 2^32 wraps to 0
    unsigned long long u = (unsigned long long)llrint(f * 4294967296.0);
    A.pos[k][s] = (uint32_t)u;
  }
}

template <typename I>
__global__ void k_fill(I* p, I v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_bin(StateView A, const RepDesc* __restrict__ rep, CellView c, int N) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = s < N;
  const int si = active ? s : 0;
  const uint32_t p = A.param[si];
  const RepDesc& R = rep[param_rep(p)];
  const int id = c.slot_a ? A.id[si] : 0;
  bin_bead(c, R, A.pos[0][si], A.pos[1][si], A.pos[2][si], p, s, id, active);
}

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 4;
constexpr int SCAN_BLOCK = SCAN_THREADS * SCAN_PER_THREAD;
// up to this many scan blocks, each adds up the block sums before it itself
// (at most 2 SCAN_SUMS_MAX ints per block) instead of a k_scan_top launch
constexpr int SCAN_SUMS_MAX = 1024;

// Inclusive scan of one int per thread over a block of NT threads (a
// multiple of 64, at most 1024); sh holds NT / 64 ints.
template <int NT>
__device__ inline int block_incl_scan(int v, int* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  __syncthreads();
  if (lane == 63) sh[wid] = v;
  __syncthreads();
  int add = 0;
  for (int w = 0; w < wid; ++w) add += sh[w];
  return v + add;
}

// Exclusive scan of the n cell counts cnt into st (st[n] = the total) and,
// with fill, a copy of st in fill (the scatter's cursors).  One block of NT
// threads: the counts pass through buf (n ints of LDS), each thread sums a
// contiguous chunk, one block scan, then each thread writes its chunk.  The
// loads of U rounds are issued before any is stored.
template <int NT, int U>
__device__ inline void block_scan_counts(const int* cnt, int* st, int* fill, int n, int* buf, int* sh) {
  for (int i0 = threadIdx.x; i0 < n; i0 += U * NT) {
    int v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = i0 + u * NT < n ? cnt[i0 + u * NT] : 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * NT < n) buf[i0 + u * NT] = v[u];
  }
  __syncthreads();
  const int per = (n + NT - 1) / NT;
  const int lo = threadIdx.x * per, hi = min(lo + per, n);
  int s = 0;
  for (int i = lo; i < hi; i += 4) {
    int v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = i + u < hi ? buf[i + u] : 0;
    s += (v[0] + v[1]) + (v[2] + v[3]);
  }
  const int inc = block_incl_scan<NT>(s, sh);
  int run = inc - s;
  for (int i = lo; i < hi; i += 4) {
    int v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = i + u < hi ? buf[i + u] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i + u < hi) buf[i + u] = run;
      run += v[u];
    }
  }
  if (threadIdx.x == NT - 1) st[n] = inc;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) {
    const int v = buf[i];
    st[i] = v;
    if (fill) fill[i] = v;
  }
  __syncthreads();  // buf may be reused at once
}

// Whole scan in one block per array (block 0: all beads, block 1: charged
// beads) for grids of up to SINGLE_SCAN_MAX cells: each thread sums a
// contiguous chunk, one block scan, then each thread writes its chunk.
// Produces start (exclusive) and, for all beads, the scatter cursor
// fill = start.
constexpr int SINGLE_SCAN_THREADS = 1024;
constexpr int SCAN_UNROLL = 16;
constexpr int SINGLE_SCAN_MAX = 38912;  // counts staged in up to 152 KiB of LDS

__global__ __launch_bounds__(SINGLE_SCAN_THREADS) void k_scan_single(CellView c) {
  __shared__ int sh[SINGLE_SCAN_THREADS / 64];
  extern __shared__ __align__(16) int buf[];  // ncells entries
  if (c.step && blockIdx.x == 0 && threadIdx.x == 0) *c.step += 1ULL;
  if (blockIdx.x == 0)
    block_scan_counts<SINGLE_SCAN_THREADS, SCAN_UNROLL>(c.counts, c.start, c.fill, c.ncells, buf, sh);
  else
    block_scan_counts<SINGLE_SCAN_THREADS, SCAN_UNROLL>(c.qcounts, c.qstart, nullptr, c.ncells, buf, sh);
}

__global__ void k_scan_reduce(CellView c, int nb) {
  __shared__ int sh[8];
  int b = blockIdx.x;
  int base = b * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
  int s0 = 0, s1 = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    int i = base + k;
    if (i < c.ncells) {
      s0 += c.counts[i];
      s1 += c.qcounts[i];
    }
  }
  int t0 = block_incl_scan<SCAN_THREADS>(s0, sh);
  int t1 = block_incl_scan<SCAN_THREADS>(s1, sh);
  if (threadIdx.x == SCAN_THREADS - 1) {
    c.bsum[b] = t0;
    c.bsum[nb + b] = t1;
  }
}

// One block: exclusive scan of the block sums (both arrays).
__global__ void k_scan_top(CellView c, int nb) {
  __shared__ int sh[8];
  if (c.step && threadIdx.x == 0) *c.step += 1ULL;
  for (int arr = 0; arr < 2; ++arr) {
    int* bs = c.bsum + arr * nb;
    int carry = 0;
    for (int base = 0; base < nb; base += SCAN_THREADS) {
      int i = base + threadIdx.x;
      int v = i < nb ? bs[i] : 0;
      int inc = block_incl_scan<SCAN_THREADS>(v, sh);
      if (i < nb) bs[i] = carry + inc - v;
      __shared__ int tot;
      if (threadIdx.x == SCAN_THREADS - 1) tot = inc;
      __syncthreads();
      carry += tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      int* st = arr == 0 ? c.start : c.qstart;
      st[c.ncells] = carry;
    }
  }
}

// Last pass: each block's scan plus its offset.  With SUMS the block adds up
// the block sums before it itself (the raw ones of k_scan_reduce; cheap
// while there are few blocks), writes the totals from the last block and
// advances the step counter, so that k_scan_top is not launched; otherwise
// k_scan_top has turned the block sums into offsets.
template <bool SUMS>
__global__ void k_scan_apply(CellView c, int nb) {
  __shared__ int sh[8];
  __shared__ int off_sh[2];
  int b = blockIdx.x;
  int base = b * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
  if constexpr (SUMS) {
    if (c.step && b == 0 && threadIdx.x == 0) *c.step += 1ULL;
    int s0 = 0, s1 = 0;
    for (int k = threadIdx.x; k < b; k += SCAN_THREADS) {
      s0 += c.bsum[k];
      s1 += c.bsum[nb + k];
    }
    const int t0 = block_incl_scan<SCAN_THREADS>(s0, sh);
    __syncthreads();
    const int t1 = block_incl_scan<SCAN_THREADS>(s1, sh);
    if (threadIdx.x == SCAN_THREADS - 1) {
      off_sh[0] = t0;
      off_sh[1] = t1;
    }
    __syncthreads();
  }
  for (int arr = 0; arr < 2; ++arr) {
    const int* cnt = arr == 0 ? c.counts : c.qcounts;
    int* st = arr == 0 ? c.start : c.qstart;
    int v[SCAN_PER_THREAD];
    int tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
      int i = base + k;
      v[k] = i < c.ncells ? cnt[i] : 0;
      tot += v[k];
    }
    int inc = block_incl_scan<SCAN_THREADS>(tot, sh);
    const int off = SUMS ? off_sh[arr] : c.bsum[arr * nb + b];
    if (SUMS && b == nb - 1 && threadIdx.x == SCAN_THREADS - 1) st[c.ncells] = off + inc;
    int run = off + inc - tot;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
      int i = base + k;
      if (i < c.ncells) {
        st[i] = run;
        if (arr == 0) c.fill[i] = run;
      }
      run += v[k];
    }
    __syncthreads();
  }
}

__global__ void k_scatter(CellView c, int N) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = s < N;
  const int cid = active ? c.cell[s] : 0;
  // fill holds the cell's next free slot (initialised to start by the scan)
  const int slot = run_atomic_add(c.fill, cid, active);
  // (slots outside the population cannot come from consistent counts; they
  // are dropped rather than written out of bounds)
  if (active && (unsigned)slot < (unsigned)N) c.tmp[slot] = s;
}

// Position p of the scattered array holds bead s of cell c in arbitrary
// order; its final slot is start[c] + (number of beads of c with a smaller
// previous index).  Charged beads get the same rank among charged beads.
__global__ void k_permute(StateView A, StateView B, uint4* __restrict__ bpk, CellView c, ChargedView q, int N) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  // the counts were consumed by the scan: clear them for the next binning
  for (int k = p; k < c.ncells; k += gridDim.x * blockDim.x) {
    c.counts[k] = 0;
    c.qcounts[k] = 0;
  }
  if (p >= N) return;
  const int s = c.tmp[p];
  // bead s's own data is requested as soon as s is known, beside its cell
  const int cid = c.cell[s];
  const uint32_t prm = A.param[s];
  const uint32_t px = A.pos[0][s], py = A.pos[1][s], pz = A.pos[2][s];
  const double vx = A.vel[0][s], vy = A.vel[1][s], vz = A.vel[2][s];
  const int id = A.id[s];
  // (clamped to the population, so inconsistent counts cannot send an
  // access out of bounds)
  const int lo = max(0, c.start[cid]), hi = min(N, c.start[cid + 1]);
  const bool charged = param_z(prm) != 0;
  // the rank among the cell's beads: their indices PB at a time, then the
  // parameters of those before s (charged beads only), each batch of loads
  // issued together
  constexpr int PB = 8;
  int rank = 0, qrank = 0;
  for (int t0 = lo; t0 < hi; t0 += PB) {
    int o[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) o[u] = t0 + u < hi ? c.tmp[t0 + u] : N;
    uint32_t po[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) po[u] = charged && o[u] < s ? A.param[o[u]] : 0u;
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      rank += o[u] < s;
      qrank += param_z(po[u]) != 0;
    }
  }
  const int n = lo + rank;
  if (n >= N) return;
  B.pos[0][n] = px;
  B.pos[1][n] = py;
  B.pos[2][n] = pz;
  B.vel[0][n] = vx;
  B.vel[1][n] = vy;
  B.vel[2][n] = vz;
  B.param[n] = prm;
  B.id[n] = id;
  if (c.slot_of && (unsigned)id < (unsigned)N) c.slot_of[id] = n;
  const uint4 rec = make_uint4(px, py, pz, prm);
  bpk[n] = rec;
  if (charged) {
    const int qn = c.qstart[cid] + qrank;
    if ((unsigned)qn < (unsigned)c.qstart[c.ncells]) {
      q.pk[qn] = rec;
      q.idx[qn] = n;
    }
  }
}

__global__ void k_commit(StateView B, StateView A, int N) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    A.pos[k][s] = B.pos[k][s];
    A.vel[k][s] = B.vel[k][s];
  }
  A.param[s] = B.param[s];
  A.id[s] = B.id[s];
}

// Column clusters (see ColLaunch).  One block: the columns' cluster counts
// are staged in LDS (loads spread over the block), each thread then takes a
// contiguous run of columns, and a block scan of the runs' counts gives every
// column its first cluster slot, numbered from its replica's first slot.
// With `fill` the scan's threads write the clusters themselves (one column
// per thread at most); otherwise each column's first slot goes to colbase
// and k_col_fill writes them, one thread per column.
constexpr int COL_THREADS = 1024;
constexpr int COL_LDS_MAX = 36864;  // columns + replicas staged in LDS (144 KiB)

__global__ __launch_bounds__(COL_THREADS) void k_col_scan(ColLaunch a, bool fill) {
  __shared__ int sh[COL_THREADS / 64];
  extern __shared__ int lds[];
  int* rfirst = lds;            // [nrep]: global cluster count before each replica
  int* rend = lds + a.nrep;     // [nrep]: ... and after it
  int* cnt = lds + 2 * a.nrep;  // [ncols]: clusters per column, then their first slot
  wave_stamp(a.stamps, 0);
  const int n = a.ncols;
  const int sh_ci = __ffs(a.ci) - 1;
  // 1. the counts, four columns per thread in flight
  for (int c0 = threadIdx.x; c0 < n; c0 += 4 * COL_THREADS) {
    int lo[4], hi[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u * COL_THREADS;
      lo[u] = c < n ? a.coltab[c].x : 0;
      hi[u] = c < n ? a.coltab[c + 1].x : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      lo[u] = a.start[lo[u]];
      hi[u] = a.start[hi[u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u * COL_THREADS;
      if (c < n) cnt[c] = (hi[u] - lo[u] + a.ci - 1) >> sh_ci;
    }
  }
  __syncthreads();
  // 2. exclusive scan over contiguous runs of columns
  const int per = (n + COL_THREADS - 1) / COL_THREADS;
  const int lo = min(n, (int)threadIdx.x * per), hi = min(lo + per, n);
  int s = 0;
  for (int c = lo; c < hi; ++c) s += cnt[c];
  const int inc = block_incl_scan<COL_THREADS>(s, sh);
  int run = inc - s;
  for (int c = lo; c < hi; ++c) {
    const int v = cnt[c];
    cnt[c] = run;
    const int r = a.coltab[c].y;
    if (c == 0 || a.coltab[c - 1].y != r) rfirst[r] = run;
    run += v;
    if (c + 1 == n || a.coltab[c + 1].y != r) rend[r] = run;
  }
  __syncthreads();
  // 3. each replica's count, and the columns' first slots (or the clusters)
  for (int r = threadIdx.x; r < a.nrep; r += COL_THREADS) a.ncl[r] = rend[r] - rfirst[r];
  for (int c = threadIdx.x; c < n; c += COL_THREADS) {
    const int2 ct = a.coltab[c];
    const int slot = a.rep_base[ct.y] + cnt[c] - rfirst[ct.y];
    if (fill) {
      const int b = a.start[ct.x], e = a.start[a.coltab[c + 1].x];
      int sl = slot;
      for (int f = b; f < e; f += a.ci) a.cl[sl++] = make_int2(f, min(a.ci, e - f));
    } else {
      a.colbase[c] = slot;
    }
  }
  wave_stamp(a.stamps, 1);
}

__global__ void k_col_fill(ColLaunch a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncols) return;
  const int b = a.start[a.coltab[c].x], e = a.start[a.coltab[c + 1].x];
  int slot = a.colbase[c];
  for (int f = b; f < e; f += a.ci) a.cl[slot++] = make_int2(f, min(a.ci, e - f));
}

inline int nblk(long long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_ingest(hipStream_t s, const double* pos_soa, int N, long long ld, const RepDesc* rep,
                   const uint32_t* param, StateView A, long long* F, int nF) {
  (void)param;
  int n = N > nF ? N : nF;
  hipLaunchKernelGGL(k_ingest, dim3(nblk(n, 256)), dim3(256), 0, s, pos_soa, ld, N, rep, A, F, F + nF,
                     F + 2LL * nF, nF);
}

void launch_fill_i64(hipStream_t s, long long* p, long long v, long long n) {
  if (n <= 0) return;
  int b = nblk(n, 256);
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_fill<long long>, dim3(b), dim3(256), 0, s, p, v, n);
}

void launch_bin(hipStream_t s, StateView A, const RepDesc* rep, CellView c, int N) {
  hipLaunchKernelGGL(k_bin, dim3(nblk(N, BEAD_THREADS)), dim3(BEAD_THREADS), 0, s, A, rep, c, N);
}

void launch_scan(hipStream_t s, CellView c) {
  if (c.ncells <= SINGLE_SCAN_MAX) {
    const size_t sh = (size_t)c.ncells * 4;
    if (sh > 65536) (void)hipFuncSetAttribute((const void*)k_scan_single, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL(k_scan_single, dim3(2), dim3(SINGLE_SCAN_THREADS), sh, s, c);
    return;
  }
  int nb = nblk(c.ncells, SCAN_BLOCK);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_THREADS), 0, s, c, nb);
  if (nb <= SCAN_SUMS_MAX) {
    hipLaunchKernelGGL(k_scan_apply<true>, dim3(nb), dim3(SCAN_THREADS), 0, s, c, nb);
    return;
  }
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_THREADS), 0, s, c, nb);
  hipLaunchKernelGGL(k_scan_apply<false>, dim3(nb), dim3(SCAN_THREADS), 0, s, c, nb);
}

void launch_scatter(hipStream_t s, CellView c, int N) {
  hipLaunchKernelGGL(k_scatter, dim3(nblk(N, BEAD_THREADS)), dim3(BEAD_THREADS), 0, s, c, N);
}

void launch_permute(hipStream_t s, StateView A, StateView B, uint4* bpk, CellView c, ChargedView q, int N) {
  hipLaunchKernelGGL(k_permute, dim3(nblk(N, BEAD_THREADS)), dim3(BEAD_THREADS), 0, s, A, B, bpk, c, q, N);
}

int col_clusters_max_entries() { return COL_LDS_MAX; }

void launch_col_clusters(hipStream_t s, const ColLaunch& a) {
  if (a.ncols <= 0) return;
  const size_t sh = ((size_t)a.ncols + 2 * (size_t)a.nrep) * 4;
  if (sh > 65536) (void)hipFuncSetAttribute((const void*)k_col_scan, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  // one column per thread of the scan: it writes the clusters itself
  const bool fill = a.ncols <= COL_THREADS;
  hipLaunchKernelGGL(k_col_scan, dim3(1), dim3(COL_THREADS), sh, s, a, fill);
  if (!fill) hipLaunchKernelGGL(k_col_fill, dim3(nblk(a.ncols, 128)), dim3(128), 0, s, a);
}

void launch_commit(hipStream_t s, StateView B, StateView A, int N) {
  hipLaunchKernelGGL(k_commit, dim3(nblk(N, 256)), dim3(256), 0, s, B, A, N);
}

}  // namespace gcme
