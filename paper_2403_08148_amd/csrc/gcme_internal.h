// Internal device structures and kernel launchers of the GCMe engine.
// Every kernel is hand-written HIP for gfx950 (64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcme {

constexpr int MAXT = 4;           // bead types per replica
constexpr int NSER = 14;          // small-r series terms stored per type pair
constexpr int TILE = 256;         // beads per tile of the per-bead kernels
constexpr int FFT_THREADS = 256;  // threads of a mesh-line work item
constexpr int YX_THREADS = 1024;  // threads of a fused y/x plane work item
constexpr int YX_SMALL_THREADS = 256;  // the same for planes up to 48 x 48

// Fixed-point scales (log2) of the force and charge-mesh accumulators.
constexpr int FSHIFT_MIXED = 32;
constexpr int FSHIFT_FP64 = 40;

// Per-replica geometry and method constants (device resident).
struct RepDesc {
  double L[3];
  double V;
  double rc, rc2;
  double beta, lB;
  double scaled[3];   // L / 2^32: fixed-point unit in length units
  float scalef[3];
  float rc2f;
  float betaf, lBf;
  float hf[3];        // cell edge
  int nc[3];          // cells per axis
  int reach[3];       // stencil half-width in cells; -1 = take the whole axis
  int nreach[3];      // ceil(rc / cell edge): neighbourhood half-width of a brick
  int cell_off;       // first global cell id
  int col_off;        // first global cell column (nc[0] nc[1] columns of nc[2] cells)
  int bead_off, n;    // bead range in the concatenated arrays
  int q_off, nq;      // charged-bead range in the compacted charged arrays
  int K[3];
  int K2h;            // K2/2 + 1
  int K2s;            // row stride of the (x, y, m) mesh layout: K2h rounded up
                      // to a multiple of 8, so that the line-batched passes'
                      // 8-line segments start on 64-byte boundaries
  long long grid_off;   // real mesh offset (K0 K1 K2 entries)
  long long cgrid_off;  // half-complex mesh offset (K0 K1 K2h entries)
  int order;
  int nt;
  int tw_off[3];      // twiddle table offset for the length of each axis
  int bsp_off[3];     // offsets of the Green factor and m/L tables per axis
  int rad_off[3];     // offset of the radix list of each axis length
  int nrad[3];
  // exact reciprocal sum (replicas with kmax > 0, which have no mesh: K = 0)
  int ek_off, ek_n;   // the replica's wave vectors in the k table
  long long sp_off;   // its partial structure factors, [charged chunk][ek_n]
};

// Pair coefficients of one type pair for the excluded-volume term:
// u = C exp2(-bl r^2), force/r = twob * u.
template <typename T>
struct GcmPar {
  T C, bl, twob;
  T fC;  // twob C: force/r = fC exp2(-bl r^2)
};

// Real-space smeared-Coulomb coefficients of one type pair.
// phi(r) = [erf(alpha r) - erf(beta r)]/r, g(r) = -(1/r) dphi/dr.
// For r^2 < rs2 both come from the series in r^2 with coefficients cphi, cg.
template <typename T>
struct ElecPar {
  T alpha, alpha2, rs2;
  T cexp;       // -alpha^2 log2(e): exp(-alpha^2 r^2) = 2^(cexp r^2)
  T tsa;        // (2/sqrt(pi)) alpha
  T pad[3];
  T cphi[NSER];
  T cg[NSER];
};

// Adjoint coefficients (derivatives with respect to sigma_ij and a_ij).
template <typename T>
struct AdjPar {
  T inv_s2;     // 1 / s_ij^2
  T dsig_i;     // sigma_ti / s_ij  (chain factor for d/dsigma_ti)
  T dsig_j;
  T s_inv;      // 1 / s_ij
  T daij_i;     // a_ti / a_ij
  T daij_j;
  T ea;         // (2/sqrt(pi)) alpha / a_ij
  T pad;
};

// One mesh-line work item: `count` lines of one replica starting at line
// index `first` of the pass (lines are enumerated per pass, see pme kernels).
struct LineItem {
  int rep;
  int first;
  int count;
  int pad;
};

// A tile of the mesh for the fused spread / gather passes: the z lines
// x0 <= x < x0 + nx, y0 <= y < y0 + ny of one replica (nxy = nx | ny << 16).
struct MeshTile {
  int rep;
  int x0, y0;
  int nxy;
};

// Tiles of consecutive beads (per-bead kernels) or of consecutive clusters
// (pair kernels) of one replica.
struct Tile {
  int rep;
  int first;   // first bead (concatenated index); pair tiles: first cluster
  int count;   // <= beads per tile; pair tiles: clusters
  int bead0;   // pair tiles: first bead of the first cluster (clusters of a
               // replica are consecutive runs of CI beads, the last one short)
};

// Workgroup size of the one-thread-per-bead kernels (binning, scatter,
// permute, integrator halves): one wavefront, so that even the 32,768-bead
// workloads spread over every compute unit.
constexpr int BEAD_THREADS = 256;

// Slots of the per-block partial sums (7 doubles: energy, virial[6]).
enum {
  SLOT_GCM = 0,
  SLOT_REAL = 1,
  SLOT_RECIP = 2,
  SLOT_KIN = 3,
  SLOT_EWALD = 4,
  SLOT_SLAB = 5,
  SLOT_BOND = 6,
  N_SLOTS = 7
};
constexpr int PART_W = 8;
// Width of a replica's energy row: ex, real, recip, corr, self, potential,
// kinetic, slab, bond.
constexpr int N_TERMS = 9;

// Device status bits.
// STATUS_SLOT_MAP: a bond or image named a bead the sort did not place
// (inconsistent cell counts); the term was skipped.
// The charge mesh has no status bit: in single precision a point is summed
// in 32-bit integers at 2^-24 of a unit charge (range +-128 unit charges);
// it collects z_i w_x w_y w_z from the beads within p mesh cells, each
// weight product at most (max M_p)^3 (0.42 for p = 3, 0.22 for p = 5), so
// it wraps only if several hundred unit charges of one sign crowd into a
// p^3-cell neighbourhood (300 at p = 3, 600 at p = 5).
// Double precision sums in 64 bits at 2^-40 (range 2^23 unit charges).
enum { STATUS_FORCE_OVERFLOW = 1, STATUS_LIST_OVERFLOW = 4, STATUS_SLOT_MAP = 8 };

// Bead parameter word: bits 0..7 type, 8..15 charge (int8), 16..31 replica.
__host__ __device__ inline uint32_t pack_param(int t, int z, int rep) {
  return (uint32_t)(t & 0xff) | ((uint32_t)(z & 0xff) << 8) | ((uint32_t)rep << 16);
}
__host__ __device__ inline int param_type(uint32_t p) { return (int)(p & 0xff); }
__host__ __device__ inline int param_z(uint32_t p) { return (int)(int8_t)((p >> 8) & 0xff); }
__host__ __device__ inline int param_rep(uint32_t p) { return (int)(p >> 16); }

// Arrays of the dynamic state (SoA).
struct StateView {
  uint32_t* pos[3];  // fractional fixed point: x / L * 2^32
  double* vel[3];
  uint32_t* param;
  int* id;           // original (concatenated) bead index
};

struct CellView {
  int* cell;         // [N] cell id of each bead of the unsorted array
  int* tmp;          // [N] bead indices scattered by cell
  int* counts;       // [Ncells]
  int* qcounts;      // [Ncells]
  int* fill;         // [Ncells]
  int* start;        // [Ncells + 1]
  int* qstart;       // [Ncells + 1]
  int* bsum;         // scan block sums [2 * nblocks]
  unsigned long long* step;  // with a step's sort: the step counter, which the
                             // scan advances by one (one thread); else null
  int* slot_of;      // [N] sorted index of each original bead index, written
                     // by the permute; null when nothing reads it (no bonds)
  int* slot_a;       // [N] index in the unsorted array of each original bead
                     // index, written by the binning; null without images
  int ncells;
};

// Global cell of a position (x-major, then y, then z within a replica).
__device__ inline int cell_of(const RepDesc& R, uint32_t ux, uint32_t uy, uint32_t uz) {
  int cx = (int)(((unsigned long long)ux * (unsigned)R.nc[0]) >> 32);
  int cy = (int)(((unsigned long long)uy * (unsigned)R.nc[1]) >> 32);
  int cz = (int)(((unsigned long long)uz * (unsigned)R.nc[2]) >> 32);
  return R.cell_off + (cx * R.nc[1] + cy) * R.nc[2] + cz;
}

// counts[key] += 1 for every lane with `active`, as one atomic per run of
// consecutive lanes with the same key (beads kept in cell order put runs of
// one cell in consecutive lanes; same-address atomics would serialise).
// Returns the counter's value before this lane's share, lanes of a run
// taking consecutive values in lane order.  Every lane of the wavefront must
// call it.
__device__ inline int run_atomic_add(int* counts, int key, bool active) {
  const int lane = threadIdx.x & 63;
  const int k = active ? key : -1 - lane;  // inactive lanes never join a run
  const int prev = __shfl_up(k, 1, 64);
  const bool head = lane == 0 || prev != k;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int start = 63 - __clzll((long long)(heads & upto));
  const unsigned long long above = heads & ~upto;
  const int end = above ? __ffsll((long long)above) - 1 : 64;
  int old = 0;
  if (head && active) old = atomicAdd(&counts[key], end - start);
  old = __shfl(old, start, 64);
  return old + (lane - start);
}

// Record bead s's cell and count it (and, if charged, among the charged).
// Every lane of the wavefront must call it (inactive lanes: active false).
__device__ inline void bin_bead(const CellView& c, const RepDesc& R, uint32_t ux, uint32_t uy, uint32_t uz,
                                uint32_t prm, int s, int id, bool active) {
  const int cid = active ? cell_of(R, ux, uy, uz) : 0;
  if (active) c.cell[s] = cid;
  if (active && c.slot_a) c.slot_a[id] = s;
  (void)run_atomic_add(c.counts, cid, active);
  (void)run_atomic_add(c.qcounts, cid, active && param_z(prm) != 0);
}

// Execution span of a launch, for the stage timers (null pointer: off):
// the first lane of every wavefront writes the GPU's constant-rate real-time
// counter at the wavefront's start (end = 0) and end (end = 1) into slot
// 2 w + end of st, w the wavefront's index in the grid.  The host takes the
// first start and the last end over the launch's wavefronts.
// The work item of this workgroup among n: the hardware hands workgroups
// to the 8 XCDs in turn (workgroup b to XCD b mod 8), each XCD with its own
// L2, so item order is remapped to give every XCD one contiguous run of
// items.  Neighbouring items (adjacent clusters, mesh tiles, batches of
// mesh lines) read mostly the same records and cache lines, which then
// come through one L2 instead of eight.  A bijection of [0, n).
__device__ inline int xcd_item(int b, int n) {
  constexpr int X = 8;
  const int per = n / X, rem = n % X, x = b % X;
  return x * per + (x < rem ? x : rem) + b / X;
}

__device__ inline void wave_stamp(unsigned long long* st, int end) {
  if (st && (threadIdx.x & 63) == 0) {
    const unsigned w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    st[2 * (size_t)w + end] = wall_clock64();
  }
}

// Packed copy of a sorted bead: x, y, z (fractional fixed point), param.
struct ChargedView {
  uint4* pk;         // charged beads in cell order
  int* idx;          // sorted bead index of each charged bead
};

// extra.hip: the slab correction and harmonic bonds, both added to F.
struct SlabLaunch {
  const RepDesc* rep;
  const Tile* tiles;        // 256-bead tiles of every replica
  int ntiles;
  const int* tile_off;      // [R+1] each replica's tiles
  const int* on;            // [R] correction switched on
  long long* mz;            // [ntiles] z_i u_iz summed per tile (exact)
  long long* F[3];
  double fscale;
  unsigned int* status;
  double* part;             // SLOT_SLAB partials [ntiles][PART_W]
};
struct BondLaunch {
  const RepDesc* rep;
  const Tile* tiles;        // 256-bond tiles (first = first bond)
  int ntiles;
  const int2* bonds;        // original bead indices, grouped by replica
  const int* slot_of;       // [N] sorted index of each original bead index
  int nbeads;               // N
  const double* k;          // [R] force constant
  const double* b;          // [R] rest length
  long long* F[3];
  double fscale;
  unsigned int* status;
  double* part;             // SLOT_BOND partials [ntiles][PART_W]
};
// Image charges: pairs (image bead, source bead) of original indices.
struct ImageLaunch {
  const RepDesc* rep;
  const int2* pairs;
  int n;
  int nbeads;
  unsigned int* status;
};
void launch_slab(hipStream_t s, const SlabLaunch& a, StateView B);
// After a binning of A: every image bead to its source's reflection across
// z = 0, with its cell and the cell counts corrected.
void launch_images(hipStream_t s, const ImageLaunch& a, StateView A, CellView c);
void launch_bonds(hipStream_t s, const BondLaunch& a, StateView B);

// ---------------------------------------------------------------------------
// Launchers (defined in the kernel translation units).
// ---------------------------------------------------------------------------

// cells.hip
void launch_ingest(hipStream_t s, const double* pos_soa, int N, long long ld, const RepDesc* rep,
                   const uint32_t* param, StateView A, long long* F, int nF);
void launch_fill_i64(hipStream_t s, long long* p, long long v, long long n);
void launch_bin(hipStream_t s, StateView A, const RepDesc* rep, CellView c, int N);
void launch_scan(hipStream_t s, CellView c);
void launch_scatter(hipStream_t s, CellView c, int N);
void launch_permute(hipStream_t s, StateView A, StateView B, uint4* bpk, CellView c, ChargedView q, int N);
void launch_commit(hipStream_t s, StateView B, StateView A, int N);

// pair.hip
// A cluster is CI consecutive beads of the sorted population (all beads, or
// the compacted charged beads) of one replica; cl[c] = (first bead,
// replica | bead count << 16).  Each cluster owns `cap` list entries.
struct PairLaunch {
  const RepDesc* rep;
  const Tile* tiles;   // force kernel: up to pair_waves_per_block() clusters of one replica
  int ntiles;
  const int2* cl;
  int ncl;
  int ci;              // beads per cluster (2, 4, 8)
  int direct;          // 1: list-free kernel (no list build, no list)
  int cap;             // list entries per cluster
  uint32_t* list;      // [ncl][cap] population indices
  int* count;          // [ncl] entries used
  const void* gcm;     // GcmPar<T>[R][MAXT][MAXT]
  const void* elec;    // ElecPar<T>[R][MAXT][MAXT]
  const void* adj;     // AdjPar<T>[R][MAXT][MAXT]
  const uint4* pk;     // packed sorted population
  const int* start;    // cell start (all beads or charged beads)
  const int* qidx;     // charged -> sorted bead index (charged kernel)
  long long* F[3];
  double* part;        // partial sums of this slot, [ntiles][PART_W]
  double* adj_part;    // adjoint partials [ntiles][MAXT * MAXT + 2 * MAXT]
  const double* vjp;   // adjoint, or null: v per sorted bead, [3][nbeads]; the
                       // adjoint sums then hold sum_i v_i . dF_i/dtheta
  int nbeads;
  double* dbead;       // adjoint, or null: per sorted bead, the derivative of E
                       // with respect to the bead's own radius (sigma in the
                       // excluded-volume kernel, a in the charged one)
  unsigned long long* pair_count;  // optional counter
  unsigned int* status;
  double fscale;       // 2^FSHIFT
  unsigned long long* stamps;  // wave_stamp slots of this launch, or null
  const int* hncl;     // half-shell kernels: column clusters in use per replica
};
void launch_nl_build(hipStream_t s, const PairLaunch& a);

// Column clusters of the half-shell pair kernels: runs of at most ci
// consecutive sorted beads (all beads, or the compacted charged beads) that
// never leave their cell column.  Each replica owns the cluster slots
// [base, base + capacity) with capacity ceil(n / ci) + its column count (an
// upper bound); k_col_clusters fills the first ncl[r] of them after every
// sort, from the cell starts, in column order.
struct ColLaunch {
  const int* start;      // cell starts of the population (all or charged beads)
  const int2* coltab;    // [ncols + 1] (first global cell, replica) per column;
                         // the last entry is (total cells, replica count)
  int ncols;
  int ci;                // beads per cluster (a power of two)
  const int* rep_base;   // [R] first cluster slot of each replica
  int2* cl;              // cluster slots: (first bead, bead count)
  int* ncl;              // [R] clusters in use
  int* colbase;          // [ncols] first cluster slot of each column (scratch)
  int nrep;
  unsigned long long* stamps;
};
void launch_col_clusters(hipStream_t s, const ColLaunch& a);
// Largest ncols + 2 nrep the column pass stages (the plan falls back to the
// cluster kernels beyond it).
int col_clusters_max_entries();

// Column-cluster pairs (`half_pairs` tuning field): every unordered pair
// within rc evaluated once by the cluster that owns it, both beads
// receiving its force (half), or from both ends with the cluster beads'
// forces only (!half).  Tiles hold up to pair_waves_per_block() cluster
// slots of one replica (Tile.first: first slot; Tile.bead0: the replica's
// first slot); a.cl / a.hncl are the column clusters and their per-replica
// counts.  The charged variant takes the charged beads' compacted records
// (a.pk), cell list (a.start) and sorted indices (a.qidx).
void launch_pair_gcm_col(hipStream_t s, const PairLaunch& a, bool fp64, bool ev, bool half);
void launch_pair_elec_col(hipStream_t s, const PairLaunch& a, bool fp64, bool ev, bool half);
void launch_pair_gcm(hipStream_t s, const PairLaunch& a, bool fp64, bool ev, bool adjoint);
void launch_pair_elec(hipStream_t s, const PairLaunch& a, bool fp64, bool ev, bool adjoint);
int pair_waves_per_block();

// pme.hip
struct PmeLaunch {
  const RepDesc* rep;
  int nrep;
  int nq;             // charged beads, all replicas
  int order;          // B-spline order (shared by all replicas)
  const uint4* qpk;   // packed charged beads (cell order)
  const int* qidx;    // charged -> sorted bead index
  const int* qstart;  // charged cell list
  const MeshTile* tiles;  // fused spread + z / z + gather passes
  int ntiles;
  int tx, ty;         // tile shape (z lines per axis)
  void* Qc;           // complex<T> half-complex mesh, per replica at cgrid_off:
                      //   plane_major: (m, x, y) at (m K0 + x) K1 + y
                      //   otherwise:   (x, y, m) at (x K1 + y) K2h + m
  int plane_major;    // the layout of the fused y/x plane pass
  const void* tw;     // complex<T> twiddles
  const int* radix;
  const void* bsp;    // T: exp(-pi^2 (m/L)^2/beta^2) / |b(m)|^2 per axis entry
  const void* freq;   // T: signed m / L per axis entry
  const LineItem* items[3];  // fused y/x planes (rep, kz), Y lines, X lines
  int plane_elems;    // complex entries of one LDS plane buffer (fused y/x pass)
  int plane_k;        // K0 = K1 shared by every replica's mesh, else 0
  int nitems[3];
  int lb[3];          // lines per item for each pass
  int maxK[3];        // longest z, y, x line
  long long* F[3];
  double* part;       // recip slot partials [nitems X][PART_W]
  unsigned int* status;
  double fscale;      // force fixed-point scale
  double qscale;      // mesh fixed-point scale
  unsigned long long* stamps;  // wave_stamp slots of this launch, or null
};
void launch_spread_z(hipStream_t s, const PmeLaunch& a, bool fp64);
void launch_fft_y(hipStream_t s, const PmeLaunch& a, bool fp64, bool inverse);
void launch_fft_x_conv(hipStream_t s, const PmeLaunch& a, bool fp64, bool ev);
void launch_fft_yx_conv(hipStream_t s, const PmeLaunch& a, bool fp64, bool ev);
size_t pme_plane_lds_bytes(int plane_elems, int maxK0, int maxK1, int maxK2, bool fp64);
// threads of a fused y/x plane workgroup for planes of plane_elems entries
int pme_plane_threads(int plane_elems);
void launch_z_gather(hipStream_t s, const PmeLaunch& a, bool fp64);
size_t pme_tile_lds_bytes(int maxK2, int tx, int ty, int order, bool fp64);

// ewald.hip: the reciprocal term of eq. ewald summed exactly over the wave
// vectors k = 2 pi (n0/L0, n1/L1, n2/L2) != 0 with |k| <= kmax, for the
// replicas that ask for it instead of the mesh.
struct EwaldK {
  int n[3];     // integer wave vector of the half space (n0 > 0; or n0 = 0, n1 > 0;
                // or n0 = n1 = 0, n2 > 0); -k is counted through ek
  int rep;
  double ek;    // 2 (2 pi lB / V) exp(-k^2 / (4 beta^2)) / k^2: energy per |S(k)|^2
  double c;     // 2 (1 + k^2 / (4 beta^2)) / k^2 (virial)
  double k[3];  // the wave vector (1 / length)
};
// Work tile of the exact sum: wave vectors k0 .. k0 + KCH - 1 of a replica
// against its charged beads q0 .. q0 + QCH - 1 (replica-relative).
struct EwaldItem {
  int rep, k0, q0, pad;
};
constexpr int EW_SK_K = 64, EW_SK_Q = 256;  // structure-factor tiles (k x charged)
constexpr int EW_F_K = 256, EW_F_Q = 64;    // force tiles
constexpr int EW_NMAX = 64;                 // largest |n_a| of a wave vector
struct EwaldLaunch {
  const RepDesc* rep;
  const EwaldK* kv;
  const EwaldItem* items_s;
  int nitems_s;
  const EwaldItem* items_f;
  int nitems_f;
  double* sp;           // partial structure factors (re, im) per replica at sp_off
  const uint4* qpk;     // packed charged beads (cell order)
  const int* qidx;      // charged -> sorted bead index
  long long* F[3];
  double* part;         // SLOT_EWALD partials [nitems_f][PART_W]
  unsigned int* status;
  double fscale;
};
void launch_ewald(hipStream_t s, const EwaldLaunch& a, bool fp64, bool ev);

// integrate.hip
struct IntLaunch {
  const RepDesc* rep;
  const Tile* tiles;
  int ntiles;
  const double* inv_mass;   // [R][MAXT]
  const double* c1;         // [R] exp(-gamma dt)
  const double* c2s;        // [R][MAXT] sqrt((1 - c1^2) kT / m)
  const double* dt;         // [R]
  const int* langevin;      // [R]
  int nbeads;
  unsigned long long seed;
  unsigned long long* step; // device counter: step being taken (advanced by
                            // the scan of each step's sort, before the
                            // integrator of the next first half reads it,
                            // so captured steps can be replayed)
  double fscale_inv;
  double* part;             // kinetic partials [ntiles][PART_W]
  unsigned long long* stamps;  // wave_stamp slots of this launch, or null
};
// First half of a step on A (kick, drift, noise; clears F); with bin != NULL
// also the binning of the new positions (as launch_bin).
void launch_int_first(hipStream_t s, const IntLaunch& a, StateView A, long long* const F[3],
                      const CellView* bin = nullptr);
// Second half kick of a step on B written back to A, then the first half of
// the next step and its binning: the same arithmetic as launch_int_last,
// launch_int_first and launch_bin in turn, in one pass.
void launch_int_between(hipStream_t s, const IntLaunch& a, StateView B, StateView A, long long* const F[3],
                        const CellView& bin);
void launch_int_last(hipStream_t s, const IntLaunch& a, StateView B, StateView A,
                     long long* const F[3], bool kin);
void launch_forces_out(hipStream_t s, StateView B, long long* const F[3], double* out, long long ld,
                       int N, double fscale_inv);
// v (original order, [3][N]) to sorted order for the force vector-Jacobian
// product.
void launch_gather_vjp(hipStream_t s, StateView B, const double* v, double* vs, int N);
// Per-bead radius derivatives to original bead order: dE/dsigma_i from dg,
// dE/da_i from dq plus the self-energy term self_a[rep][type] z_i^2.
void launch_bead_adj_out(hipStream_t s, StateView B, const double* dg, const double* dq, const double* self_a,
                         double* out_sigma, double* out_a, int N);
void launch_state_out(hipStream_t s, StateView A, const RepDesc* rep, double* pos, double* vel,
                      long long ld, int N);
struct FinalLaunch {
  const RepDesc* rep;
  int nrep;
  const double* part[N_SLOTS];
  const int* slot_off[N_SLOTS];  // [R+1] partial ranges per replica
  const double* consts;          // [R][2]: E_corr, E_self
  double* energy;                // [R][N_TERMS] or null
  double* virial;                // [R][6] or null
  int have_kin;
  const double* adj_part[2];     // gcm, real adjoint partials
  const int* adj_off[2];
  const double* Avals;           // [R][MAXT*MAXT]
  const double* dself;           // [R][MAXT] d U_self / d a_t
  double* dE_dA;
  double* dE_dsigma;
  double* dE_da;
  double adj_scale;              // 1, or 2 for the force vector-Jacobian
                                 // product (its pair sums are not halved)
  int vjp;                       // the adjoint holds sum_i v_i . dF_i/dtheta
};
void launch_finalize(hipStream_t s, const FinalLaunch& a);

}  // namespace gcme
