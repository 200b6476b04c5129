// Host side of the GCMe engine: C ABI, validation, device buffers, mesh and
// cell plans, per-type-pair tables, hipGraph-captured steps and the
// autotuner.  All arithmetic of the method runs in the kernels of cells.hip,
// pair.hip, pme.hip and integrate.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/gcme.h"
#include "gcme_internal.h"

using namespace gcme;

static_assert(GCME_N_TERMS == N_TERMS, "energy row width");

// The no-alloc entry point's device memory: one static array per GPU,
// created with the library's code object on that GPU and held until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current (scratch_address below).
static __device__ __align__(256) unsigned char scratch[GCME_NOALLOC_SCRATCH_BYTES];

namespace {

// A bump allocator over a device region the library already holds (the
// static scratch of the no-alloc entry point).  While one is set for the
// calling thread, DevBuf::alloc carves from it and never calls hipMalloc;
// such buffers are never freed.
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  size_t need = 0;  // bytes the last refused request would have needed
};
thread_local Arena* t_arena = nullptr;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool in_arena = false;
  ~DevBuf() {
    if (p && !in_arena) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    if (n == 0) n = 64;
    if (t_arena) {
      const size_t off = (t_arena->used + 255) & ~(size_t)255;
      if (off + n > t_arena->size) {
        t_arena->need = std::max(t_arena->need, off + n);
        return hipErrorOutOfMemory;
      }
      if (p && !in_arena) (void)hipFree(p);
      p = t_arena->base + off;
      bytes = n;
      in_arena = true;
      t_arena->used = off + n;
      return hipSuccess;
    }
    if (p && !in_arena) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    in_arena = false;
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

struct HostRep {
  bool set = false;
  double box[3] = {0, 0, 0};
  double rc = 0, beta = 0, lB = 0, kT = 0, dt = 0, gamma = 0;
  int K[3] = {0, 0, 0};
  int order = 0;
  double kmax = 0;  // > 0: exact reciprocal sum over |k| <= kmax, no mesh
  int nt = 0;
  double A[MAXT * MAXT] = {};
  double sigma[MAXT] = {};
  double a[MAXT] = {};
  double mass[MAXT] = {1, 1, 1, 1};
  uint32_t flags = 0;
  double bond_k = 0, bond_b = 0;  // harmonic bonds k/2 (r - b)^2
};

bool smooth(int k) {
  if (k < 1) return false;
  while (k % 2 == 0) k /= 2;
  while (k % 3 == 0) k /= 3;
  return k == 1;
}

std::vector<int> radices(int K) {
  std::vector<int> r;
  while (K % 4 == 0) {
    r.push_back(4);
    K /= 4;
  }
  while (K % 2 == 0) {
    r.push_back(2);
    K /= 2;
  }
  while (K % 3 == 0) {
    r.push_back(3);
    K /= 3;
  }
  return r;
}

// Cardinal B-spline M_n(x) on [0, n] (host, for the mesh moduli).
double bspl(int n, double x) {
  if (x < 0.0 || x >= (double)n) return 0.0;
  if (n == 1) return 1.0;
  return (x * bspl(n - 1, x) + ((double)n - x) * bspl(n - 1, x - 1.0)) / (double)(n - 1);
}

}  // namespace

struct gcme_ctx {
  std::string err;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t cap_stream = nullptr;
  hipStream_t aux[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
  int R = 0;
  std::vector<int> nb, boff;
  int N = 0;
  bool fp64 = false;
  uint64_t seed = 0;
  std::vector<HostRep> hp;
  // state
  bool have_state = false;
  bool forces_valid = false;
  uint64_t step = 0;
  std::vector<int> h_type, h_z;
  std::vector<int> nq, qoff;
  int NQ = 0;
  // tuning
  gcme_tuning tune{3, 8, 4, 50, 3, 0, 0, 0, 0, 0, 0};  // list-free pairs, three stream branches, 4 x 4 mesh tiles
  bool plan_dirty = true;
  // device buffers
  DevBuf a_pos[3], a_vel[3], a_param, a_id;
  DevBuf b_pos[3], b_vel[3], b_param, b_id;
  DevBuf cell, tmp, counts, qcounts, fill, start, qstart, bsum;
  DevBuf b_pk, q_pk, q_idx;
  DevBuf F;
  DevBuf Qc, d_mtiles, d_gtiles;
  DevBuf d_rep, d_gcm, d_elec, d_adj;
  DevBuf d_tw, d_rad, d_bsp, d_freq;
  DevBuf d_items[3];
  DevBuf d_cl_g, d_cl_q, d_tiles_g, d_tiles_q, d_tiles_256;
  // half-shell excluded-volume pairs: cell columns (first cell, replica),
  // each replica's first cluster slot, the column clusters, their count per
  // replica, the pair tiles and their partial-sum rows
  DevBuf d_coltab, d_colbase, d_colbase_q, d_hbase, d_hcl, d_hncl, d_htiles, part_h, d_off_h;
  int ncols = 0, ntiles_h = 0, hci = 8;
  // the same for the charged beads' real-space pairs
  DevBuf d_hqbase, d_hqcl, d_hqncl, d_hqtiles, part_hq, d_off_hq;
  int ntiles_hq = 0, hqci = 4;
  int ncols_tmp = 0;  // build_plan's running column count
  DevBuf list_g, list_q, cnt_g, cnt_q;
  DevBuf part[N_SLOTS], adjp[2];
  DevBuf d_off[N_SLOTS], d_adj_off[2];
  DevBuf d_consts, d_Avals, d_dself;
  // per-bead radius derivatives (sorted order) and the self term's factor
  DevBuf dbead_g, dbead_q, d_self_a;
  bool per_bead = false;
  DevBuf vjp_sorted;  // force vector-Jacobian product: v in sorted order
  bool vjp = false;
  DevBuf d_imass, d_c1, d_c2s, d_dt, d_lang;
  DevBuf d_status, d_step, d_pairs;
  DevBuf d_ewk, d_ew_items_s, d_ew_items_f, ew_sp;  // exact reciprocal sums
  int nitems_ew_s = 0, nitems_ew_f = 0;
  // slab correction and bonds
  DevBuf d_slab_on, slab_mz, d_bond_kb, d_bonds, d_btiles, slot_of;
  bool any_slab = false;
  int ntiles_b = 0;
  std::vector<std::vector<int2>> bonds;  // per replica, original bead indices
  long long nbonds = 0;
  // image charges: (image, source) pairs; checked against types and charges
  std::vector<int2> images;
  DevBuf d_images, slot_a;
  int nimages = 0;
  bool images_checked = true;
  // plan sizes
  int ncells = 0;
  long long grid_total = 0, cgrid_total = 0;
  int ncl_g = 0, ncl_q = 0, ntiles_g = 0, ntiles_q = 0, ntiles_256 = 0;
  int cap_g = 64, cap_q = 64;
  int nmtiles = 0, mtx = 4, mty = 4;     // spread tiles
  int ngtiles = 0, gtx = 4, gty = 4;     // gather tiles
  bool yx_fused = false;  // y and x passes in one LDS plane kernel
  int plane_elems = 0;
  int lds_max = 65536;  // dynamic LDS a workgroup may use
  int nitems[3] = {0, 0, 0};
  int lb[3] = {0, 0, 0};
  int maxK[3] = {0, 0, 0};
  int order = 5;
  std::vector<RepDesc> rep;
  // graphs
  //   g_mid: a step after the first half (sort, forces, then the second half
  //          fused with the next step's first half and binning)
  //   g_last / g_obs: the same, ending with the plain second half (g_obs also
  //          accumulates the energy, virial and kinetic partials)
  //   g_midn: MID_BATCH consecutive g_mid steps in one graph (one launch)
  hipGraphExec_t g_mid = nullptr, g_midn = nullptr, g_last = nullptr, g_obs = nullptr;
  // stage timers (gcme_time_stages): while `timing` is set, the enqueue
  // functions hand every one-kernel stage's launch the stamp slots
  // stamps + 2 stamp_off[stage] (one pair per wavefront, stamp_nw[stage])
  bool timing = false;
  DevBuf stamps;
  size_t stamp_off[GCME_N_STAGES] = {};
  int stamp_nw[GCME_N_STAGES] = {};

  ~gcme_ctx() {
    drop_graphs();
    for (auto& e : ev_join)
      if (e) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (auto& a : aux)
      if (a) (void)hipStreamDestroy(a);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
  void drop_graphs() {
    if (g_mid) (void)hipGraphExecDestroy(g_mid);
    if (g_midn) (void)hipGraphExecDestroy(g_midn);
    if (g_last) (void)hipGraphExecDestroy(g_last);
    if (g_obs) (void)hipGraphExecDestroy(g_obs);
    g_mid = g_midn = g_last = g_obs = nullptr;
  }
  double fscale() const { return std::ldexp(1.0, fp64 ? FSHIFT_FP64 : FSHIFT_MIXED); }
  double qscale() const { return std::ldexp(1.0, fp64 ? FSHIFT_FP64 : FSHIFT_MIXED); }
};

namespace {

constexpr int MID_BATCH = 8;  // steps per graph launch in long runs

thread_local std::string g_create_err;

gcme_status fail(gcme_handle h, gcme_status s, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_create_err = msg;
  return s;
}

#define HIPCHK(h, expr)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail(h, e_ == hipErrorOutOfMemory ? GCME_ENOMEM : GCME_EDEVICE,                     \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                            \
  } while (0)

StateView view(DevBuf* pos, DevBuf* vel, DevBuf& param, DevBuf& id) {
  StateView v;
  for (int k = 0; k < 3; ++k) {
    v.pos[k] = pos[k].as<uint32_t>();
    v.vel[k] = vel[k].as<double>();
  }
  v.param = param.as<uint32_t>();
  v.id = id.as<int>();
  return v;
}

StateView viewA(gcme_handle h) { return view(h->a_pos, h->a_vel, h->a_param, h->a_id); }
StateView viewB(gcme_handle h) { return view(h->b_pos, h->b_vel, h->b_param, h->b_id); }

CellView cview(gcme_handle h) {
  CellView c;
  c.cell = h->cell.as<int>();
  c.tmp = h->tmp.as<int>();
  c.counts = h->counts.as<int>();
  c.qcounts = h->qcounts.as<int>();
  c.fill = h->fill.as<int>();
  c.start = h->start.as<int>();
  c.qstart = h->qstart.as<int>();
  c.bsum = h->bsum.as<int>();
  c.step = nullptr;
  c.slot_of = h->nbonds > 0 ? h->slot_of.as<int>() : nullptr;
  c.slot_a = h->nimages > 0 ? h->slot_a.as<int>() : nullptr;
  c.ncells = h->ncells;
  return c;
}

ChargedView qview(gcme_handle h) {
  ChargedView q;
  q.pk = h->q_pk.as<uint4>();
  q.idx = h->q_idx.as<int>();
  return q;
}

long long* Fk(gcme_handle h, int k) { return h->F.as<long long>() + (size_t)k * h->N; }

template <typename T>
hipError_t upload_buf(std::vector<T>& v, DevBuf& b, hipStream_t s) {
  hipError_t e = b.alloc(v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}
// a table to the device; a failed allocation or copy ends the calling
// function with its status
#define upload(v, b, s) HIPCHK(h, upload_buf(v, b, s))

std::vector<Tile> make_tiles(const std::vector<int>& off, const std::vector<int>& cnt, int per,
                             std::vector<int>& tile_off) {
  std::vector<Tile> t;
  tile_off.assign(off.size() + 1, 0);
  for (size_t r = 0; r < off.size(); ++r) {
    tile_off[r] = (int)t.size();
    for (int f = 0; f < cnt[r]; f += per) t.push_back(Tile{(int)r, off[r] + f, std::min(per, cnt[r] - f), 0});
  }
  tile_off[off.size()] = (int)t.size();
  return t;
}

// Series coefficients of phi(r) = [erf(alpha r) - erf(beta r)]/r and
// g(r) = -(1/r) dphi/dr in powers of r^2, from the Maclaurin series of erf.
// alpha^k - beta^k is formed as (alpha - beta) sum alpha^i beta^(k-1-i) so
// that nearly equal alpha and beta lose no digits.
void erf_series(double al, double be, double* cphi, double* cg) {
  const double tsp = 2.0 / std::sqrt(M_PI);
  auto D = [&](int k) {
    double s = 0;
    for (int i = 0; i < k; ++i) s += std::pow(al, i) * std::pow(be, k - 1 - i);
    return (al - be) * s;
  };
  double fact = 1.0;  // n!
  for (int n = 0; n < NSER; ++n) {
    if (n > 0) fact *= n;
    double sgn = (n % 2 == 0) ? 1.0 : -1.0;
    cphi[n] = tsp * sgn * D(2 * n + 1) / (fact * (2 * n + 1));
    // g: sum_m (-1)^m D(2m+3) 2(m+1) r^{2m} / ((m+1)! (2m+3))
    cg[n] = tsp * sgn * D(2 * n + 3) * 2.0 * (n + 1) / (fact * (n + 1) * (2 * n + 3));
  }
}

template <typename T>
void build_tables(gcme_handle h, std::vector<GcmPar<T>>& g, std::vector<ElecPar<T>>& e, std::vector<AdjPar<T>>& ad) {
  const int R = h->R;
  g.assign((size_t)R * MAXT * MAXT, GcmPar<T>{});
  e.assign((size_t)R * MAXT * MAXT, ElecPar<T>{});
  ad.assign((size_t)R * MAXT * MAXT, AdjPar<T>{});
  const double log2e = 1.4426950408889634;
  for (int r = 0; r < R; ++r) {
    const HostRep& p = h->hp[r];
    for (int t = 0; t < p.nt; ++t)
      for (int u = 0; u < p.nt; ++u) {
        size_t q = ((size_t)r * MAXT + t) * MAXT + u;
        double s2 = p.sigma[t] * p.sigma[t] + p.sigma[u] * p.sigma[u];
        double b = 3.0 / (2.0 * s2);
        const double C = p.A[t * p.nt + u] * std::pow(3.0 / (2.0 * M_PI * s2), 1.5);
        g[q].C = (T)C;
        g[q].bl = (T)(b * log2e);
        g[q].twob = (T)(2.0 * b);
        g[q].fC = (T)(2.0 * b * C);
        double aij = std::sqrt(p.a[t] * p.a[t] + p.a[u] * p.a[u]);
        double al = std::sqrt(M_PI / 2.0) / aij;
        e[q].alpha = (T)al;
        e[q].alpha2 = (T)(al * al);
        if constexpr (std::is_same<T, float>::value) {
          // the same float operations as the kernel's for beta, so that
          // alpha == beta (as floats) gives equal Gaussians, bit for bit
          const float af = (float)al;
          e[q].cexp = -(af * af) * 1.44269504088896341f;
          e[q].tsa = 1.12837916709551257f * af;
        } else {
          e[q].cexp = (T)(-al * al * log2e);
          e[q].tsa = (T)(2.0 / std::sqrt(M_PI) * al);
        }
        // the series is used where both alpha r and beta r stay below 1/2,
        // which bounds its truncation after 8 (FP32) or 14 (FP64) terms
        double rs = 0.5 / std::max(al, p.beta);
        e[q].rs2 = (T)(rs * rs);
        double cp[NSER], cgv[NSER];
        erf_series(al, p.beta, cp, cgv);
        for (int n = 0; n < NSER; ++n) {
          e[q].cphi[n] = (T)cp[n];
          e[q].cg[n] = (T)cgv[n];
        }
        double s = std::sqrt(s2);
        ad[q].inv_s2 = (T)(1.0 / s2);
        ad[q].s_inv = (T)(1.0 / s);
        ad[q].dsig_i = (T)(p.sigma[t] / s);
        ad[q].dsig_j = (T)(p.sigma[u] / s);
        ad[q].daij_i = (T)(p.a[t] / aij);
        ad[q].daij_j = (T)(p.a[u] / aij);
        ad[q].ea = (T)(2.0 / std::sqrt(M_PI) * al / aij);
      }
  }
}

template <typename T>
void build_mesh_tables(gcme_handle h, std::vector<T>& tw, std::vector<T>& bsp, std::vector<T>& frq,
                       std::vector<int>& rad) {
  std::map<int, std::pair<int, int>> kmap;  // K -> (tw offset in complex entries, rad offset)
  tw.clear();
  bsp.clear();
  frq.clear();
  rad.clear();
  for (int r = 0; r < h->R; ++r) {
    RepDesc& d = h->rep[r];
    const HostRep& p = h->hp[r];
    if (p.kmax > 0) continue;  // exact reciprocal sum: no mesh
    for (int ax = 0; ax < 3; ++ax) {
      int K = p.K[ax];
      auto it = kmap.find(K);
      if (it == kmap.end()) {
        int to = (int)(tw.size() / 2);
        for (int e = 0; e < K; ++e) {
          double ang = -2.0 * M_PI * (double)e / (double)K;
          tw.push_back((T)std::cos(ang));
          tw.push_back((T)std::sin(ang));
        }
        int ro = (int)rad.size();
        for (int x : radices(K)) rad.push_back(x);
        it = kmap.emplace(K, std::make_pair(to, ro)).first;
      }
      d.tw_off[ax] = it->second.first;
      d.rad_off[ax] = it->second.second;
      d.nrad[ax] = (int)radices(K).size();
      // 1/|b(m)|^2 with the odd-order Nyquist zero replaced by the mean of
      // its neighbours, and the signed frequency m/L
      std::vector<double> mod(K);
      for (int m = 0; m < K; ++m) {
        double re = 0, im = 0;
        for (int k = 0; k <= p.order - 2; ++k) {
          double w = bspl(p.order, (double)(k + 1));
          double ang = 2.0 * M_PI * (double)m * (double)k / (double)K;
          re += w * std::cos(ang);
          im += w * std::sin(ang);
        }
        mod[m] = re * re + im * im;
      }
      for (int m = 0; m < K; ++m)
        if (mod[m] < 1e-7) mod[m] = 0.5 * (mod[(m - 1 + K) % K] + mod[(m + 1) % K]);
      // Green's function factor of the axis: the Gaussian of eq. ewald's
      // reciprocal sum factorises over the axes
      d.bsp_off[ax] = (int)bsp.size();
      for (int m = 0; m < K; ++m) {
        int ms = m <= K / 2 ? m : m - K;
        const double f = (double)ms / p.box[ax];
        bsp.push_back((T)(std::exp(-M_PI * M_PI * f * f / (p.beta * p.beta)) / mod[m]));
        frq.push_back((T)f);
      }
    }
  }
}

// Clusters of `ci` consecutive beads of each replica's sorted population
// (all beads, or the compacted charged beads), tiled in groups of
// pair_waves_per_block() clusters of one replica (one pair-kernel workgroup
// each, one partial-sum row per workgroup).  The list capacity per cluster is
// bounded from the population density: a cluster fills its cell column over
// roughly ci / (rho h^2) (plus up to two cells, since beads within a cell are
// not ordered in z), and its list is at most the population inside the
// cutoff shell of that box; the slack covers density fluctuations, and a
// list that still overflows is reported as GCME_EOVERFLOW.
void plan_clusters(gcme_handle h, bool charged, int ci, std::vector<int2>& cl, std::vector<Tile>& tiles,
                   std::vector<int>& toff, int& cap) {
  const int wpb = pair_waves_per_block();
  cl.clear();
  tiles.clear();
  toff.assign(h->R + 1, 0);
  double cmax = 64.0;
  for (int r = 0; r < h->R; ++r) {
    const RepDesc& d = h->rep[r];
    // an all-reciprocal replica has no real-space electrostatic pairs
    const bool skip = charged && (h->hp[r].flags & GCME_FLAG_ALL_RECIPROCAL);
    const int n = skip ? 0 : charged ? h->nq[r] : h->nb[r];
    const int off = charged ? h->qoff[r] : h->boff[r];
    toff[r] = (int)tiles.size();
    if (n == 0) continue;
    const int c0 = (int)cl.size();
    for (int f = 0; f < n; f += ci) cl.push_back(make_int2(off + f, r | (std::min(ci, n - f) << 16)));
    const int c1 = (int)cl.size();
    for (int c = c0; c < c1; c += wpb) tiles.push_back(Tile{r, c, std::min(wpb, c1 - c), off + (c - c0) * ci});
    const double rho = (double)n / d.V;
    const double hx = d.L[0] / d.nc[0], hy = d.L[1] / d.nc[1], hz = d.L[2] / d.nc[2];
    const double beads = ci + 4.0 * std::sqrt((double)ci) + 4.0;
    const double ez = std::min(d.L[2], 2.0 * hz + beads / (rho * hx * hy));
    const double ex = std::min(d.L[0], 2.0 * hx), ey = std::min(d.L[1], 2.0 * hy);
    const double rc = d.rc;
    double vol = ex * ey * ez + 2.0 * rc * (ex * ey + ey * ez + ez * ex) + M_PI * rc * rc * (ex + ey + ez) +
                 4.0 / 3.0 * M_PI * rc * rc * rc;
    vol = std::min(vol, d.V);
    const double mean = rho * vol;
    double c = mean * (1.0 + h->tune.list_slack_pct / 100.0) + 4.0 * std::sqrt(mean) + 64.0;
    c = std::min(c, (double)n + 64.0);
    cmax = std::max(cmax, c);
  }
  toff[h->R] = (int)tiles.size();
  cap = ((int)std::ceil(cmax) + 63) & ~63;
}

// The column-cluster mode of the excluded-volume (charged) pairs:
// 0 = cluster kernels, 1 = half shell, 2 = both ends (tuning half_pairs).
int col_mode(gcme_handle h, bool charged) { return (h->tune.half_pairs >> (charged ? 2 : 0)) & 3; }

gcme_status build_plan(gcme_handle h) {
  hipStream_t s = h->stream;
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, hipStreamSynchronize(s));
  h->drop_graphs();
  const int R = h->R;
  h->rep.assign(R, RepDesc{});
  int cell_off = 0;
  h->ncols_tmp = 0;
  long long goff = 0, cgoff = 0;
  h->order = h->hp[0].order;
  for (int ax = 0; ax < 3; ++ax) h->maxK[ax] = 0;
  for (int r = 0; r < R; ++r) {
    const HostRep& p = h->hp[r];
    RepDesc& d = h->rep[r];
    for (int k = 0; k < 3; ++k) {
      d.L[k] = p.box[k];
      d.scaled[k] = p.box[k] / 4294967296.0;
      d.scalef[k] = (float)d.scaled[k];
      int nc = (int)std::floor(p.box[k] * h->tune.cells_per_cutoff / p.rc);
      nc = std::max(1, std::min(nc, 1024));
      d.nc[k] = nc;
      double hcell = p.box[k] / nc;
      d.hf[k] = (float)hcell;
      int reach = (int)std::ceil(p.rc / hcell - 1e-9);
      d.reach[k] = (2 * reach + 1 > nc) ? -1 : reach;
      d.nreach[k] = std::max(1, reach);
      d.K[k] = p.K[k];
    }
    d.V = p.box[0] * p.box[1] * p.box[2];
    d.rc = p.rc;
    d.rc2 = p.rc * p.rc;
    d.rc2f = (float)d.rc2;
    d.beta = p.beta;
    d.betaf = (float)p.beta;
    d.lB = p.lB;
    d.lBf = (float)p.lB;
    d.cell_off = cell_off;
    cell_off += d.nc[0] * d.nc[1] * d.nc[2];
    d.col_off = h->ncols_tmp;
    h->ncols_tmp += d.nc[0] * d.nc[1];
    d.bead_off = h->boff[r];
    d.n = h->nb[r];
    d.q_off = h->qoff[r];
    d.nq = h->nq[r];
    d.K2h = p.K[2] > 0 ? p.K[2] / 2 + 1 : 0;  // no mesh: exact reciprocal sum
    d.K2s = (d.K2h + 7) & ~7;
    d.grid_off = goff;
    d.cgrid_off = cgoff;
    goff += (long long)p.K[0] * p.K[1] * p.K[2];
    cgoff += (long long)p.K[0] * p.K[1] * d.K2s;
    d.order = p.order;
    d.nt = p.nt;
    h->maxK[0] = std::max(h->maxK[0], p.K[2]);  // z pass line length
    h->maxK[1] = std::max(h->maxK[1], p.K[1]);
    h->maxK[2] = std::max(h->maxK[2], p.K[0]);
  }
  h->ncells = cell_off;
  h->grid_total = goff;
  h->cgrid_total = cgoff;

  const size_t cs = h->fp64 ? 16 : 8;
  // lines per mesh work item: two LDS buffers of LB+1 padded lines stay
  // below 64 KiB together with the kernels' static reduction buffer
  const int cap = h->fp64 ? 2048 : 4096;
  // z lines are contiguous: about 1024 points per work item; strided y/x
  // lines are batched along z (at least 8 adjacent lines for coalescing)
  for (int ps = 0; ps < 3; ++ps) {
    const int mk = std::max(1, h->maxK[ps]);  // 0 when no replica has a mesh
    int want = ps == 0 ? std::max(1, 1024 / mk) : std::max(8, 1024 / mk);
    int fit = cap / mk - 2;
    h->lb[ps] = std::max(1, std::min(64, std::min(want, fit)));
  }

  // mesh tables
  std::vector<int> rad;
  if (h->fp64) {
    std::vector<double> tw, bsp, frq;
    build_mesh_tables<double>(h, tw, bsp, frq, rad);
    upload(tw, h->d_tw, s);
    upload(bsp, h->d_bsp, s);
    upload(frq, h->d_freq, s);
    std::vector<GcmPar<double>> g;
    std::vector<ElecPar<double>> e;
    std::vector<AdjPar<double>> ad;
    build_tables<double>(h, g, e, ad);
    upload(g, h->d_gcm, s);
    upload(e, h->d_elec, s);
    upload(ad, h->d_adj, s);
    HIPCHK(h, hipStreamSynchronize(s));
  } else {
    std::vector<float> tw, bsp, frq;
    build_mesh_tables<float>(h, tw, bsp, frq, rad);
    upload(tw, h->d_tw, s);
    upload(bsp, h->d_bsp, s);
    upload(frq, h->d_freq, s);
    std::vector<GcmPar<float>> g;
    std::vector<ElecPar<float>> e;
    std::vector<AdjPar<float>> ad;
    build_tables<float>(h, g, e, ad);
    upload(g, h->d_gcm, s);
    upload(e, h->d_elec, s);
    upload(ad, h->d_adj, s);
    HIPCHK(h, hipStreamSynchronize(s));
  }
  upload(rad, h->d_rad, s);

  // mesh line work items
  std::vector<LineItem> items[3];
  std::vector<int> item_off(R + 1, 0);
  for (int r = 0; r < R; ++r) {
    const RepDesc& d = h->rep[r];
    item_off[r] = (int)items[2].size();
    if (d.K2h == 0) continue;  // no mesh (exact reciprocal sum)
    // balanced batches of the K2/2+1 strided lines
    int c1 = (d.K2h + h->lb[1] - 1) / h->lb[1], b1 = (d.K2h + c1 - 1) / c1;
    int c2 = (d.K2h + h->lb[2] - 1) / h->lb[2], b2 = (d.K2h + c2 - 1) / c2;
    // batches of whole 8-line segments where the batch size allows: each
    // batch then starts on a 64-byte boundary of its rows
    if (h->lb[1] >= 8) b1 = h->lb[1] / 8 * 8;
    if (h->lb[2] >= 8) b2 = h->lb[2] / 8 * 8;
    for (int x = 0; x < d.K[0]; ++x)
      for (int kz = 0; kz < d.K2h; kz += b1)
        items[1].push_back(LineItem{r, x * d.K2h + kz, std::min(b1, d.K2h - kz), 0});
    for (int y = 0; y < d.K[1]; ++y)
      for (int kz = 0; kz < d.K2h; kz += b2)
        items[2].push_back(LineItem{r, y * d.K2h + kz, std::min(b2, d.K2h - kz), 0});
  }
  item_off[R] = (int)items[2].size();
  // one kz plane per work item when a K0 x K1 plane fits twice in LDS
  h->plane_elems = 0;
  for (int r = 0; r < R; ++r) h->plane_elems = std::max(h->plane_elems, (h->rep[r].K[0] + 1) * (h->rep[r].K[1] + 1));
  h->yx_fused = pme_plane_lds_bytes(h->plane_elems, h->maxK[2], h->maxK[1], h->maxK[0], h->fp64) <= (size_t)h->lds_max;
  if (h->yx_fused) {
    for (int r = 0; r < R; ++r) {
      item_off[r] = (int)items[0].size();
      for (int kz = 0; kz < h->rep[r].K2h; ++kz) items[0].push_back(LineItem{r, kz, 1, 0});
    }
    item_off[R] = (int)items[0].size();
  }
  // mesh tiles of the fused spread and gather passes, each with its own
  // shape: the tuning's z lines per tile (4 x 4 by default; the gather's
  // default is the spread's), halved along the longer side while the two
  // LDS line buffers would not fit
  auto tiles_of = [&](int tx, int ty, int& ox, int& oy, std::vector<MeshTile>& t) -> bool {
    ox = tx;
    oy = ty;
    while (ox * oy > 1 && pme_tile_lds_bytes(h->maxK[0], ox, oy, h->order, h->fp64) > (size_t)h->lds_max) {
      if (ox >= oy)
        ox /= 2;
      else
        oy /= 2;
    }
    if (pme_tile_lds_bytes(h->maxK[0], ox, oy, h->order, h->fp64) > (size_t)h->lds_max) return false;
    t.clear();
    for (int r = 0; r < R; ++r) {
      const RepDesc& d = h->rep[r];
      for (int x = 0; x < d.K[0]; x += ox)
        for (int y = 0; y < d.K[1]; y += oy)
          t.push_back(MeshTile{r, x, y, std::min(ox, d.K[0] - x) | (std::min(oy, d.K[1] - y) << 16)});
    }
    return true;
  };
  std::vector<MeshTile> mtiles, gtiles;
  const int stx = h->tune.mesh_tile_x > 0 ? h->tune.mesh_tile_x : 4;
  const int sty = h->tune.mesh_tile_y > 0 ? h->tune.mesh_tile_y : 4;
  if (!tiles_of(stx, sty, h->mtx, h->mty, mtiles) ||
      !tiles_of(h->tune.gather_tile_x > 0 ? h->tune.gather_tile_x : stx,
                h->tune.gather_tile_y > 0 ? h->tune.gather_tile_y : sty, h->gtx, h->gty, gtiles))
    return fail(h, GCME_EUNSUPPORTED, "mesh z length too large for the LDS of one workgroup");
  h->nmtiles = h->NQ > 0 ? (int)mtiles.size() : 0;
  h->ngtiles = h->NQ > 0 ? (int)gtiles.size() : 0;
  upload(mtiles, h->d_mtiles, s);
  upload(gtiles, h->d_gtiles, s);
  for (int ps = 0; ps < 3; ++ps) {
    h->nitems[ps] = (int)items[ps].size();
    upload(items[ps], h->d_items[ps], s);
  }

  // exact reciprocal sums: the half-space wave vectors of each replica with
  // kmax > 0 (|k| <= kmax, the same enumeration and test as the definition
  // of the sum), its tiles, and room for the partial structure factors
  std::vector<EwaldK> ewk;
  std::vector<EwaldItem> ews, ewf;
  std::vector<int> ew_off(R + 1, 0);
  long long sp_total = 0;
  for (int r = 0; r < R; ++r) {
    RepDesc& d = h->rep[r];
    const HostRep& p = h->hp[r];
    d.ek_off = (int)ewk.size();
    d.ek_n = 0;
    d.sp_off = sp_total;
    ew_off[r] = (int)ewf.size();
    if (!(p.kmax > 0)) continue;
    int nmax[3];
    for (int k = 0; k < 3; ++k) nmax[k] = (int)std::floor(p.kmax * p.box[k] / (2.0 * M_PI));
    const double V = p.box[0] * p.box[1] * p.box[2];
    for (int n0 = 0; n0 <= nmax[0]; ++n0)
      for (int n1 = -nmax[1]; n1 <= nmax[1]; ++n1)
        for (int n2 = -nmax[2]; n2 <= nmax[2]; ++n2) {
          if (n0 == 0 && (n1 < 0 || (n1 == 0 && n2 <= 0))) continue;
          const double k0 = 2.0 * M_PI * n0 / p.box[0], k1 = 2.0 * M_PI * n1 / p.box[1],
                       k2 = 2.0 * M_PI * n2 / p.box[2];
          const double kk = k0 * k0 + k1 * k1 + k2 * k2;
          if (kk > p.kmax * p.kmax) continue;
          EwaldK e{};
          e.n[0] = n0;
          e.n[1] = n1;
          e.n[2] = n2;
          e.rep = r;
          const double x = kk / (4.0 * p.beta * p.beta);
          e.ek = 2.0 * (2.0 * M_PI * p.lB / V) * std::exp(-x) / kk;
          e.c = 2.0 * (1.0 + x) / kk;
          e.k[0] = k0;
          e.k[1] = k1;
          e.k[2] = k2;
          ewk.push_back(e);
        }
    d.ek_n = (int)ewk.size() - d.ek_off;
    const int nq = h->nq[r];
    if (nq == 0 || d.ek_n == 0) continue;
    for (int k0 = 0; k0 < d.ek_n; k0 += EW_SK_K)
      for (int q0 = 0; q0 < nq; q0 += EW_SK_Q) ews.push_back(EwaldItem{r, k0, q0, 0});
    for (int k0 = 0; k0 < d.ek_n; k0 += EW_F_K)
      for (int q0 = 0; q0 < nq; q0 += EW_F_Q) ewf.push_back(EwaldItem{r, k0, q0, 0});
    sp_total += (long long)((nq + EW_SK_Q - 1) / EW_SK_Q) * d.ek_n;
  }
  ew_off[R] = (int)ewf.size();
  h->nitems_ew_s = (int)ews.size();
  h->nitems_ew_f = (int)ewf.size();
  upload(ewk, h->d_ewk, s);
  upload(ews, h->d_ew_items_s, s);
  upload(ewf, h->d_ew_items_f, s);
  HIPCHK(h, h->ew_sp.alloc((size_t)std::max(1LL, sp_total) * 16));

  // clusters, tiles and neighbour lists
  std::vector<int> toff_g, toff_q, toff_256;
  std::vector<int2> clg, clq;
  std::vector<Tile> tg, tq;
  plan_clusters(h, false, h->tune.beads_per_cluster, clg, tg, toff_g, h->cap_g);
  plan_clusters(h, true, h->tune.charges_per_cluster, clq, tq, toff_q, h->cap_q);
  std::vector<Tile> t256 = make_tiles(h->boff, h->nb, 256, toff_256);
  h->ncl_g = (int)clg.size();
  h->ncl_q = (int)clq.size();
  h->ntiles_g = (int)tg.size();
  h->ntiles_q = (int)tq.size();
  h->ntiles_256 = (int)t256.size();
  upload(clg, h->d_cl_g, s);
  upload(clq, h->d_cl_q, s);
  upload(tg, h->d_tiles_g, s);
  upload(tq, h->d_tiles_q, s);
  upload(t256, h->d_tiles_256, s);
  // the list-free kernels read no list
  const bool dg = h->tune.direct_pairs & 1, dq = (h->tune.direct_pairs >> 1) & 1;
  HIPCHK(h, h->list_g.alloc(dg ? 64 : (size_t)std::max(1, h->ncl_g) * h->cap_g * 4));
  HIPCHK(h, h->list_q.alloc(dq ? 64 : (size_t)std::max(1, h->ncl_q) * h->cap_q * 4));
  HIPCHK(h, h->cnt_g.alloc((size_t)std::max(1, h->ncl_g) * 4));
  HIPCHK(h, h->cnt_q.alloc((size_t)std::max(1, h->ncl_q) * 4));
  upload(toff_g, h->d_off[SLOT_GCM], s);
  upload(toff_q, h->d_off[SLOT_REAL], s);
  upload(item_off, h->d_off[SLOT_RECIP], s);
  upload(toff_256, h->d_off[SLOT_KIN], s);
  upload(ew_off, h->d_off[SLOT_EWALD], s);
  upload(toff_g, h->d_adj_off[0], s);
  upload(toff_q, h->d_adj_off[1], s);
  HIPCHK(h, h->part[SLOT_GCM].alloc((size_t)std::max(1, h->ntiles_g) * PART_W * 8));
  HIPCHK(h, h->part[SLOT_REAL].alloc((size_t)std::max(1, h->ntiles_q) * PART_W * 8));
  HIPCHK(h, h->part[SLOT_RECIP].alloc((size_t)std::max(1, std::max(h->nitems[0], h->nitems[2])) * PART_W * 8));
  HIPCHK(h, h->part[SLOT_KIN].alloc((size_t)std::max(1, h->ntiles_256) * PART_W * 8));
  HIPCHK(h, h->part[SLOT_EWALD].alloc((size_t)std::max(1, h->nitems_ew_f) * PART_W * 8));
  HIPCHK(h, h->adjp[0].alloc((size_t)std::max(1, h->ntiles_g) * (MAXT * MAXT + 2 * MAXT) * 8));
  HIPCHK(h, h->adjp[1].alloc((size_t)std::max(1, h->ntiles_q) * (MAXT * MAXT + 2 * MAXT) * 8));

  // half-shell pairs: the column table, each replica's cluster slots
  // (ceil(n / ci) + its column count bounds the column clusters) and tiles
  // of pair_waves_per_block() slots
  h->ncols = h->ncols_tmp;
  h->ntiles_h = h->ntiles_hq = 0;
  // (beyond what the column pass can stage, the cluster kernels run instead)
  const bool half_fits = h->ncols + 2 * R <= col_clusters_max_entries();
  if ((col_mode(h, false) || col_mode(h, true)) && half_fits) {
    std::vector<int2> coltab;
    coltab.reserve((size_t)h->ncols + 1);
    for (int r = 0; r < R; ++r) {
      const RepDesc& d = h->rep[r];
      for (int x = 0; x < d.nc[0]; ++x)
        for (int y = 0; y < d.nc[1]; ++y) coltab.push_back(make_int2(d.cell_off + (x * d.nc[1] + y) * d.nc[2], r));
    }
    coltab.push_back(make_int2(h->ncells, R));
    upload(coltab, h->d_coltab, s);
    // (one per population: the two column passes may run concurrently)
    HIPCHK(h, h->d_colbase.alloc((size_t)(h->ncols + 1) * 4));
    HIPCHK(h, h->d_colbase_q.alloc((size_t)(h->ncols + 1) * 4));
  }
  // each population's cluster slots and tiles (n: its beads per replica)
  auto plan_half = [&](const std::vector<int>& n, int ci, DevBuf& base, DevBuf& cl, DevBuf& ncl, DevBuf& tiles,
                       DevBuf& part, DevBuf& off, int& ntiles) -> gcme_status {
    std::vector<int> hbase(R), toff(R + 1);
    std::vector<Tile> th;
    const int wpb = pair_waves_per_block();
    int slots = 0;
    for (int r = 0; r < R; ++r) {
      const RepDesc& d = h->rep[r];
      const int cap = n[r] == 0 ? 0 : (n[r] + ci - 1) / ci + d.nc[0] * d.nc[1];
      hbase[r] = slots;
      toff[r] = (int)th.size();
      for (int c = 0; c < cap; c += wpb) th.push_back(Tile{r, slots + c, std::min(wpb, cap - c), slots});
      slots += cap;
    }
    toff[R] = (int)th.size();
    ntiles = (int)th.size();
    if (th.empty()) th.push_back(Tile{0, 0, 0, 0});
    upload(hbase, base, s);
    upload(th, tiles, s);
    upload(toff, off, s);
    HIPCHK(h, cl.alloc((size_t)std::max(1, slots) * 8));
    HIPCHK(h, ncl.alloc((size_t)R * 4));
    HIPCHK(h, hipMemsetAsync(ncl.p, 0, (size_t)R * 4, s));
    HIPCHK(h, part.alloc((size_t)std::max(1, ntiles) * PART_W * 8));
    return GCME_OK;
  };
  if (col_mode(h, false) && half_fits) {
    h->hci = h->tune.beads_per_cluster < 4 ? 4 : h->tune.beads_per_cluster;
    gcme_status e = plan_half(h->nb, h->hci, h->d_hbase, h->d_hcl, h->d_hncl, h->d_htiles, h->part_h, h->d_off_h,
                              h->ntiles_h);
    if (e != GCME_OK) return e;
  }
  if (col_mode(h, true) && h->NQ > 0 && half_fits) {
    h->hqci = h->tune.charges_per_cluster < 4 ? 4 : h->tune.charges_per_cluster;
    gcme_status e = plan_half(h->nq, h->hqci, h->d_hqbase, h->d_hqcl, h->d_hqncl, h->d_hqtiles, h->part_hq,
                              h->d_off_hq, h->ntiles_hq);
    if (e != GCME_OK) return e;
  }

  // slab correction (per 256-bead tile) and bonds (per 256-bond tile)
  {
    std::vector<int> on(R, 0);
    std::vector<double> kb(2 * R, 0.0);
    h->any_slab = false;
    for (int r = 0; r < R; ++r) {
      on[r] = (h->hp[r].flags & GCME_FLAG_SLAB_CORRECTION) && h->nq[r] > 0 ? 1 : 0;
      h->any_slab |= on[r] != 0;
      kb[r] = h->hp[r].bond_k;
      kb[R + r] = h->hp[r].bond_b;
    }
    upload(on, h->d_slab_on, s);
    upload(kb, h->d_bond_kb, s);
    HIPCHK(h, h->slab_mz.alloc((size_t)std::max(1, h->ntiles_256) * 8));
    HIPCHK(h, h->part[SLOT_SLAB].alloc((size_t)std::max(1, h->ntiles_256) * PART_W * 8));
    upload(toff_256, h->d_off[SLOT_SLAB], s);
    std::vector<int2> bl;
    std::vector<int> bcnt(R), bfirst(R), toff_b;
    for (int r = 0; r < R; ++r) {
      bfirst[r] = (int)bl.size();
      bcnt[r] = (int)h->bonds[r].size();
      bl.insert(bl.end(), h->bonds[r].begin(), h->bonds[r].end());
    }
    std::vector<Tile> tb = make_tiles(bfirst, bcnt, 256, toff_b);
    h->ntiles_b = (int)tb.size();
    h->nbonds = (long long)bl.size();
    if (bl.empty()) bl.push_back(int2{0, 0});
    if (tb.empty()) tb.push_back(Tile{0, 0, 0, 0});
    upload(bl, h->d_bonds, s);
    upload(tb, h->d_btiles, s);
    upload(toff_b, h->d_off[SLOT_BOND], s);
    HIPCHK(h, h->part[SLOT_BOND].alloc((size_t)std::max(1, h->ntiles_b) * PART_W * 8));
    std::vector<int2> im = h->images;
    h->nimages = (int)im.size();
    if (im.empty()) im.push_back(int2{0, 0});
    upload(im, h->d_images, s);
  }

  // cells
  int nbs = (h->ncells + 1023) / 1024;
  HIPCHK(h, h->counts.alloc((size_t)h->ncells * 4));
  HIPCHK(h, h->qcounts.alloc((size_t)h->ncells * 4));
  HIPCHK(h, h->fill.alloc((size_t)h->ncells * 4));
  HIPCHK(h, h->start.alloc((size_t)(h->ncells + 1) * 4));
  HIPCHK(h, h->qstart.alloc((size_t)(h->ncells + 1) * 4));
  HIPCHK(h, h->bsum.alloc((size_t)2 * (nbs + 1) * 4));
  HIPCHK(h, hipMemsetAsync(h->counts.p, 0, (size_t)h->ncells * 4, s));
  HIPCHK(h, hipMemsetAsync(h->qcounts.p, 0, (size_t)h->ncells * 4, s));

  // half-complex mesh
  HIPCHK(h, h->Qc.alloc((size_t)h->cgrid_total * cs));

  // integrator constants, energy constants
  std::vector<double> imass(R * MAXT, 1.0), c1(R), c2s(R * MAXT, 0.0), dtv(R), consts(2 * R), Av(R * MAXT * MAXT, 0.0),
      dself(R * MAXT, 0.0);
  std::vector<int> lang(R);
  for (int r = 0; r < R; ++r) {
    const HostRep& p = h->hp[r];
    double cc = std::exp(-p.gamma * p.dt);
    c1[r] = cc;
    dtv[r] = p.dt;
    lang[r] = p.gamma > 0.0 ? 1 : 0;
    for (int t = 0; t < p.nt; ++t) {
      imass[r * MAXT + t] = 1.0 / p.mass[t];
      c2s[r * MAXT + t] = std::sqrt((1.0 - cc * cc) * p.kT / p.mass[t]);
      for (int u = 0; u < p.nt; ++u) Av[(size_t)r * MAXT * MAXT + t * MAXT + u] = p.A[t * p.nt + u];
    }
    // constants of eq. ewald: U_corr and U_self, and dU_self/da_t
    double sz2 = 0, sza = 0;
    for (int i = h->boff[r]; i < h->boff[r] + h->nb[r]; ++i) {
      double zz = (double)h->h_z[i] * h->h_z[i];
      int t = h->h_type[i];
      sz2 += zz;
      sza += zz / p.a[t];
      dself[r * MAXT + t] += -0.5 * p.lB * zz / (p.a[t] * p.a[t]);
    }
    consts[2 * r] = -p.lB * p.beta / std::sqrt(M_PI) * sz2;
    consts[2 * r + 1] = 0.5 * p.lB * sza;
  }
  upload(imass, h->d_imass, s);
  upload(c1, h->d_c1, s);
  upload(c2s, h->d_c2s, s);
  upload(dtv, h->d_dt, s);
  upload(lang, h->d_lang, s);
  upload(consts, h->d_consts, s);
  upload(Av, h->d_Avals, s);
  upload(dself, h->d_dself, s);
  {
    std::vector<double> sa(R * MAXT, 0.0);
    for (int r = 0; r < R; ++r)
      for (int t = 0; t < h->hp[r].nt; ++t) sa[r * MAXT + t] = -0.5 * h->hp[r].lB / (h->hp[r].a[t] * h->hp[r].a[t]);
    upload(sa, h->d_self_a, s);
  }
  upload(h->rep, h->d_rep, s);
  HIPCHK(h, hipStreamSynchronize(s));
  h->plan_dirty = false;
  return GCME_OK;
}

PairLaunch pair_args(gcme_handle h, bool charged) {
  PairLaunch a{};
  a.rep = h->d_rep.as<RepDesc>();
  a.gcm = h->d_gcm.p;
  a.elec = h->d_elec.p;
  a.adj = h->d_adj.p;
  for (int k = 0; k < 3; ++k) a.F[k] = Fk(h, k);
  a.status = h->d_status.as<unsigned>();
  a.fscale = h->fscale();
  if (charged) {
    a.tiles = h->d_tiles_q.as<Tile>();
    a.ntiles = h->ntiles_q;
    a.cl = h->d_cl_q.as<int2>();
    a.ncl = h->ncl_q;
    a.ci = h->tune.charges_per_cluster;
    a.direct = (h->tune.direct_pairs >> 1) & 1;
    a.cap = h->cap_q;
    a.list = h->list_q.as<uint32_t>();
    a.count = h->cnt_q.as<int>();
    a.pk = h->q_pk.as<uint4>();
    a.start = h->qstart.as<int>();
    a.qidx = h->q_idx.as<int>();
    a.part = h->part[SLOT_REAL].as<double>();
    a.adj_part = h->adjp[1].as<double>();
    a.dbead = h->per_bead ? h->dbead_q.as<double>() : nullptr;
    a.vjp = h->vjp ? h->vjp_sorted.as<double>() : nullptr;
    a.nbeads = h->N;
  } else {
    a.tiles = h->d_tiles_g.as<Tile>();
    a.ntiles = h->ntiles_g;
    a.cl = h->d_cl_g.as<int2>();
    a.ncl = h->ncl_g;
    a.ci = h->tune.beads_per_cluster;
    a.direct = h->tune.direct_pairs & 1;
    a.cap = h->cap_g;
    a.list = h->list_g.as<uint32_t>();
    a.count = h->cnt_g.as<int>();
    a.pk = h->b_pk.as<uint4>();
    a.start = h->start.as<int>();
    a.part = h->part[SLOT_GCM].as<double>();
    a.adj_part = h->adjp[0].as<double>();
    a.dbead = h->per_bead ? h->dbead_g.as<double>() : nullptr;
    a.vjp = h->vjp ? h->vjp_sorted.as<double>() : nullptr;
    a.nbeads = h->N;
  }
  return a;
}

EwaldLaunch ewald_args(gcme_handle h) {
  EwaldLaunch a{};
  a.rep = h->d_rep.as<RepDesc>();
  a.kv = h->d_ewk.as<EwaldK>();
  a.items_s = h->d_ew_items_s.as<EwaldItem>();
  a.nitems_s = h->nitems_ew_s;
  a.items_f = h->d_ew_items_f.as<EwaldItem>();
  a.nitems_f = h->nitems_ew_f;
  a.sp = h->ew_sp.as<double>();
  a.qpk = h->q_pk.as<uint4>();
  a.qidx = h->q_idx.as<int>();
  for (int k = 0; k < 3; ++k) a.F[k] = Fk(h, k);
  a.part = h->part[SLOT_EWALD].as<double>();
  a.status = h->d_status.as<unsigned>();
  a.fscale = h->fscale();
  return a;
}

SlabLaunch slab_args(gcme_handle h) {
  SlabLaunch a{};
  a.rep = h->d_rep.as<RepDesc>();
  a.tiles = h->d_tiles_256.as<Tile>();
  a.ntiles = h->any_slab ? h->ntiles_256 : 0;
  a.tile_off = h->d_off[SLOT_SLAB].as<int>();
  a.on = h->d_slab_on.as<int>();
  a.mz = h->slab_mz.as<long long>();
  for (int k = 0; k < 3; ++k) a.F[k] = Fk(h, k);
  a.fscale = h->fscale();
  a.status = h->d_status.as<unsigned>();
  a.part = h->part[SLOT_SLAB].as<double>();
  return a;
}

BondLaunch bond_args(gcme_handle h) {
  BondLaunch a{};
  a.rep = h->d_rep.as<RepDesc>();
  a.tiles = h->d_btiles.as<Tile>();
  a.ntiles = h->ntiles_b;
  a.bonds = h->d_bonds.as<int2>();
  a.slot_of = h->slot_of.as<int>();
  a.nbeads = h->N;
  a.k = h->d_bond_kb.as<double>();
  a.b = a.k + h->R;
  for (int k = 0; k < 3; ++k) a.F[k] = Fk(h, k);
  a.fscale = h->fscale();
  a.status = h->d_status.as<unsigned>();
  a.part = h->part[SLOT_BOND].as<double>();
  return a;
}

PmeLaunch pme_args(gcme_handle h) {
  PmeLaunch a{};
  a.rep = h->d_rep.as<RepDesc>();
  a.nrep = h->R;
  a.nq = h->NQ;
  a.order = h->order;
  a.qpk = h->q_pk.as<uint4>();
  for (int k = 0; k < 3; ++k) {
    a.F[k] = Fk(h, k);
    a.items[k] = h->d_items[k].as<LineItem>();
    a.nitems[k] = h->nitems[k];
    a.lb[k] = h->lb[k];
    a.maxK[k] = h->maxK[k];
  }
  a.qidx = h->q_idx.as<int>();
  a.qstart = h->qstart.as<int>();
  a.tiles = h->d_mtiles.as<MeshTile>();
  a.ntiles = h->nmtiles;
  a.tx = h->mtx;
  a.ty = h->mty;
  a.Qc = h->Qc.p;
  a.plane_major = h->yx_fused ? 1 : 0;
  a.plane_elems = h->plane_elems;
  a.plane_k = -1;  // K0 = K1 of every replica with a mesh, else 0
  for (int r = 0; r < h->R; ++r) {
    const int k0 = h->rep[r].K[0], k1 = h->rep[r].K[1];
    if (k0 == 0) continue;
    if (a.plane_k < 0) a.plane_k = k0 == k1 ? k0 : 0;
    if (k0 != a.plane_k || k1 != a.plane_k) a.plane_k = 0;
  }
  if (a.plane_k < 0) a.plane_k = 0;
  a.tw = h->d_tw.p;
  a.radix = h->d_rad.as<int>();
  a.bsp = h->d_bsp.p;
  a.freq = h->d_freq.p;
  a.part = h->part[SLOT_RECIP].as<double>();
  a.status = h->d_status.as<unsigned>();
  a.fscale = h->fscale();
  a.qscale = h->qscale();
  return a;
}

// The gather's launch: the mesh launch with the gather's own tiles.
PmeLaunch gather_args(gcme_handle h, PmeLaunch p) {
  p.tiles = h->d_gtiles.as<MeshTile>();
  p.ntiles = h->ngtiles;
  p.tx = h->gtx;
  p.ty = h->gty;
  return p;
}

IntLaunch int_args(gcme_handle h) {
  IntLaunch a{};
  a.rep = h->d_rep.as<RepDesc>();
  a.tiles = h->d_tiles_256.as<Tile>();
  a.ntiles = h->ntiles_256;
  a.inv_mass = h->d_imass.as<double>();
  a.c1 = h->d_c1.as<double>();
  a.c2s = h->d_c2s.as<double>();
  a.dt = h->d_dt.as<double>();
  a.langevin = h->d_lang.as<int>();
  a.nbeads = h->N;
  a.seed = h->seed;
  a.step = h->d_step.as<unsigned long long>();
  a.fscale_inv = 1.0 / h->fscale();
  a.part = h->part[SLOT_KIN].as<double>();
  return a;
}

// Stage indices of gcme_stage_name.
enum {
  ST_INT_FIRST = 0, ST_SORT, ST_LIST_GCM, ST_PAIR_GCM, ST_LIST_ELEC, ST_PAIR_ELEC, ST_SPREAD, ST_FFT_Y,
  ST_FFT_CONV, ST_FFT_Y_INV, ST_GATHER, ST_INT_LAST
};

// The stamp slots of a stage's launch while the context times its stages,
// else null.
unsigned long long* stamps_for(gcme_handle h, int stage) {
  return h->timing ? h->stamps.as<unsigned long long>() + 2 * h->stamp_off[stage] : nullptr;
}

// Whether an evaluation's excluded-volume (charged) pairs take the
// half-shell kernel (not with parameter derivatives, which the cluster
// kernels provide).
bool half_gcm(gcme_handle h, bool adj) { return col_mode(h, false) && !adj && h->ntiles_h > 0; }
bool half_elec(gcme_handle h, bool adj) { return col_mode(h, true) && !adj && h->ntiles_hq > 0; }

PairLaunch pair_args_half(gcme_handle h, bool charged) {
  PairLaunch a = pair_args(h, charged);
  if (charged) {
    a.tiles = h->d_hqtiles.as<Tile>();
    a.ntiles = h->ntiles_hq;
    a.cl = h->d_hqcl.as<int2>();
    a.hncl = h->d_hqncl.as<int>();
    a.ci = h->hqci;
    a.part = h->part_hq.as<double>();
  } else {
    a.tiles = h->d_htiles.as<Tile>();
    a.ntiles = h->ntiles_h;
    a.cl = h->d_hcl.as<int2>();
    a.hncl = h->d_hncl.as<int>();
    a.ci = h->hci;
    a.part = h->part_h.as<double>();
  }
  return a;
}

ColLaunch col_args(gcme_handle h, bool charged) {
  ColLaunch c{};
  c.start = charged ? h->qstart.as<int>() : h->start.as<int>();
  c.coltab = h->d_coltab.as<int2>();
  c.ncols = h->ncols;
  c.ci = charged ? h->hqci : h->hci;
  c.rep_base = charged ? h->d_hqbase.as<int>() : h->d_hbase.as<int>();
  c.cl = charged ? h->d_hqcl.as<int2>() : h->d_hcl.as<int2>();
  c.ncl = charged ? h->d_hqncl.as<int>() : h->d_hncl.as<int>();
  c.colbase = charged ? h->d_colbase_q.as<int>() : h->d_colbase.as<int>();
  c.nrep = h->R;
  return c;
}

// The excluded-volume pairs of an evaluation on stream s.
void enqueue_gcm_pairs(gcme_handle h, hipStream_t s, bool ev, bool adj) {
  if (half_gcm(h, adj)) {
    ColLaunch c = col_args(h, false);
    c.stamps = stamps_for(h, ST_LIST_GCM);
    launch_col_clusters(s, c);
    PairLaunch g = pair_args_half(h, false);
    g.stamps = stamps_for(h, ST_PAIR_GCM);
    launch_pair_gcm_col(s, g, h->fp64, ev, col_mode(h, false) == 1);
    return;
  }
  PairLaunch g = pair_args(h, false);
  g.stamps = stamps_for(h, ST_LIST_GCM);
  launch_nl_build(s, g);
  g.stamps = stamps_for(h, ST_PAIR_GCM);
  launch_pair_gcm(s, g, h->fp64, ev, adj);
}

// The charged beads' real-space pairs of an evaluation on stream s.
void enqueue_elec_pairs(gcme_handle h, hipStream_t s, bool ev, bool adj) {
  if (half_elec(h, adj)) {
    ColLaunch c = col_args(h, true);
    c.stamps = stamps_for(h, ST_LIST_ELEC);
    launch_col_clusters(s, c);
    PairLaunch q = pair_args_half(h, true);
    q.stamps = stamps_for(h, ST_PAIR_ELEC);
    launch_pair_elec_col(s, q, h->fp64, ev, col_mode(h, true) == 1);
    return;
  }
  PairLaunch q = pair_args(h, true);
  q.stamps = stamps_for(h, ST_LIST_ELEC);
  launch_nl_build(s, q);
  q.stamps = stamps_for(h, ST_PAIR_ELEC);
  launch_pair_elec(s, q, h->fp64, ev, adj);
}

// Sort the state A into B by cell (and the charged copy), on stream s;
// bin = false when the integrator has already binned A.
void enqueue_sort(gcme_handle h, hipStream_t s, bool bin = true) {
  // counts are left cleared by the previous permute (and at plan build)
  CellView c = cview(h);
  // a step's sort (after the integrator's binning) starts the next step:
  // its scan advances the step counter
  if (!bin) c.step = h->d_step.as<unsigned long long>();
  if (bin) launch_bin(s, viewA(h), h->d_rep.as<RepDesc>(), c, h->N);
  if (h->nimages > 0) {
    ImageLaunch im{};
    im.rep = h->d_rep.as<RepDesc>();
    im.pairs = h->d_images.as<int2>();
    im.n = h->nimages;
    im.nbeads = h->N;
    im.status = h->d_status.as<unsigned>();
    launch_images(s, im, viewA(h), c);
  }
  launch_scan(s, c);
  launch_scatter(s, c, h->N);
  launch_permute(s, viewA(h), viewB(h), h->b_pk.as<uint4>(), c, qview(h), h->N);
}

// Forces (and partial sums if ev) on the sorted copy B; F must be cleared.
// The excluded-volume kernel, the charged real-space kernel and the mesh
// chain are independent and all add into the integer force accumulator, so
// they run as three concurrent branches (fork/join with events; captured as
// parallel graph branches).
void enqueue_forces(gcme_handle h, hipStream_t s, bool ev, bool adj) {
  if (h->NQ == 0) {
    enqueue_gcm_pairs(h, s, ev, adj);
    launch_bonds(s, bond_args(h), viewB(h));
    return;
  }
  // Stream of each part by layout (gcme_tuning.stream_layout).  A
  // dependency between streams costs several microseconds in a captured
  // graph, against about two within one, so fewer branches can win even
  // though the parts then overlap less.  Parts are issued in the order
  // listed (a captured graph submits its nodes in that order).
  //   layout: excluded-volume pairs, charged pairs, mesh chain (0 = the
  //   context's stream, 1 and 2 = the second and third), issue order
  struct Layout {
    int g, q, p;
    char order[4];
  };
  static const Layout kLayouts[6] = {{0, 1, 2, "gqp"}, {0, 0, 2, "gqp"}, {1, 1, 0, "pqg"},
                                     {1, 1, 0, "gqp"}, {0, 1, 1, "gpq"}, {1, 0, 0, "gpq"}};
  // a context without auxiliary streams (the no-alloc entry point's) runs
  // the three parts in sequence on s
  static const Layout kSingle = {0, 0, 0, "gqp"};
  const Layout& L = h->aux[0] ? kLayouts[h->tune.stream_layout] : kSingle;
  hipStream_t st3[3] = {s, h->aux[0], h->aux[1]};
  hipStream_t sg = st3[L.g], sq = st3[L.q], sp = st3[L.p];
  const bool use1 = L.g == 1 || L.q == 1 || L.p == 1, use2 = L.g == 2 || L.q == 2 || L.p == 2;
  if (use1 || use2) (void)hipEventRecord(h->ev_fork, s);
  if (use1) (void)hipStreamWaitEvent(h->aux[0], h->ev_fork, 0);
  if (use2) (void)hipStreamWaitEvent(h->aux[1], h->ev_fork, 0);
  PmeLaunch p = pme_args(h);
  auto gcm = [&]() { enqueue_gcm_pairs(h, sg, ev, adj); };
  auto elec = [&]() { enqueue_elec_pairs(h, sq, ev, adj); };
  auto mesh = [&]() {
    p.stamps = stamps_for(h, ST_SPREAD);
    launch_spread_z(sp, p, h->fp64);
    if (h->yx_fused) {
      p.stamps = stamps_for(h, ST_FFT_CONV);
      launch_fft_yx_conv(sp, p, h->fp64, ev);
    } else {
      p.stamps = stamps_for(h, ST_FFT_Y);
      launch_fft_y(sp, p, h->fp64, false);
      p.stamps = stamps_for(h, ST_FFT_CONV);
      launch_fft_x_conv(sp, p, h->fp64, ev);
      p.stamps = stamps_for(h, ST_FFT_Y_INV);
      launch_fft_y(sp, p, h->fp64, true);
    }
    p.stamps = stamps_for(h, ST_GATHER);
    launch_z_gather(sp, gather_args(h, p), h->fp64);
    p.stamps = nullptr;
    // replicas with the exact reciprocal sum instead of a mesh
    launch_ewald(sp, ewald_args(h), h->fp64, ev);
    // the slab systems' extra terms (none in bulk)
    launch_slab(sp, slab_args(h), viewB(h));
    launch_bonds(sp, bond_args(h), viewB(h));
  };
  for (int k = 0; k < 3; ++k) {
    if (L.order[k] == 'g') gcm();
    if (L.order[k] == 'q') elec();
    if (L.order[k] == 'p') mesh();
  }
  if (use1) {
    (void)hipEventRecord(h->ev_join[0], h->aux[0]);
    (void)hipStreamWaitEvent(s, h->ev_join[0], 0);
  }
  if (use2) {
    (void)hipEventRecord(h->ev_join[1], h->aux[1]);
    (void)hipStreamWaitEvent(s, h->ev_join[1], 0);
  }
}

void enqueue_outputs(gcme_handle h, hipStream_t s, const gcme_io* io, bool kin) {
  long long* const F3[3] = {Fk(h, 0), Fk(h, 1), Fk(h, 2)};
  if (io->force) launch_forces_out(s, viewB(h), F3, io->force, h->N, h->N, 1.0 / h->fscale());
  bool adj = io->dE_dA || io->dE_dsigma || io->dE_da;
  if (io->energy || io->virial || adj) {
    FinalLaunch f{};
    f.rep = h->d_rep.as<RepDesc>();
    f.nrep = h->R;
    for (int sl = 0; sl < N_SLOTS; ++sl) {
      f.part[sl] = h->part[sl].as<double>();
      f.slot_off[sl] = h->d_off[sl].as<int>();
    }
    if (half_gcm(h, adj)) {
      f.part[SLOT_GCM] = h->part_h.as<double>();
      f.slot_off[SLOT_GCM] = h->d_off_h.as<int>();
    }
    if (half_elec(h, adj)) {
      f.part[SLOT_REAL] = h->part_hq.as<double>();
      f.slot_off[SLOT_REAL] = h->d_off_hq.as<int>();
    }
    if (h->NQ == 0) {
      // no charged beads: the charged kernels did not run, their slots are empty ranges
      f.part[SLOT_REAL] = nullptr;
      f.part[SLOT_RECIP] = nullptr;
      f.part[SLOT_EWALD] = nullptr;
    }
    if (!h->any_slab) f.part[SLOT_SLAB] = nullptr;
    if (h->ntiles_b == 0) f.part[SLOT_BOND] = nullptr;
    f.consts = h->d_consts.as<double>();
    f.energy = io->energy;
    f.virial = io->virial;
    f.have_kin = kin ? 1 : 0;
    f.adj_part[0] = h->adjp[0].as<double>();
    f.adj_part[1] = h->NQ > 0 ? h->adjp[1].as<double>() : nullptr;
    f.adj_off[0] = h->d_adj_off[0].as<int>();
    f.adj_off[1] = h->d_adj_off[1].as<int>();
    f.Avals = h->d_Avals.as<double>();
    f.dself = h->d_dself.as<double>();
    f.dE_dA = io->dE_dA;
    f.dE_dsigma = io->dE_dsigma;
    f.dE_da = io->dE_da;
    f.adj_scale = io->force_vjp ? 2.0 : 1.0;
    f.vjp = io->force_vjp ? 1 : 0;
    launch_finalize(s, f);
  }
}

gcme_status check_ready(gcme_handle h) {
  if (!h) return GCME_EINVAL;
  for (int r = 0; r < h->R; ++r)
    if (!h->hp[r].set) return fail(h, GCME_ESTATE, "parameters not set for replica " + std::to_string(r));
  if (!h->have_state) return fail(h, GCME_ESTATE, "state not set (gcme_set_state)");
  if (!h->images_checked) {
    // an image bead: immobile type, the opposite charge of its source
    for (const int2& pr : h->images) {
      const int r = (int)(std::upper_bound(h->boff.begin(), h->boff.begin() + h->R, pr.x) - h->boff.begin()) - 1;
      if (!std::isinf(h->hp[r].mass[h->h_type[pr.x]]))
        return fail(h, GCME_EINVAL, "an image bead's type must have infinite mass");
      if (h->h_z[pr.x] != -h->h_z[pr.y])
        return fail(h, GCME_EINVAL, "an image bead's charge must be the opposite of its source's");
    }
    h->images_checked = true;
  }
  if (h->plan_dirty) return build_plan(h);
  return GCME_OK;
}

// One full evaluation on stream s: sort, forces, commit B -> A.
void enqueue_eval(gcme_handle h, hipStream_t s, bool ev, bool adj) {
  enqueue_sort(h, s);
  enqueue_forces(h, s, ev, adj);
}

// n steps of the integrator (forces of the current state in F, indexed in
// the order of A) are: the first half of step 1 with the binning of its new
// positions (kick, drift, noise; clears F), then per step the rest of the
// sort and the forces, and between steps the second half kick fused with the
// next first half and binning; the last step ends with the plain second half
// kick, written back to A.  enqueue_step_rest enqueues all of a step but its
// first half: `between` selects the fused ending.
void enqueue_step_rest(gcme_handle h, hipStream_t s, bool between, bool ev) {
  IntLaunch ia = int_args(h);
  long long* const F3[3] = {Fk(h, 0), Fk(h, 1), Fk(h, 2)};
  enqueue_sort(h, s, false);
  enqueue_forces(h, s, ev, false);
  ia.stamps = stamps_for(h, ST_INT_LAST);
  if (between)
    launch_int_between(s, ia, viewB(h), viewA(h), F3, cview(h));
  else
    launch_int_last(s, ia, viewB(h), viewA(h), F3, ev);
}

gcme_status capture(gcme_handle h, bool between, bool ev, hipGraphExec_t* out, int repeat = 1) {
  hipGraph_t g = nullptr;
  HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < repeat; ++k) enqueue_step_rest(h, h->cap_stream, between, ev);
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (e != hipSuccess) return fail(h, GCME_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(h, GCME_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  return GCME_OK;
}

// The graphs of a run of steps without observation: one step (g_mid),
// MID_BATCH steps (g_midn) and the last step (g_last).
gcme_status prepare_graphs(gcme_handle h) {
  gcme_status st = GCME_OK;
  if (!h->g_mid) st = capture(h, true, false, &h->g_mid);
  if (st == GCME_OK && !h->g_midn) st = capture(h, true, false, &h->g_midn, MID_BATCH);
  if (st == GCME_OK && !h->g_last) st = capture(h, false, false, &h->g_last);
  return st;
}

gcme_status ensure_forces(gcme_handle h) {
  if (h->forces_valid) return GCME_OK;
  launch_fill_i64(h->stream, h->F.as<long long>(), 0, 3LL * h->N);
  enqueue_eval(h, h->stream, false, false);
  launch_commit(h->stream, viewB(h), viewA(h), h->N);
  HIPCHK(h, hipGetLastError());
  h->forces_valid = true;
  return GCME_OK;
}

// The per-bead device buffers of a context (their sizes depend only on the
// bead count), cleared where a first read needs zeros.  Without `derivs`
// the buffers only the per-bead derivatives, the force vector-Jacobian
// product, bonds and images use are left at a minimal size.
bool alloc_bead_buffers(gcme_handle h, bool derivs) {
  const size_t N = (size_t)h->N, Nd = derivs ? N : 1;
  bool ok = true;
  for (int k = 0; k < 3; ++k) {
    ok &= h->a_pos[k].alloc(N * 4) == hipSuccess;
    ok &= h->b_pos[k].alloc(N * 4) == hipSuccess;
    ok &= h->a_vel[k].alloc(N * 8) == hipSuccess;
    ok &= h->b_vel[k].alloc(N * 8) == hipSuccess;
  }
  ok &= h->a_param.alloc(N * 4) == hipSuccess;
  ok &= h->b_param.alloc(N * 4) == hipSuccess;
  ok &= h->a_id.alloc(N * 4) == hipSuccess;
  ok &= h->b_pk.alloc(N * 16) == hipSuccess;
  ok &= h->b_id.alloc(N * 4) == hipSuccess;
  ok &= h->cell.alloc(N * 4) == hipSuccess;
  ok &= h->tmp.alloc(N * 4) == hipSuccess;
  ok &= h->slot_of.alloc(Nd * 4) == hipSuccess;
  ok &= h->slot_a.alloc(Nd * 4) == hipSuccess;
  ok &= h->dbead_g.alloc(Nd * 8) == hipSuccess;
  ok &= h->dbead_q.alloc(Nd * 8) == hipSuccess;
  ok &= h->vjp_sorted.alloc(Nd * 24) == hipSuccess;
  ok &= h->F.alloc(N * 24) == hipSuccess;
  ok &= h->d_status.alloc(64) == hipSuccess;
  ok &= h->d_step.alloc(64) == hipSuccess;
  ok &= h->d_pairs.alloc(64) == hipSuccess;
  if (!ok) return false;
  ok &= hipMemsetAsync(h->d_status.p, 0, 64, h->stream) == hipSuccess;
  ok &= hipMemsetAsync(h->d_step.p, 0, 64, h->stream) == hipSuccess;
  ok &= hipMemsetAsync(h->F.p, 0, N * 24, h->stream) == hipSuccess;
  ok &= hipMemsetAsync(h->slot_of.p, 0, Nd * 4, h->stream) == hipSuccess;
  ok &= hipMemsetAsync(h->slot_a.p, 0, Nd * 4, h->stream) == hipSuccess;
  ok &= hipStreamSynchronize(h->stream) == hipSuccess;
  return ok;
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of the current device's scratch (device `dev`).
gcme_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(nullptr, GCME_EDEVICE, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, GCME_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GCME_OK;
}

}  // namespace

extern "C" {

gcme_status gcme_create(const gcme_create_info* info, gcme_handle* out) {
  if (!info || !out) return fail(nullptr, GCME_EINVAL, "null argument");
  if (info->n_replicas < 1 || info->n_replicas > 65535 || !info->n_beads)
    return fail(nullptr, GCME_EINVAL, "n_replicas must be in 1..65535 with a host n_beads array");
  if (info->precision != GCME_FP64 && info->precision != GCME_MIXED)
    return fail(nullptr, GCME_EINVAL, "precision must be GCME_FP64 or GCME_MIXED");
  long long total = 0;
  for (int r = 0; r < info->n_replicas; ++r) {
    if (info->n_beads[r] < 2) return fail(nullptr, GCME_EINVAL, "every replica needs >= 2 beads");
    total += info->n_beads[r];
  }
  if (total > (1LL << 30)) return fail(nullptr, GCME_EINVAL, "too many beads");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(nullptr, GCME_EDEVICE, "no HIP device");
  if (info->device < 0 || info->device >= ndev) return fail(nullptr, GCME_EINVAL, "bad device ordinal");
  gcme_handle h = new gcme_ctx();
  h->device = info->device;
  if (hipSetDevice(h->device) != hipSuccess) {
    delete h;
    return fail(nullptr, GCME_EDEVICE, "hipSetDevice failed");
  }
  h->R = info->n_replicas;
  h->nb.assign(info->n_beads, info->n_beads + h->R);
  h->boff.assign(h->R, 0);
  for (int r = 1; r < h->R; ++r) h->boff[r] = h->boff[r - 1] + h->nb[r - 1];
  h->N = (int)total;
  h->fp64 = info->precision == GCME_FP64;
  h->seed = info->seed;
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) == hipSuccess && lds > 0)
      h->lds_max = lds - 4096;  // less the kernels' static LDS
  }
  h->hp.assign(h->R, HostRep{});
  h->bonds.assign(h->R, {});
  h->nq.assign(h->R, 0);
  h->qoff.assign(h->R, 0);
  if (info->stream) {
    h->stream = (hipStream_t)info->stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      delete h;
      return fail(nullptr, GCME_EDEVICE, "stream creation failed");
    }
    h->own_stream = true;
  }
  bool sok = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) == hipSuccess;
  for (auto& a : h->aux) sok &= hipStreamCreateWithFlags(&a, hipStreamNonBlocking) == hipSuccess;
  sok &= hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) == hipSuccess;
  for (auto& e : h->ev_join) sok &= hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (!sok) {
    delete h;
    return fail(nullptr, GCME_EDEVICE, "stream/event creation failed");
  }
  if (!alloc_bead_buffers(h, true)) {
    delete h;
    return fail(nullptr, GCME_ENOMEM, "device allocation failed");
  }
  *out = h;
  return GCME_OK;
}

gcme_status gcme_set_params(gcme_handle h, int32_t replica, const gcme_params* p) {
  if (!h || !p) return h ? fail(h, GCME_EINVAL, "null params") : GCME_EINVAL;
  if (replica < -1 || replica >= h->R) return fail(h, GCME_EINVAL, "replica out of range");
  for (int k = 0; k < 3; ++k)
    if (!(p->box[k] > 0.0) || !std::isfinite(p->box[k])) return fail(h, GCME_EGEOMETRY, "box edges must be > 0");
  if (!(p->cutoff > 0.0)) return fail(h, GCME_EGEOMETRY, "cutoff must be > 0");
  for (int k = 0; k < 3; ++k)
    if (p->cutoff > 0.5 * p->box[k] * (1.0 + 1e-12))
      return fail(h, GCME_EGEOMETRY, "cutoff exceeds half the box edge (minimum image)");
  if (!(p->beta > 0.0)) return fail(h, GCME_EINVAL, "beta must be > 0");
  if (!(p->lB >= 0.0)) return fail(h, GCME_EINVAL, "lB must be >= 0");
  if (p->order < 3 || p->order > 8) return fail(h, GCME_EUNSUPPORTED, "B-spline order must be 3..8");
  if (!(p->kmax >= 0.0) || !std::isfinite(p->kmax)) return fail(h, GCME_EINVAL, "kmax must be >= 0");
  if (p->kmax > 0.0) {
    // exact reciprocal sum: the integer wave vectors per axis stay bounded
    for (int k = 0; k < 3; ++k)
      if (p->kmax * p->box[k] / (2.0 * M_PI) > (double)EW_NMAX)
        return fail(h, GCME_EUNSUPPORTED, "kmax L / (2 pi) must be <= 64 on every axis");
  } else {
    for (int k = 0; k < 3; ++k) {
      int K = p->grid[k];
      if (K < 8 || K > 512 || !smooth(K)) return fail(h, GCME_EUNSUPPORTED, "mesh sizes must be 2^a 3^b in 8..512");
      if (p->order > K / 2) return fail(h, GCME_EUNSUPPORTED, "order must be <= K/2");
    }
  }
  if (p->n_types < 1 || p->n_types > MAXT) return fail(h, GCME_EUNSUPPORTED, "n_types must be 1..4");
  if (!p->A || !p->sigma || !p->a) return fail(h, GCME_EINVAL, "A, sigma and a are required");
  const int nt = p->n_types;
  for (int t = 0; t < nt; ++t) {
    if (!(p->sigma[t] > 0.0) || !(p->a[t] > 0.0)) return fail(h, GCME_EINVAL, "sigma and a must be > 0");
    if (p->mass && !(p->mass[t] > 0.0)) return fail(h, GCME_EINVAL, "masses must be > 0");
    for (int u = 0; u < nt; ++u) {
      double x = p->A[t * nt + u], y = p->A[u * nt + t];
      if (!std::isfinite(x) || std::fabs(x - y) > 1e-12 * std::max(1.0, std::fabs(x)))
        return fail(h, GCME_EINVAL, "A must be finite and symmetric");
    }
  }
  if (!(p->kT >= 0.0) || !(p->dt >= 0.0) || !(p->gamma >= 0.0)) return fail(h, GCME_EINVAL, "kT, dt, gamma must be >= 0");
  if (!(p->bond_k >= 0.0) || !std::isfinite(p->bond_k) || !(p->bond_b >= 0.0) || !std::isfinite(p->bond_b))
    return fail(h, GCME_EINVAL, "bond_k and bond_b must be finite and >= 0");
  if (p->flags & ~(GCME_FLAG_STRICT_CONTACT | GCME_FLAG_ALL_RECIPROCAL | GCME_FLAG_SLAB_CORRECTION))
    return fail(h, GCME_EINVAL, "unknown flag");
  double beta = p->beta;
  if (p->flags & GCME_FLAG_ALL_RECIPROCAL) {
    // beta = alpha_ij = sqrt(pi/2)/a_ij with a_ij = sqrt(2) a: one radius for all
    for (int t = 1; t < nt; ++t)
      if (std::fabs(p->a[t] - p->a[0]) > 1e-12 * p->a[0])
        return fail(h, GCME_EINVAL, "the all-reciprocal splitting needs one charge radius a for every type");
    beta = std::sqrt(M_PI) / (2.0 * p->a[0]);
  }
  if (p->flags & GCME_FLAG_STRICT_CONTACT) {
    // no-collapse condition between unit charges of opposite sign
    for (int t = 0; t < nt; ++t)
      for (int u = 0; u < nt; ++u) {
        double s2 = p->sigma[t] * p->sigma[t] + p->sigma[u] * p->sigma[u];
        double aij = std::sqrt(p->a[t] * p->a[t] + p->a[u] * p->a[u]);
        double lhs = p->A[t * nt + u] / std::pow(s2, 1.5);
        double rhs = 4.0 * std::pow(M_PI, 1.5) * p->lB / (std::pow(3.0, 1.5) * aij);
        if (!(lhs > rhs)) return fail(h, GCME_EINVAL, "contact repulsion does not exceed contact attraction");
      }
  }
  int r0 = replica < 0 ? 0 : replica, r1 = replica < 0 ? h->R : replica + 1;
  for (int r = 0; r < h->R; ++r)
    if (h->hp[r].set && (r < r0 || r >= r1) && h->hp[r].order != p->order)
      return fail(h, GCME_EUNSUPPORTED, "all replicas must use the same B-spline order");
  for (int r = r0; r < r1; ++r) {
    HostRep& q = h->hp[r];
    for (int k = 0; k < 3; ++k) {
      q.box[k] = p->box[k];
      q.K[k] = p->kmax > 0.0 ? 0 : p->grid[k];  // no mesh with the exact sum
    }
    q.kmax = p->kmax;
    q.rc = p->cutoff;
    q.beta = beta;
    q.lB = p->lB;
    q.kT = p->kT;
    q.dt = p->dt;
    q.gamma = p->gamma;
    q.order = p->order;
    q.nt = nt;
    q.flags = p->flags;
    q.bond_k = p->bond_k;
    q.bond_b = p->bond_b;
    for (int i = 0; i < nt * nt; ++i) q.A[i] = p->A[i];
    for (int t = 0; t < nt; ++t) {
      q.sigma[t] = p->sigma[t];
      q.a[t] = p->a[t];
      q.mass[t] = p->mass ? p->mass[t] : 1.0;
    }
    q.set = true;
  }
  h->plan_dirty = true;
  h->forces_valid = false;
  h->images_checked = h->images.empty();
  if (h->have_state) {
    // types must stay within the new type count
    for (int r = r0; r < r1; ++r)
      for (int i = h->boff[r]; i < h->boff[r] + h->nb[r]; ++i)
        if (h->h_type[i] >= h->hp[r].nt) {
          h->have_state = false;
          return fail(h, GCME_EINVAL, "state has bead types beyond n_types; set the state again");
        }
  }
  return GCME_OK;
}

gcme_status gcme_set_bonds(gcme_handle h, int64_t n_bonds, const int32_t* pairs) {
  if (!h) return GCME_EINVAL;
  if (n_bonds < 0 || (n_bonds > 0 && !pairs)) return fail(h, GCME_EINVAL, "n_bonds must be >= 0, pairs non-null");
  if (n_bonds > (int64_t)1 << 30) return fail(h, GCME_EUNSUPPORTED, "at most 2^30 bonds");
  std::vector<std::vector<int2>> by(h->R);
  for (int64_t m = 0; m < n_bonds; ++m) {
    const int i = pairs[2 * m], j = pairs[2 * m + 1];
    if (i < 0 || j < 0 || i >= h->N || j >= h->N || i == j)
      return fail(h, GCME_EINVAL, "bond indices must be distinct beads in 0..N-1");
    // the replica of bead i (replicas are consecutive index ranges)
    const int r = (int)(std::upper_bound(h->boff.begin(), h->boff.begin() + h->R, i) - h->boff.begin()) - 1;
    if (j < h->boff[r] || j >= h->boff[r] + h->nb[r]) return fail(h, GCME_EINVAL, "a bond joins two replicas");
    by[r].push_back(int2{i, j});
  }
  h->bonds.swap(by);
  h->plan_dirty = true;
  h->forces_valid = false;
  return GCME_OK;
}

gcme_status gcme_set_images(gcme_handle h, int64_t n_images, const int32_t* pairs) {
  if (!h) return GCME_EINVAL;
  if (n_images < 0 || (n_images > 0 && !pairs)) return fail(h, GCME_EINVAL, "n_images must be >= 0, pairs non-null");
  if (n_images > h->N) return fail(h, GCME_EINVAL, "more images than beads");
  std::vector<char> role(h->N, 0);  // 1 image, 2 source
  std::vector<int2> im;
  im.reserve((size_t)n_images);
  for (int64_t m = 0; m < n_images; ++m) {
    const int i = pairs[2 * m], j = pairs[2 * m + 1];
    if (i < 0 || j < 0 || i >= h->N || j >= h->N || i == j)
      return fail(h, GCME_EINVAL, "image and source must be distinct beads in 0..N-1");
    const int r = (int)(std::upper_bound(h->boff.begin(), h->boff.begin() + h->R, i) - h->boff.begin()) - 1;
    if (j < h->boff[r] || j >= h->boff[r] + h->nb[r]) return fail(h, GCME_EINVAL, "an image in another replica");
    if (role[i] != 0 || role[j] == 1) return fail(h, GCME_EINVAL, "a bead is an image twice, or an image and a source");
    role[i] = 1;
    role[j] = 2;
    im.push_back(int2{i, j});
  }
  h->images.swap(im);
  h->images_checked = false;
  h->plan_dirty = true;
  h->forces_valid = false;
  return GCME_OK;
}

gcme_status gcme_set_state(gcme_handle h, const double* pos, const double* vel, const int32_t* type,
                           const int32_t* z) {
  if (!h) return GCME_EINVAL;
  if (!pos || !type || !z) return fail(h, GCME_EINVAL, "pos, type and z are required");
  for (int r = 0; r < h->R; ++r)
    if (!h->hp[r].set) return fail(h, GCME_ESTATE, "set parameters before the state");
  HIPCHK(h, hipSetDevice(h->device));
  const int N = h->N;
  std::vector<int> t(N), zz(N);
  HIPCHK(h, hipMemcpyAsync(t.data(), type, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(zz.data(), z, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  std::vector<int> nq(h->R, 0), qoff(h->R, 0);
  int NQ = 0;
  for (int r = 0; r < h->R; ++r) {
    long long net = 0;
    qoff[r] = NQ;
    for (int i = h->boff[r]; i < h->boff[r] + h->nb[r]; ++i) {
      if (t[i] < 0 || t[i] >= h->hp[r].nt) return fail(h, GCME_EINVAL, "bead type out of range");
      if (zz[i] < -127 || zz[i] > 127) return fail(h, GCME_EINVAL, "charge numbers must be in -127..127");
      net += zz[i];
      if (zz[i] != 0) ++nq[r];
    }
    if (net != 0) return fail(h, GCME_ENONNEUTRAL, "replica " + std::to_string(r) + " is not neutral");
    NQ += nq[r];
  }
  std::vector<uint32_t> prm(N);
  std::vector<int> id(N);
  for (int r = 0; r < h->R; ++r)
    for (int i = h->boff[r]; i < h->boff[r] + h->nb[r]; ++i) {
      prm[i] = pack_param(t[i], zz[i], r);
      id[i] = i;
    }
  h->h_type = t;
  h->h_z = zz;
  h->nq = nq;
  h->qoff = qoff;
  h->NQ = NQ;
  HIPCHK(h, h->q_pk.alloc((size_t)std::max(1, NQ) * 16));
  HIPCHK(h, h->q_idx.alloc((size_t)std::max(1, NQ) * 4));
  HIPCHK(h, hipMemcpyAsync(h->a_param.p, prm.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(h->a_id.p, id.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream));
  for (int k = 0; k < 3; ++k) {
    if (vel)
      HIPCHK(h, hipMemcpyAsync(h->a_vel[k].p, vel + (size_t)k * N, (size_t)N * 8, hipMemcpyDeviceToDevice, h->stream));
    else
      HIPCHK(h, hipMemsetAsync(h->a_vel[k].p, 0, (size_t)N * 8, h->stream));
  }
  // the state is new: rebuild the plan (charged ranges, constants)
  h->plan_dirty = true;
  h->have_state = true;
  h->images_checked = h->images.empty();
  gcme_status st = build_plan(h);
  if (st != GCME_OK) return st;
  launch_ingest(h->stream, pos, N, N, h->d_rep.as<RepDesc>(), nullptr, viewA(h), h->F.as<long long>(), N);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemsetAsync(h->d_step.p, 0, 8, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->step = 0;
  h->forces_valid = false;
  return GCME_OK;
}

gcme_status gcme_get_state(gcme_handle h, double* pos, double* vel, uint64_t* step) {
  if (!h) return GCME_EINVAL;
  if (!h->have_state) return fail(h, GCME_ESTATE, "state not set");
  HIPCHK(h, hipSetDevice(h->device));
  if (h->plan_dirty) {
    gcme_status st = build_plan(h);
    if (st != GCME_OK) return st;
  }
  if (pos || vel) launch_state_out(h->stream, viewA(h), h->d_rep.as<RepDesc>(), pos, vel, h->N, h->N);
  HIPCHK(h, hipGetLastError());
  if (step) *step = h->step;
  return GCME_OK;
}

gcme_status gcme_forces_energy(gcme_handle h, const gcme_io* io) {
  if (!h) return GCME_EINVAL;
  if (!io) return fail(h, GCME_EINVAL, "null io");
  gcme_status st = check_ready(h);
  if (st != GCME_OK) return st;
  if (io->dE_da || io->dE_da_bead)
    for (int r = 0; r < h->R; ++r)
      if (h->hp[r].flags & GCME_FLAG_ALL_RECIPROCAL)
        return fail(h, GCME_EUNSUPPORTED, "dE/da is not provided with the all-reciprocal splitting");
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = h->stream;
  if (io->pos)
    launch_ingest(s, io->pos, h->N, h->N, h->d_rep.as<RepDesc>(), nullptr, viewA(h), h->F.as<long long>(), h->N);
  else
    launch_fill_i64(s, h->F.as<long long>(), 0, 3LL * h->N);
  const bool pb = io->dE_dsigma_bead || io->dE_da_bead;
  bool adj = io->dE_dA || io->dE_dsigma || io->dE_da || pb;
  if (io->force_vjp && (pb || !adj))
    return fail(h, GCME_EINVAL, "force_vjp needs dE_dA, dE_dsigma or dE_da and no per-bead outputs");
  bool ev = io->energy || io->virial || adj;
  // uncharged beads get no charged-kernel store
  if (pb) launch_fill_i64(s, h->dbead_q.as<long long>(), 0, h->N);
  h->per_bead = pb;
  h->vjp = io->force_vjp != nullptr;
  if (h->vjp) {
    // v to the sorted order the pair kernels index
    enqueue_sort(h, s);
    launch_gather_vjp(s, viewB(h), io->force_vjp, h->vjp_sorted.as<double>(), h->N);
    enqueue_forces(h, s, ev, adj);
  } else {
    enqueue_eval(h, s, ev, adj);
  }
  h->per_bead = false;
  h->vjp = false;
  enqueue_outputs(h, s, io, false);
  if (pb)
    launch_bead_adj_out(s, viewB(h), h->dbead_g.as<double>(), h->dbead_q.as<double>(), h->d_self_a.as<double>(),
                        io->dE_dsigma_bead, io->dE_da_bead, h->N);
  launch_commit(s, viewB(h), viewA(h), h->N);
  HIPCHK(h, hipGetLastError());
  h->forces_valid = true;
  return GCME_OK;
}

gcme_status gcme_forces_energy_noalloc(const gcme_params* p, int32_t n_beads, int32_t precision,
                                       const double* pos, const int32_t* type, const int32_t* z, double* force,
                                       double* energy, double* virial, void* stream) {
  if (!p || !pos || !type || !z) return fail(nullptr, GCME_EINVAL, "params, pos, type and z are required");
  if (n_beads < 2) return fail(nullptr, GCME_EINVAL, "n_beads must be >= 2");
  if (precision != GCME_FP64 && precision != GCME_MIXED)
    return fail(nullptr, GCME_EINVAL, "precision must be GCME_FP64 or GCME_MIXED");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, GCME_EDEVICE, "no current HIP device");
  void* base = nullptr;
  gcme_status st = scratch_address(dev, &base);
  if (st != GCME_OK) return st;
  // a transient context on the caller's stream: no streams, events or
  // graphs of its own, every device buffer carved from the scratch
  gcme_handle h = new gcme_ctx();
  h->device = dev;
  h->stream = (hipStream_t)stream;
  h->R = 1;
  h->nb.assign(1, n_beads);
  h->boff.assign(1, 0);
  h->N = n_beads;
  h->fp64 = precision == GCME_FP64;
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
      h->lds_max = lds - 4096;
  }
  h->hp.assign(1, HostRep{});
  h->bonds.assign(1, {});
  h->nq.assign(1, 0);
  h->qoff.assign(1, 0);
  Arena arena;
  arena.base = (char*)base;
  arena.size = GCME_NOALLOC_SCRATCH_BYTES;
  t_arena = &arena;
  if (!alloc_bead_buffers(h, false)) {
    st = GCME_ENOMEM;
    h->err = "device buffers";
  }
  if (st == GCME_OK) st = gcme_set_params(h, -1, p);
  if (st == GCME_OK) st = gcme_set_state(h, pos, nullptr, type, z);
  if (st == GCME_OK) {
    gcme_io io{};
    io.force = force;
    io.energy = energy;
    io.virial = virial;
    st = gcme_forces_energy(h, &io);
  }
  if (st == GCME_OK) st = gcme_sync(h);
  t_arena = nullptr;
  if (st == GCME_ENOMEM && arena.need > 0) {
    g_create_err = "the evaluation needs " + std::to_string(arena.need) + " bytes of device scratch, more than the " +
                   std::to_string((size_t)GCME_NOALLOC_SCRATCH_BYTES) +
                   " of the no-alloc entry point (use a context from gcme_create)";
  } else if (st != GCME_OK) {
    g_create_err = h->err;
  }
  delete h;
  return st;
}

gcme_status gcme_step(gcme_handle h, int32_t n_steps, const gcme_io* observe) {
  if (!h) return GCME_EINVAL;
  if (n_steps < 0) return fail(h, GCME_EINVAL, "n_steps must be >= 0");
  if (observe && observe->pos) return fail(h, GCME_EINVAL, "observe->pos must be NULL");
  if (observe && n_steps > 0 && (observe->dE_dsigma_bead || observe->dE_da_bead || observe->force_vjp))
    return fail(h, GCME_EINVAL, "per-bead derivatives and force_vjp come from gcme_forces_energy");
  gcme_status st = check_ready(h);
  if (st != GCME_OK) return st;
  HIPCHK(h, hipSetDevice(h->device));
  st = ensure_forces(h);
  if (st != GCME_OK) return st;
  if (n_steps == 0) {
    if (observe) {
      // re-evaluate at the current positions to fill the outputs
      return gcme_forces_energy(h, observe);
    }
    // no step: capture the graphs a run will replay, if a change of
    // parameters or tuning dropped them
    return prepare_graphs(h);
  }
  bool obs = observe != nullptr;
  // every graph a run of steps replays is captured at the first run after a
  // change of plan or tuning, whatever that run's length, so that a later
  // run of any length launches graphs only (capture and instantiation are
  // host work of milliseconds)
  st = prepare_graphs(h);
  if (st != GCME_OK) return st;
  hipGraphExec_t* last = obs ? &h->g_obs : &h->g_last;
  if (!*last) {
    st = capture(h, false, obs, last);
    if (st != GCME_OK) return st;
  }
  {
    IntLaunch ia = int_args(h);
    long long* const F3[3] = {Fk(h, 0), Fk(h, 1), Fk(h, 2)};
    CellView c = cview(h);
    launch_int_first(h->stream, ia, viewA(h), F3, &c);
  }
  // long runs replay MID_BATCH steps per graph launch: the host-side cost of a
  // launch (tens of microseconds) is paid once per batch
  int rest = n_steps - 1;
  for (; rest >= MID_BATCH; rest -= MID_BATCH) HIPCHK(h, hipGraphLaunch(h->g_midn, h->stream));
  for (int i = 0; i < rest; ++i) HIPCHK(h, hipGraphLaunch(h->g_mid, h->stream));
  HIPCHK(h, hipGraphLaunch(*last, h->stream));
  if (obs) {
    // the step left A == B (same order); outputs read B and the partials
    enqueue_outputs(h, h->stream, observe, true);
    HIPCHK(h, hipGetLastError());
  }
  h->step += (uint64_t)n_steps;
  return GCME_OK;
}

gcme_status gcme_sync(gcme_handle h) {
  if (!h) return GCME_EINVAL;
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  unsigned st = 0;
  HIPCHK(h, hipMemcpy(&st, h->d_status.p, 4, hipMemcpyDeviceToHost));
  if (st) {
    HIPCHK(h, hipMemset(h->d_status.p, 0, 4));
    if (st & STATUS_LIST_OVERFLOW)
      return fail(h, GCME_EOVERFLOW, "neighbour list capacity exceeded (raise gcme_tuning.list_slack_pct)");
    if (st & STATUS_SLOT_MAP)
      return fail(h, GCME_EDEVICE, "a bond or image named a bead the sort did not place (inconsistent state)");
    return fail(h, GCME_EOVERFLOW, "fixed-point force accumulator overflow (forces too large)");
  }
  return GCME_OK;
}

const char* gcme_last_error(gcme_handle h) { return h ? h->err.c_str() : g_create_err.c_str(); }

gcme_status gcme_get_tuning(gcme_handle h, gcme_tuning* t) {
  if (!h || !t) return GCME_EINVAL;
  *t = h->tune;
  return GCME_OK;
}

gcme_status gcme_set_tuning(gcme_handle h, const gcme_tuning* t) {
  if (!h || !t) return GCME_EINVAL;
  gcme_tuning n = h->tune;
  if (t->cells_per_cutoff >= 0) {
    if (t->cells_per_cutoff < 1 || t->cells_per_cutoff > 4) return fail(h, GCME_EINVAL, "cells_per_cutoff in 1..4");
    n.cells_per_cutoff = t->cells_per_cutoff;
  }
  auto okc = [](int v) { return v == 2 || v == 4 || v == 8; };
  if (t->beads_per_cluster >= 0) {
    if (!okc(t->beads_per_cluster)) return fail(h, GCME_EINVAL, "beads_per_cluster in {2,4,8}");
    n.beads_per_cluster = t->beads_per_cluster;
  }
  if (t->charges_per_cluster >= 0) {
    if (!okc(t->charges_per_cluster)) return fail(h, GCME_EINVAL, "charges_per_cluster in {2,4,8}");
    n.charges_per_cluster = t->charges_per_cluster;
  }
  if (t->list_slack_pct >= 0) {
    if (t->list_slack_pct > 1000) return fail(h, GCME_EINVAL, "list_slack_pct in 0..1000");
    n.list_slack_pct = t->list_slack_pct;
  }
  if (t->direct_pairs >= 0) {
    if (t->direct_pairs > 3) return fail(h, GCME_EINVAL, "direct_pairs in 0..3");
    n.direct_pairs = t->direct_pairs;
  }
  if (t->half_pairs >= 0) {
    if ((t->half_pairs & 3) > 2 || ((t->half_pairs >> 2) & 3) > 2 || t->half_pairs > 15)
      return fail(h, GCME_EINVAL, "half_pairs: two bits per pair type, each 0..2");
    n.half_pairs = t->half_pairs;
  }
  if (t->stream_layout >= 0) {
    if (t->stream_layout > 5) return fail(h, GCME_EINVAL, "stream_layout in 0..5");
    if (t->stream_layout != h->tune.stream_layout) h->drop_graphs();  // no new plan needed
    n.stream_layout = t->stream_layout;
    h->tune.stream_layout = n.stream_layout;
  }
  {
    const int32_t* in[4] = {&t->mesh_tile_x, &t->mesh_tile_y, &t->gather_tile_x, &t->gather_tile_y};
    int32_t* out[4] = {&n.mesh_tile_x, &n.mesh_tile_y, &n.gather_tile_x, &n.gather_tile_y};
    for (int k = 0; k < 4; ++k) {
      if (*in[k] < 0) continue;
      if (*in[k] > 16) return fail(h, GCME_EINVAL, "mesh and gather tile sizes in 0..16");
      *out[k] = *in[k];
    }
  }
  if (n.cells_per_cutoff != h->tune.cells_per_cutoff || n.beads_per_cluster != h->tune.beads_per_cluster ||
      n.charges_per_cluster != h->tune.charges_per_cluster || n.list_slack_pct != h->tune.list_slack_pct ||
      n.direct_pairs != h->tune.direct_pairs || n.mesh_tile_x != h->tune.mesh_tile_x ||
      n.mesh_tile_y != h->tune.mesh_tile_y || n.gather_tile_x != h->tune.gather_tile_x ||
      n.gather_tile_y != h->tune.gather_tile_y || n.half_pairs != h->tune.half_pairs) {
    h->tune = n;
    h->plan_dirty = true;
    h->drop_graphs();
  }
  return GCME_OK;
}

gcme_status gcme_count_pairs(gcme_handle h, uint64_t* n_pairs) {
  if (!h || !n_pairs) return GCME_EINVAL;
  gcme_status st = check_ready(h);
  if (st != GCME_OK) return st;
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = h->stream;
  enqueue_sort(h, s);
  HIPCHK(h, hipMemsetAsync(h->d_pairs.p, 0, 8, s));
  PairLaunch g = pair_args(h, false);
  g.pair_count = h->d_pairs.as<unsigned long long>();
  // counting run: forces go to a separate buffer so the state's forces stay valid
  DevBuf cnt_F;
  HIPCHK(h, cnt_F.alloc((size_t)h->N * 24));
  for (int k = 0; k < 3; ++k) g.F[k] = cnt_F.as<long long>() + (size_t)k * h->N;
  launch_nl_build(s, g);
  launch_pair_gcm(s, g, h->fp64, false, false);
  HIPCHK(h, hipGetLastError());
  unsigned long long c = 0;
  HIPCHK(h, hipMemcpyAsync(&c, h->d_pairs.p, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  *n_pairs = c / 2;
  // sorting B does not disturb A or F
  return GCME_OK;
}

gcme_status gcme_autotune(gcme_handle h) {
  if (!h) return GCME_EINVAL;
  gcme_status st = check_ready(h);
  if (st != GCME_OK) return st;
  HIPCHK(h, hipSetDevice(h->device));
  st = ensure_forces(h);
  if (st != GCME_OK) return st;
  hipStream_t s = h->stream;
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  // every candidate is timed on the current state (forces only); the forces
  // are restored afterwards
  DevBuf saveF;
  HIPCHK(h, saveF.alloc((size_t)h->N * 24));
  HIPCHK(h, hipMemcpyAsync(saveF.p, h->F.p, (size_t)h->N * 24, hipMemcpyDeviceToDevice, s));
  const int keep_layout = h->tune.stream_layout;
  // 1. stream-launched evaluations over cell size, cluster sizes and lists
  std::vector<std::pair<float, gcme_tuning>> cands;
  const int ncc_list[] = {2, 3, 4};
  const int ci_list[] = {2, 4, 8};
  // per pair type: 0 = neighbour lists, 1 = list-free, 2 = column clusters
  // half shell, 3 = column clusters both ends (clusters of 4 or 8)
  for (int ncc : ncc_list)
    for (int cg : ci_list)
      for (int cq : ci_list)
        for (int mg = 0; mg < 4; ++mg)
          for (int mq = 0; mq < 4; ++mq) {
          if (h->NQ == 0 && (cq != ci_list[0] || mq > 0)) continue;
          if ((mg >= 2 && cg == 2) || (mq >= 2 && cq == 2)) continue;
          const int dp = (mg > 0 ? 1 : 0) | (mq > 0 ? 2 : 0);
          const int hp = (mg >= 2 ? mg - 1 : 0) | ((mq >= 2 ? mq - 1 : 0) << 2);
          gcme_tuning t{ncc, cg, cq, -1, dp, keep_layout, -1, -1, -1, -1, hp};
          if (gcme_set_tuning(h, &t) != GCME_OK) continue;
          if (build_plan(h) != GCME_OK) continue;
          float ms = 0;
          for (int rep = 0; rep < 3; ++rep) {
            launch_fill_i64(s, h->F.as<long long>(), 0, 3LL * h->N);
            (void)hipEventRecord(e0, s);
            enqueue_eval(h, s, false, false);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float m = 0;
            (void)hipEventElapsedTime(&m, e0, e1);
            if (rep > 0) ms += m;
          }
          cands.push_back({ms, t});
        }
  std::sort(cands.begin(), cands.end(),
            [](const std::pair<float, gcme_tuning>& x, const std::pair<float, gcme_tuning>& y) { return x.first < y.first; });
  gcme_tuning best = cands.empty() ? h->tune : cands[0].second;
  // 1b. the mesh tile shapes, for the best of them, the spread's then the
  //     gather's: whole evaluations are timed, since the mesh passes run
  //     beside the pair kernels.  A shape the plan has to shrink to fit LDS
  //     is the smaller one, not retimed.
  if (h->NQ > 0) {
    static const int kShapes[][2] = {{4, 4}, {2, 2}, {2, 4}, {4, 2}, {8, 4}, {4, 8}, {8, 8}, {16, 8}, {16, 16}, {1, 1}};
    for (int pass = 0; pass < 2; ++pass) {
      float best_ms = 1e30f;
      int bx = pass == 0 ? best.mesh_tile_x : best.gather_tile_x, by = pass == 0 ? best.mesh_tile_y : best.gather_tile_y;
      for (const auto& sh : kShapes) {
        gcme_tuning t = best;
        (pass == 0 ? t.mesh_tile_x : t.gather_tile_x) = sh[0];
        (pass == 0 ? t.mesh_tile_y : t.gather_tile_y) = sh[1];
        if (gcme_set_tuning(h, &t) != GCME_OK) continue;
        if (build_plan(h) != GCME_OK) continue;
        if (h->nmtiles == 0) break;  // no mesh: nothing to choose
        if ((pass == 0 ? h->mtx : h->gtx) != sh[0] || (pass == 0 ? h->mty : h->gty) != sh[1]) continue;
        float ms = 0;
        for (int rep = 0; rep < 3; ++rep) {
          launch_fill_i64(s, h->F.as<long long>(), 0, 3LL * h->N);
          (void)hipEventRecord(e0, s);
          enqueue_eval(h, s, false, false);
          (void)hipEventRecord(e1, s);
          (void)hipEventSynchronize(e1);
          float m = 0;
          (void)hipEventElapsedTime(&m, e0, e1);
          if (rep > 0) ms += m;
        }
        if (ms < best_ms) {
          best_ms = ms;
          bx = sh[0];
          by = sh[1];
        }
      }
      (pass == 0 ? best.mesh_tile_x : best.gather_tile_x) = bx;
      (pass == 0 ? best.mesh_tile_y : best.gather_tile_y) = by;
    }
    for (auto& c : cands) {
      c.second.mesh_tile_x = best.mesh_tile_x;
      c.second.mesh_tile_y = best.mesh_tile_y;
      c.second.gather_tile_x = best.gather_tile_x;
      c.second.gather_tile_y = best.gather_tile_y;
    }
  }
  // 2. the best few, with every charged-cluster size and stream layout, as
  //    replays of the captured step graph from the saved state: stream
  //    dependencies cost differently in a graph, and only whole steps show
  //    how the branches overlap the sort and the integrator.  The state
  //    (order, positions, velocities, forces, step counter) is restored
  //    before each candidate and at the end.
  if (h->NQ > 0) {
    const size_t N = (size_t)h->N;
    DevBuf sp[3], sv[3], sprm, sid, sstep;
    for (int k = 0; k < 3; ++k) {
      HIPCHK(h, sp[k].alloc(N * 4));
      HIPCHK(h, sv[k].alloc(N * 8));
      HIPCHK(h, hipMemcpyAsync(sp[k].p, h->a_pos[k].p, N * 4, hipMemcpyDeviceToDevice, s));
      HIPCHK(h, hipMemcpyAsync(sv[k].p, h->a_vel[k].p, N * 8, hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(h, sprm.alloc(N * 4));
    HIPCHK(h, sid.alloc(N * 4));
    HIPCHK(h, sstep.alloc(8));
    HIPCHK(h, hipMemcpyAsync(sprm.p, h->a_param.p, N * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipMemcpyAsync(sid.p, h->a_id.p, N * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipMemcpyAsync(sstep.p, h->d_step.p, 8, hipMemcpyDeviceToDevice, s));
    auto restore = [&]() -> hipError_t {
      hipError_t e = hipSuccess;
      for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        e = hipMemcpyAsync(h->a_pos[k].p, sp[k].p, N * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h->a_vel[k].p, sv[k].p, N * 8, hipMemcpyDeviceToDevice, s);
      }
      if (e == hipSuccess) e = hipMemcpyAsync(h->a_param.p, sprm.p, N * 4, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(h->a_id.p, sid.p, N * 4, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(h->d_step.p, sstep.p, 8, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(h->F.p, saveF.p, N * 24, hipMemcpyDeviceToDevice, s);
      return e;
    };
    float best_t = 1e30f;
    std::vector<gcme_tuning> second;
    for (size_t c = 0; c < cands.size() && second.size() < 4 * 3; ++c) {
      for (int cq : ci_list) {
        gcme_tuning t = cands[c].second;
        t.charges_per_cluster = cq;
        bool dup = false;
        for (const gcme_tuning& u : second)
          dup = dup || (u.cells_per_cutoff == t.cells_per_cutoff && u.beads_per_cluster == t.beads_per_cluster &&
                        u.charges_per_cluster == t.charges_per_cluster && u.direct_pairs == t.direct_pairs &&
                        u.half_pairs == t.half_pairs);
        if (!dup) second.push_back(t);
      }
    }
    for (const gcme_tuning& base : second) {
      for (int lay = 0; lay < 6; ++lay) {
        gcme_tuning t = base;
        t.stream_layout = lay;
        if (gcme_set_tuning(h, &t) != GCME_OK) continue;
        if (build_plan(h) != GCME_OK) continue;  // also clears the cell counts
        hipGraphExec_t ex = nullptr;
        if (capture(h, true, false, &ex) != GCME_OK) continue;
        HIPCHK(h, restore());
        {
          IntLaunch ia = int_args(h);
          long long* const F3[3] = {Fk(h, 0), Fk(h, 1), Fk(h, 2)};
          CellView c = cview(h);
          launch_int_first(s, ia, viewA(h), F3, &c);
        }
        constexpr int WARM = 5, REPS = 20;
        for (int r = 0; r < WARM; ++r) (void)hipGraphLaunch(ex, s);
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < REPS; ++r) (void)hipGraphLaunch(ex, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float m = 0;
        (void)hipEventElapsedTime(&m, e0, e1);
        (void)hipGraphExecDestroy(ex);
        if (m < best_t) {
          best_t = m;
          best = t;
        }
      }
    }
    HIPCHK(h, restore());
    HIPCHK(h, hipMemsetAsync(h->d_status.p, 0, 4, s));
    HIPCHK(h, hipStreamSynchronize(s));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  gcme_set_tuning(h, &best);
  st = build_plan(h);
  if (st != GCME_OK) return st;
  HIPCHK(h, hipMemcpyAsync(h->F.p, saveF.p, (size_t)h->N * 24, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipStreamSynchronize(s));
  HIPCHK(h, hipGetLastError());
  return GCME_OK;
}

static const char* kStageNames[GCME_N_STAGES] = {"int_first", "sort",       "list_gcm",  "pair_gcm",
                                                  "list_elec", "pair_elec",  "spread_z",  "fft_y",
                                                  "fft_conv",  "fft_y_inv",  "z_gather",  "int_last"};

const char* gcme_stage_name(int32_t i) { return (i >= 0 && i < GCME_N_STAGES) ? kStageNames[i] : nullptr; }

gcme_status gcme_profile_step(gcme_handle h, int32_t n_reps, double* ms) {
  if (!h || !ms || n_reps < 1) return h ? fail(h, GCME_EINVAL, "n_reps >= 1 and ms required") : GCME_EINVAL;
  gcme_status st = check_ready(h);
  if (st != GCME_OK) return st;
  HIPCHK(h, hipSetDevice(h->device));
  st = ensure_forces(h);
  if (st != GCME_OK) return st;
  hipStream_t s = h->stream;
  const size_t N = (size_t)h->N;
  // save what the repeated stages disturb
  DevBuf sp[3], sv[3], sF;
  for (int k = 0; k < 3; ++k) {
    HIPCHK(h, sp[k].alloc(N * 4));
    HIPCHK(h, sv[k].alloc(N * 8));
    HIPCHK(h, hipMemcpyAsync(sp[k].p, h->a_pos[k].p, N * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipMemcpyAsync(sv[k].p, h->a_vel[k].p, N * 8, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(h, sF.alloc(N * 24));
  HIPCHK(h, hipMemcpyAsync(sF.p, h->F.p, N * 24, hipMemcpyDeviceToDevice, s));
  enqueue_sort(h, s);
  IntLaunch ia = int_args(h);
  long long* const F3[3] = {Fk(h, 0), Fk(h, 1), Fk(h, 2)};
  PairLaunch g = pair_args(h, false);
  PairLaunch q = pair_args(h, true);
  PmeLaunch p = pme_args(h);
  auto stage = [&](int i, hipStream_t st2) {
    switch (i) {
      case 0: launch_int_first(st2, ia, viewA(h), F3); break;
      case 1: enqueue_sort(h, st2); break;
      case 2:
        if (half_gcm(h, false))
          launch_col_clusters(st2, col_args(h, false));
        else
          launch_nl_build(st2, g);
        break;
      case 3:
        if (half_gcm(h, false))
          launch_pair_gcm_col(st2, pair_args_half(h, false), h->fp64, false, col_mode(h, false) == 1);
        else
          launch_pair_gcm(st2, g, h->fp64, false, false);
        break;
      case 4:
        if (half_elec(h, false))
          launch_col_clusters(st2, col_args(h, true));
        else
          launch_nl_build(st2, q);
        break;
      case 5:
        if (half_elec(h, false))
          launch_pair_elec_col(st2, pair_args_half(h, true), h->fp64, false, col_mode(h, true) == 1);
        else
          launch_pair_elec(st2, q, h->fp64, false, false);
        break;
      case 6: launch_spread_z(st2, p, h->fp64); break;
      case 7:
        if (!h->yx_fused) launch_fft_y(st2, p, h->fp64, false);
        break;
      case 8:
        if (h->yx_fused)
          launch_fft_yx_conv(st2, p, h->fp64, false);
        else
          launch_fft_x_conv(st2, p, h->fp64, false);
        break;
      case 9:
        if (!h->yx_fused) launch_fft_y(st2, p, h->fp64, true);
        break;
      case 10: launch_z_gather(st2, gather_args(h, p), h->fp64); break;
      default: launch_int_last(st2, ia, viewB(h), viewA(h), F3, false); break;
    }
  };
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  for (int i = 0; i < GCME_N_STAGES; ++i) {
    ms[i] = 0.0;
    if (h->NQ == 0 && i >= 4 && i <= 10) continue;
    if (h->yx_fused && (i == 7 || i == 9)) continue;
    // one full evaluation first, so a stage that works in place (the mesh
    // passes) starts from the data a step would give it
    launch_fill_i64(s, h->F.as<long long>(), 0, 3LL * h->N);
    enqueue_eval(h, s, false, false);
    hipGraph_t gr = nullptr;
    hipGraphExec_t ex = nullptr;
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < n_reps; ++r) stage(i, h->cap_stream);
    HIPCHK(h, hipStreamEndCapture(h->cap_stream, &gr));
    HIPCHK(h, hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
    (void)hipGraphDestroy(gr);
    HIPCHK(h, hipGraphLaunch(ex, s));
    launch_fill_i64(s, h->F.as<long long>(), 0, 3LL * h->N);
    enqueue_eval(h, s, false, false);
    HIPCHK(h, hipEventRecord(e0, s));
    HIPCHK(h, hipGraphLaunch(ex, s));
    HIPCHK(h, hipEventRecord(e1, s));
    HIPCHK(h, hipEventSynchronize(e1));
    float m = 0;
    HIPCHK(h, hipEventElapsedTime(&m, e0, e1));
    ms[i] = (double)m / n_reps;
    (void)hipGraphExecDestroy(ex);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // restore
  for (int k = 0; k < 3; ++k) {
    HIPCHK(h, hipMemcpyAsync(h->a_pos[k].p, sp[k].p, N * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->a_vel[k].p, sv[k].p, N * 8, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(h, hipMemcpyAsync(h->F.p, sF.p, N * 24, hipMemcpyDeviceToDevice, s));
  unsigned long long stepv = h->step;
  HIPCHK(h, hipMemcpyAsync(h->d_step.p, &stepv, 8, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemsetAsync(h->d_status.p, 0, 4, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return GCME_OK;
}

gcme_status gcme_time_stages(gcme_handle h, int32_t n_steps, double* ms) {
  if (!h || !ms || n_steps < 1) return h ? fail(h, GCME_EINVAL, "n_steps >= 1 and ms required") : GCME_EINVAL;
  gcme_status st = check_ready(h);
  if (st != GCME_OK) return st;
  HIPCHK(h, hipSetDevice(h->device));
  st = ensure_forces(h);
  if (st != GCME_OK) return st;
  int khz = 0;
  HIPCHK(h, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device));
  if (khz <= 0) return fail(h, GCME_EDEVICE, "no wall-clock rate");
  // stamp slots of every one-kernel stage's launch (wavefronts per launch
  // from the launch shapes; the sort is several kernels and is not timed)
  auto waves = [&](int i) -> int {
    const int wpb = pair_waves_per_block();
    const int nbead_blk = (h->N + BEAD_THREADS - 1) / BEAD_THREADS * (BEAD_THREADS / 64);
    const bool dg = h->tune.direct_pairs & 1, dq = (h->tune.direct_pairs >> 1) & 1;
    const bool mesh = h->NQ > 0 && h->nmtiles > 0;
    switch (i) {
      case ST_INT_FIRST: return nbead_blk;
      case ST_LIST_GCM: return half_gcm(h, false) ? 16 : dg ? 0 : (h->ncl_g + wpb - 1) / wpb * wpb;
      case ST_PAIR_GCM: return half_gcm(h, false) ? h->ntiles_h * wpb : h->ntiles_g * wpb;
      case ST_LIST_ELEC:
        return h->NQ == 0 ? 0 : half_elec(h, false) ? 16 : dq ? 0 : (h->ncl_q + wpb - 1) / wpb * wpb;
      case ST_PAIR_ELEC: return h->NQ == 0 ? 0 : half_elec(h, false) ? h->ntiles_hq * wpb : h->ntiles_q * wpb;
      case ST_SPREAD: return mesh ? h->nmtiles * (FFT_THREADS / 64) : 0;
      case ST_GATHER: return mesh ? h->ngtiles * (FFT_THREADS / 64) : 0;
      case ST_FFT_Y:
      case ST_FFT_Y_INV: return mesh && !h->yx_fused ? h->nitems[1] * (FFT_THREADS / 64) : 0;
      case ST_FFT_CONV:
        return !mesh ? 0
               : h->yx_fused ? h->nitems[0] * (pme_plane_threads(h->plane_elems) / 64)
                             : h->nitems[2] * (FFT_THREADS / 64);
      case ST_INT_LAST: return h->ntiles_256 * (256 / 64);
      default: return 0;
    }
  };
  size_t tot = 0;
  for (int i = 0; i < GCME_N_STAGES; ++i) {
    h->stamp_off[i] = tot;
    h->stamp_nw[i] = waves(i);
    tot += (size_t)h->stamp_nw[i];
  }
  HIPCHK(h, h->stamps.alloc(std::max<size_t>(1, tot) * 16));
  // a one-step graph (the last-step variant, so every step ends with the
  // state committed) whose launches write the stamps
  hipGraphExec_t ex = nullptr;
  h->timing = true;
  st = capture(h, false, false, &ex);
  h->timing = false;
  if (st != GCME_OK) return st;
  hipStream_t s = h->stream;
  std::vector<unsigned long long> hs(2 * std::max<size_t>(1, tot));
  double sum[GCME_N_STAGES] = {};
  IntLaunch ia = int_args(h);
  ia.stamps = h->stamps.as<unsigned long long>() + 2 * h->stamp_off[ST_INT_FIRST];
  long long* const F3[3] = {Fk(h, 0), Fk(h, 1), Fk(h, 2)};
  hipError_t err = hipSuccess;
  for (int k = 0; k < n_steps && err == hipSuccess; ++k) {
    CellView c = cview(h);
    err = hipMemsetAsync(h->stamps.p, 0, tot * 16, s);
    launch_int_first(s, ia, viewA(h), F3, &c);
    if (err == hipSuccess) err = hipGraphLaunch(ex, s);
    if (err == hipSuccess) err = hipMemcpyAsync(hs.data(), h->stamps.p, tot * 16, hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    // each stage's span: its first wavefront's start to its last one's end
    // (a wavefront that leaves early records no end)
    for (int i = 0; i < GCME_N_STAGES && err == hipSuccess; ++i) {
      unsigned long long t0 = ~0ull, t1 = 0;
      for (int w = 0; w < h->stamp_nw[i]; ++w) {
        const unsigned long long a0 = hs[2 * (h->stamp_off[i] + w)], a1 = hs[2 * (h->stamp_off[i] + w) + 1];
        if (a0) t0 = std::min(t0, a0);
        if (a1) t1 = std::max(t1, a1);
      }
      if (t1 > t0 && t0 != ~0ull) sum[i] += (double)(t1 - t0) / (double)khz;
    }
  }
  (void)hipGraphExecDestroy(ex);
  HIPCHK(h, err);
  h->step += (uint64_t)n_steps;
  for (int i = 0; i < GCME_N_STAGES; ++i) ms[i] = sum[i] / n_steps;
  return GCME_OK;
}

void gcme_destroy(gcme_handle h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  delete h;
}

}  // extern "C"
