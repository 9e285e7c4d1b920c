// mcx_capi.cpp - the C ABI of libmcx and the generation driver.
//
// The host side validates and copies the problem, carves the caller's
// workspace, and runs the power iteration: per generation it enqueues the
// birth kernel, then {advance, collide} iterations on the caller's stream
// while the live-particle count (read back asynchronously a few iterations
// behind) bounds the grid of the next launch, then the history-based tail
// kernel and the generation-end kernels.  Nothing of the transport runs on
// the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <deque>
#include <mutex>
#include <vector>

#include "mcx.h"
#include "mcx_launch.hpp"

using namespace mcx;

namespace {

constexpr int RING = 64;
constexpr int DEFAULT_BLOCK = 512;  // event kernels (the collision kernel's reservations)
constexpr int DEFAULT_BLOCK_CE = 256;  // continuous-energy event kernels
constexpr int DEFAULT_TAIL = 4096;
constexpr int DEFAULT_TAIL_MAX = 1 << 17;  // the tail's serial chains, not its size, bound it
constexpr int DEFAULT_LOOKAHEAD = 4;
constexpr int64_t DEFAULT_MAX_EVENTS = 100000;
constexpr int DEFAULT_FLIGHTS = 8;
constexpr int DEFAULT_ROUNDS = 1;
// live-count bound from which an advance launch stages its flux tally in LDS
constexpr int32_t DEFAULT_LDS_TALLY_MIN = 1 << 19;
// flights per particle of the LDS-staged launches (the large ones): fewer
// than the small launches' `flights`, so that lanes idle less behind the
// wavefront's longest chain of crossings
constexpr int DEFAULT_LT_FLIGHTS = 5;
constexpr int LT_BLOCK = 768;  // threads per block of the LDS-staged advance kernel
// polls (about a microsecond each) before a wait of the asynchronous engine
// gives up and reports an error
constexpr uint64_t ASYNC_SPIN_LIMIT = 1ull << 22;

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(char* b) : base(b) {}
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

double fixed_point_scale(double max_term) {
  // largest power of two with max_term * scale < 2^61
  if (!(max_term > 0.0) || !std::isfinite(max_term)) return std::ldexp(1.0, 61);
  int e;
  std::frexp(max_term, &e);  // max_term < 2^e
  return std::ldexp(1.0, 61 - e);
}

// Largest i with grid[i] <= e within [0, n - 2] (the device's bisection).
template <class R>
int host_interval(const R* grid, int n, R e) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (grid[mid] <= e)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Bucket start points of the interval search over a positive increasing
// grid: bucket b covers the bit patterns base + (b << shift) ... base +
// ((b + 1) << shift) - 1; hash[b] is the interval of the bucket's smallest
// value, hash[n_hash] that of the grid's end.  About two buckets per point.
template <class R, class U>
void build_hash(const std::vector<R>& grid, std::vector<int>* hash, int* shift, U* base) {
  const int n = (int)grid.size();
  U b0, b1;
  std::memcpy(&b0, &grid[0], sizeof(U));
  std::memcpy(&b1, &grid[n - 1], sizeof(U));
  const uint64_t span = (uint64_t)(b1 - b0);
  int s = 0;
  while ((span >> s) + 1 > (uint64_t)2 * (uint64_t)n) ++s;
  const uint64_t nb = (span >> s) + 1;
  hash->assign(nb + 1, 0);
  for (uint64_t b = 0; b <= nb; ++b) {
    const uint64_t key = b << s;
    R e;
    if (key > span) {
      e = grid[n - 1];
    } else {
      const U bits = (U)(b0 + key);
      std::memcpy(&e, &bits, sizeof(U));
    }
    (*hash)[b] = host_interval<R>(grid.data(), n, e);
  }
  *shift = s;
  *base = b0;
}

}  // namespace

// Device layout carved from the caller's workspace.
struct Dev {
  uint32_t N = 0, fis_cap = 0;
  int n_bins = 0, stripes = 1;
  size_t n_cnt_slots = 0;
  Tables T{};
  Bank bank[3]{};
  Records R{};
  Accum A{};
  double *src_x = nullptr, *src_y = nullptr, *src_e = nullptr;
  int32_t* src_g = nullptr;
  double *can_x = nullptr, *can_y = nullptr, *can_e = nullptr;
  int32_t* can_g = nullptr;
  uint32_t *offs = nullptr, *chunk_sum = nullptr, *scan_total = nullptr;
  uint32_t *cnt_live = nullptr, *cnt_col = nullptr;
  double *gen_k = nullptr, *gen_h = nullptr, *gen_tal = nullptr;
  unsigned long long* gen_cnt = nullptr;
  uint32_t* gen_m = nullptr;
  double *k_used = nullptr, *xi0 = nullptr, *k_stat = nullptr;
  double *tal_stat = nullptr;  // [mean flux | mean prod | sigma flux | sigma prod]
  uint32_t* ent_hist = nullptr;
  uint32_t* bk_fill = nullptr;  // per bucket of canonical positions: sites filed
  Staging st{};                 // sites filed by bucket (k-eigenvalue runs)
  double* tl_part = nullptr;  // per-block production sums of the generation tallies
  uint32_t* gen_status = nullptr;  // [n_gen_max] status bits per generation
  // persistent engine: per-history outputs, work counter
  unsigned long long* h_kcol = nullptr;
  unsigned long long* h_kabs = nullptr;
  uint32_t* h_cnt = nullptr;
  uint32_t* work = nullptr;
  // asynchronous engine: particle pool and global queues
  AsyncBufs ab{};
  uint64_t n_hist = 0;
  // batches: problem descriptors and per-problem results
  ProbDesc* probs = nullptr;
  unsigned long long* prob_cnt = nullptr;  // [P][N_CNT]
  unsigned long long* prob_k = nullptr;    // [P][4] 128-bit k_col, k_abs sums
  double* prob_kres = nullptr;             // [P][3]
  double* b_flux = nullptr;                // [bins]
  double* b_prod = nullptr;
  unsigned long long* acc_base = nullptr;
  size_t acc_words = 0;
  unsigned long long* rec_base = nullptr;
  size_t rec_words = 0;
};

struct mcx_ctx {
  mcx_options opt{};
  std::string err;
  hipStream_t stream = nullptr;

  // problem on the host
  bool has_geo = false, has_xs = false, has_src = false, bound = false;
  int nx = 0, ny = 0, n_univ = 0, max_rings = 0, bc[4] = {0, 0, 0, 0};
  double pitch = 0, x0 = 0, y0 = 0;
  std::vector<int> n_rings, mats, pin_map;
  std::vector<double> radii;
  int n_mat = 0, G = 0;
  std::vector<double> sig_t, nusf, sst, cum_s, cum_chi;
  std::vector<float> sig_t_f, nusf_f, sst_f, cum_s_f, cum_chi_f;  // FP32-mixed tables
  std::vector<int> last_s, last_chi, fissile;
  mcx_source src{};

  // time-dependent fixed source (empty t_edges = off)
  std::vector<double> t_edges, t_speed;

  // continuous-energy data (ce = true replaces the multigroup tables)
  bool ce = false;
  int ce_n_nuc = 0, ce_n_pts = 0, ce_max_nuc = 0, ce_n_ebins = 0;
  std::vector<double> ce_grid, ce_xs, ce_awr, ce_dens, ce_edges;
  std::vector<int> ce_mat_n, ce_mat_nuc;
  double ce_nu = 0, ce_watt_a = 0, ce_watt_b = 0, ce_e_max = 0, ce_e_cut = 0;
  double ce_src_energy = 0;
  double ce_sigt_min = 0;
  std::vector<double> ce_tf, ce_s;  // ce_xs split into (t, f) pairs and s, same order
  std::vector<float> ce_f32[6];     // binary32 grid, (t, f), masses, densities, edges, s
  std::vector<int> ce_hash, ce_hash_f;
  int ce_hash_shift = 0, ce_hash_shift_f = 0;
  uint64_t ce_hash_base = 0;
  uint32_t ce_hash_base_f = 0;

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int n_gen_max = 0;
  // device limits for the LDS-staged advance kernel
  int dev_cus = 256;
  size_t lds_block_max = 65536;
  Dev d;

  // results of the last run
  int last_n_gen = 0, last_n_inactive = 0, req_n_inactive = 0;
  int run_last_gen = -1;  // the last generation of the run in progress
  bool ran = false, can_continue = false;
  std::vector<double> h_gen_k, h_gen_h, h_kstat;
  std::vector<unsigned long long> h_gen_cnt;
  std::vector<uint32_t> h_gen_m;
  std::vector<mcx_record> h_rec;
  std::vector<mcx_event> h_ev;
  mcx_timing timing{};

  // batches of fixed-source problems (persistent engine)
  bool batch = false;
  int n_probs = 0;
  struct BProb {
    int nx, ny, max_rings, pin_base, univ_base, radii_base, mats_base, bin_base, n_bins;
    double pitch, x0, y0;
    int bc[4];
    uint64_t seed, prob, hist_base;
    uint32_t n_hist;
  };
  std::vector<BProb> bprobs;
  uint64_t batch_hist = 0;
  int batch_bins = 0;
  bool batch_ran = false;
  std::vector<double> h_bk;
  std::vector<unsigned long long> h_bcnt;
  PersistentCfg pcfg{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream the batch graph is recorded on

  // host-side synchronisation helpers
  uint32_t* h_pin = nullptr;  // [RING] live counts + [RING..] status words
  hipEvent_t ev_ring[RING]{};
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  std::vector<hipEvent_t> ev_pool;
  bool time_gen = true;  // the current generation's launches are timed
  std::vector<int> ev_kind;  // 0 advance, 1 collide, 2 tail (pairs in ev_pool)
};

static int fail(mcx_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

static int hip_fail(mcx_ctx* c, hipError_t e, const char* what) {
  return fail(c, MCX_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                               \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
  } while (0)

extern "C" {

int mcx_create(mcx_ctx** out, const mcx_options* opt) {
  if (!out) return MCX_EINVAL;
  *out = nullptr;
  mcx_ctx* c = new (std::nothrow) mcx_ctx();
  if (!c) return MCX_ENOMEM;
  if (opt) c->opt = *opt;
  // block_size == 0: DEFAULT_BLOCK (multigroup) or DEFAULT_BLOCK_CE, resolved per run
  if (c->opt.block_size != 0 &&
      (c->opt.block_size < 64 || c->opt.block_size > 1024 || c->opt.block_size % 64)) {
    delete c;
    return MCX_EINVAL;
  }
  if (c->opt.precision != MCX_FP64 && c->opt.precision != MCX_FP32_MIXED) {
    delete c;
    return MCX_EINVAL;
  }
  // tail_threshold == 0: N / 8 within [DEFAULT_TAIL, DEFAULT_TAIL_MAX] (resolved per run)
  if (c->opt.lookahead <= 0) c->opt.lookahead = DEFAULT_LOOKAHEAD;
  if (c->opt.lookahead > RING - 2) c->opt.lookahead = RING - 2;
  if (c->opt.max_events <= 0) c->opt.max_events = DEFAULT_MAX_EVENTS;
  if (c->opt.flights == 0) c->opt.flights = DEFAULT_FLIGHTS;
  if (c->opt.lds_tally_min == 0) c->opt.lds_tally_min = DEFAULT_LDS_TALLY_MIN;
  if (c->opt.lt_flights == 0) c->opt.lt_flights = std::min(c->opt.flights, DEFAULT_LT_FLIGHTS);
  if (c->opt.lt_flights < 0 || c->opt.lt_flights > 65536) {
    delete c;
    return MCX_EINVAL;
  }
  if (c->opt.rounds == 0) c->opt.rounds = DEFAULT_ROUNDS;
  if (c->opt.rounds < 1 || c->opt.rounds * (c->opt.block_size ? c->opt.block_size : DEFAULT_BLOCK) > 4096) {
    delete c;
    return MCX_EINVAL;
  }
  if (c->opt.flights < 0 || c->opt.flights > 65536) {
    delete c;
    return MCX_EINVAL;
  }
  if (c->opt.engine != MCX_ENGINE_EVENT && c->opt.engine != MCX_ENGINE_PERSISTENT &&
      c->opt.engine != MCX_ENGINE_MONOLITHIC && c->opt.engine != MCX_ENGINE_ASYNC) {
    delete c;
    return MCX_EINVAL;
  }
  if ((c->opt.engine == MCX_ENGINE_PERSISTENT || c->opt.engine == MCX_ENGINE_ASYNC) &&
      c->opt.record_histories) {
    delete c;
    return MCX_EINVAL;
  }
  if (c->opt.event_log < 0 || c->opt.event_log > 65536 ||
      (c->opt.event_log > 0 && !c->opt.record_histories)) {
    delete c;
    return MCX_EINVAL;
  }
  {
    int dev_cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->opt.device) == hipSuccess) {
      dev_cus = prop.multiProcessorCount;
      c->lds_block_max = prop.sharedMemPerBlock;
    }
    c->dev_cus = dev_cus;
    c->pcfg.block = c->opt.p_block ? c->opt.p_block : 256;
    c->pcfg.slots = c->opt.p_slots ? c->opt.p_slots : 512;
    // persistent: two workgroups per CU; asynchronous: one per two CUs (its
    // queue counters are shared by every workgroup: fewer contend less)
    c->pcfg.grid = c->opt.p_grid ? c->opt.p_grid
                                 : c->opt.engine == MCX_ENGINE_ASYNC ? std::max(1, dev_cus / 2)
                                                                     : 2 * dev_cus;
    c->pcfg.tau = c->opt.p_tau > 0.0 ? c->opt.p_tau : 0.75;
    c->pcfg.sort = c->opt.p_sort;
    if (c->opt.p_sort != 0 && c->opt.p_sort != 1) {
      delete c;
      return MCX_EINVAL;
    }
    if (!persistent_config_valid(c->pcfg.block, c->pcfg.slots) || c->pcfg.tau > 1.0 ||
        c->opt.p_grid < 0 || c->opt.p_grid > (1 << 20)) {
      delete c;
      return MCX_EINVAL;
    }
  }
  c->stream = (hipStream_t)c->opt.stream;
  if (hipSetDevice(c->opt.device) != hipSuccess) {
    delete c;
    return MCX_EDEVICE;
  }
  if (hipHostMalloc((void**)&c->h_pin, sizeof(uint32_t) * (RING + 16), hipHostMallocDefault) !=
      hipSuccess) {
    delete c;
    return MCX_EDEVICE;
  }
  for (int k = 0; k < RING; ++k) {
    if (hipEventCreateWithFlags(&c->ev_ring[k], hipEventDisableTiming) != hipSuccess) {
      mcx_destroy(c);
      return MCX_EDEVICE;
    }
  }
  if (hipEventCreate(&c->ev_start) != hipSuccess || hipEventCreate(&c->ev_stop) != hipSuccess) {
    mcx_destroy(c);
    return MCX_EDEVICE;
  }
  *out = c;
  return MCX_OK;
}

void mcx_destroy(mcx_ctx* c) {
  if (!c) return;
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (int k = 0; k < RING; ++k)
    if (c->ev_ring[k]) (void)hipEventDestroy(c->ev_ring[k]);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->ev_start) (void)hipEventDestroy(c->ev_start);
  if (c->ev_stop) (void)hipEventDestroy(c->ev_stop);
  if (c->h_pin) (void)hipHostFree(c->h_pin);
  delete c;
}

const char* mcx_last_error(const mcx_ctx* c) { return c ? c->err.c_str() : "null context"; }

int mcx_load_geometry(mcx_ctx* c, const mcx_geometry* g) {
  if (!c || !g) return MCX_EINVAL;
  if (g->nx < 1 || g->ny < 1 || g->nx > 4095 || g->ny > 4095 || !(g->pitch > 0.0) ||
      !std::isfinite(g->pitch) || !std::isfinite(g->x0) || !std::isfinite(g->y0))
    return fail(c, MCX_EINVAL, "lattice size or pitch");
  if (g->n_univ < 1 || g->max_rings < 1 || g->max_rings > 254 || !g->n_rings || !g->radii ||
      !g->mats || !g->pin_map)
    return fail(c, MCX_EINVAL, "universe description");
  for (int k = 0; k < 4; ++k)
    if (g->bc[k] != MCX_VACUUM && g->bc[k] != MCX_REFLECT) return fail(c, MCX_EINVAL, "bc");
  const int mr1 = g->max_rings + 1;
  for (int k = 0; k < g->nx * g->ny; ++k)
    if (g->pin_map[k] < 0 || g->pin_map[k] >= g->n_univ) return fail(c, MCX_EINVAL, "pin map");
  for (int u = 0; u < g->n_univ; ++u) {
    const int nr = g->n_rings[u];
    if (nr < 0 || nr > g->max_rings) return fail(c, MCX_EINVAL, "ring count");
    double prev = 0.0;
    for (int k = 0; k < nr; ++k) {
      const double r = g->radii[u * g->max_rings + k];
      if (!(r > prev) || !(r < 0.5 * g->pitch)) return fail(c, MCX_EINVAL, "ring radius");
      prev = r;
    }
    for (int k = 0; k <= nr; ++k)
      if (g->mats[u * mr1 + k] < 0) return fail(c, MCX_EINVAL, "ring material");
  }
  if (c->batch) {  // a single problem replaces the batch: its tables go too
    c->has_xs = false;
    c->batch = false;
  }
  c->nx = g->nx;
  c->ny = g->ny;
  c->pitch = g->pitch;
  c->x0 = g->x0;
  c->y0 = g->y0;
  for (int k = 0; k < 4; ++k) c->bc[k] = g->bc[k];
  c->n_univ = g->n_univ;
  c->max_rings = g->max_rings;
  c->n_rings.assign(g->n_rings, g->n_rings + g->n_univ);
  c->radii.assign(g->radii, g->radii + (size_t)g->n_univ * g->max_rings);
  c->mats.assign(g->mats, g->mats + (size_t)g->n_univ * mr1);
  c->pin_map.assign(g->pin_map, g->pin_map + (size_t)g->nx * g->ny);
  c->has_geo = true;
  c->batch = false;
  c->bound = false;
  return MCX_OK;
}

int mcx_load_mg_xs(mcx_ctx* c, int32_t n_mat, int32_t n_grp, const double* sig_t,
                   const double* sig_s, const double* nu_sig_f, const double* chi) {
  if (!c || !sig_t || !sig_s || !nu_sig_f || !chi) return MCX_EINVAL;
  if (n_mat < 1 || n_grp < 1 || n_grp > 65535) return fail(c, MCX_EINVAL, "xs sizes");
  const size_t MG = (size_t)n_mat * n_grp;
  std::vector<double> sst(MG), cum_s(MG * n_grp), cum_chi(MG);
  std::vector<int> last_s(MG), last_chi(n_mat), fis(n_mat, 0);
  for (int m = 0; m < n_mat; ++m) {
    double cchi = 0.0;
    int lc = n_grp - 1;
    bool found_c = false;
    for (int g = 0; g < n_grp; ++g) {
      const size_t mg = (size_t)m * n_grp + g;
      if (!(sig_t[mg] > 0.0) || !std::isfinite(sig_t[mg]))
        return fail(c, MCX_EINVAL, "sig_t must be positive");
      if (!(nu_sig_f[mg] >= 0.0) || !std::isfinite(nu_sig_f[mg]) || !(chi[mg] >= 0.0))
        return fail(c, MCX_EINVAL, "nu_sig_f and chi must be nonnegative");
      if (nu_sig_f[mg] > 0.0) fis[m] = 1;
      double run = 0.0;
      int ls = n_grp - 1;
      bool found_s = false;
      for (int h = 0; h < n_grp; ++h) {
        const double v = sig_s[mg * n_grp + h];
        if (!(v >= 0.0) || !std::isfinite(v)) return fail(c, MCX_EINVAL, "sig_s must be >= 0");
        run += v;
        cum_s[mg * n_grp + h] = run;
        if (v > 0.0) {
          ls = h;
          found_s = true;
        }
      }
      (void)found_s;
      sst[mg] = run;
      last_s[mg] = ls;
      if (run > sig_t[mg]) return fail(c, MCX_EINVAL, "scattering exceeds sig_t");
      cchi += chi[mg];
      cum_chi[mg] = cchi;
      if (chi[mg] > 0.0) {
        lc = g;
        found_c = true;
      }
    }
    last_chi[m] = lc;
    if (fis[m]) {
      if (!found_c || std::fabs(cchi - 1.0) > 1e-6)
        return fail(c, MCX_EINVAL, "fission spectrum of a fissile material must sum to 1");
      for (int g = 0; g < n_grp; ++g) {
        const size_t mg = (size_t)m * n_grp + g;
        if (nu_sig_f[mg] > 0.0 && !(sig_t[mg] - sst[mg] > 0.0))
          return fail(c, MCX_EINVAL, "fissile group without absorption");
      }
    }
  }
  // binary32 tables: values rounded once, running sums accumulated in binary32
  std::vector<float> sig_t_f(MG), nusf_f(MG), sst_f(MG), cum_s_f(MG * n_grp), cum_chi_f(MG);
  for (int m = 0; m < n_mat; ++m) {
    float cchi = 0.0f;
    for (int g = 0; g < n_grp; ++g) {
      const size_t mg = (size_t)m * n_grp + g;
      sig_t_f[mg] = (float)sig_t[mg];
      nusf_f[mg] = (float)nu_sig_f[mg];
      float run = 0.0f;
      for (int h = 0; h < n_grp; ++h) {
        run += (float)sig_s[mg * n_grp + h];
        cum_s_f[mg * n_grp + h] = run;
      }
      // a valid row (sum of sig_s <= sig_t in binary64) can round above
      // binary32 sig_t when scattering is (nearly) the whole cross section:
      // clamp the running sums there, so the scatter probability is 1
      if (run > sig_t_f[mg]) {
        run = sig_t_f[mg];
        for (int h = 0; h < n_grp; ++h)
          cum_s_f[mg * n_grp + h] = std::min(cum_s_f[mg * n_grp + h], run);
      }
      sst_f[mg] = run;
      cchi += (float)chi[mg];
      cum_chi_f[mg] = cchi;
    }
  }
  if (c->batch) {  // a single problem replaces the batch: its lattices go too
    c->has_geo = false;
    c->batch = false;
  }
  c->sig_t_f = std::move(sig_t_f);
  c->nusf_f = std::move(nusf_f);
  c->sst_f = std::move(sst_f);
  c->cum_s_f = std::move(cum_s_f);
  c->cum_chi_f = std::move(cum_chi_f);
  c->n_mat = n_mat;
  c->G = n_grp;
  c->sig_t.assign(sig_t, sig_t + MG);
  c->nusf.assign(nu_sig_f, nu_sig_f + MG);
  c->sst = std::move(sst);
  c->cum_s = std::move(cum_s);
  c->cum_chi = std::move(cum_chi);
  c->last_s = std::move(last_s);
  c->last_chi = std::move(last_chi);
  c->fissile = std::move(fis);
  c->has_xs = true;
  c->ce = false;
  c->bound = false;
  return MCX_OK;
}

int mcx_load_ce_xs(mcx_ctx* c, const mcx_ce_data* d) {
  if (!c || !d) return MCX_EINVAL;
  if (d->n_nuc < 1 || d->n_pts < 2 || d->n_mat < 1 || d->max_nuc < 1 || d->n_ebins < 1 ||
      (int64_t)d->n_nuc * d->n_pts > (int64_t(1) << 28) ||
      (int64_t)d->n_mat * d->max_nuc * d->n_pts > (int64_t(1) << 28) || !d->e_grid || !d->sig_t ||
      !d->sig_s || !d->sig_f || !d->awr || !d->mat_n || !d->mat_nuc || !d->mat_dens ||
      !d->e_edges)
    return fail(c, MCX_EINVAL, "continuous-energy sizes");
  if (!(d->nu >= 0.0) || !std::isfinite(d->nu) || !(d->watt_a > 0.0) || !(d->watt_b >= 0.0) ||
      !(d->e_max > 0.0) || !(d->e_cut >= 0.0) || !std::isfinite(d->e_max) ||
      !(d->src_energy >= 0.0) || !std::isfinite(d->src_energy))
    return fail(c, MCX_EINVAL, "continuous-energy constants");
  for (int k = 0; k + 1 < d->n_pts; ++k)
    if (!(d->e_grid[k] < d->e_grid[k + 1]) || !std::isfinite(d->e_grid[k + 1]) ||
        !(d->e_grid[0] > 0.0))
      return fail(c, MCX_EINVAL, "energy grid must increase");
  for (int k = 0; k < d->n_ebins; ++k)
    if (!(d->e_edges[k] < d->e_edges[k + 1])) return fail(c, MCX_EINVAL, "tally edges must increase");
  const size_t NP = (size_t)d->n_nuc * d->n_pts;
  for (size_t k = 0; k < NP; ++k)
    if (!(d->sig_s[k] >= 0.0) || !(d->sig_f[k] >= 0.0) || !(d->sig_t[k] >= d->sig_s[k]) ||
        !std::isfinite(d->sig_t[k]))
      return fail(c, MCX_EINVAL, "pointwise cross sections (need 0 <= sig_s <= sig_t, sig_f >= 0)");
  for (int n = 0; n < d->n_nuc; ++n)
    if (!(d->awr[n] > 0.0) || !std::isfinite(d->awr[n])) return fail(c, MCX_EINVAL, "target mass");
  std::vector<int> fis(d->n_mat, 0);
  double sigt_min = 1e300;
  for (int m = 0; m < d->n_mat; ++m) {
    if (d->mat_n[m] < 1 || d->mat_n[m] > d->max_nuc) return fail(c, MCX_EINVAL, "material size");
    for (int k = 0; k < d->mat_n[m]; ++k) {
      const int n = d->mat_nuc[m * d->max_nuc + k];
      const double dens = d->mat_dens[m * d->max_nuc + k];
      if (n < 0 || n >= d->n_nuc || !(dens >= 0.0) || !std::isfinite(dens))
        return fail(c, MCX_EINVAL, "material nuclide or density");
      if (dens > 0.0 && d->nu > 0.0)
        for (int q = 0; q < d->n_pts; ++q)
          if (d->sig_f[(size_t)n * d->n_pts + q] > 0.0) {
            fis[m] = 1;
            break;
          }
    }
    // the macroscopic total is piecewise linear in energy: its minimum is at
    // a grid point
    for (int q = 0; q < d->n_pts; ++q) {
      double st = 0.0;
      for (int k = 0; k < d->mat_n[m]; ++k)
        st += d->mat_dens[m * d->max_nuc + k] *
              d->sig_t[(size_t)d->mat_nuc[m * d->max_nuc + k] * d->n_pts + q];
      sigt_min = std::min(sigt_min, st);
    }
  }
  if (!(sigt_min > 0.0)) return fail(c, MCX_EINVAL, "a material has zero total cross section");
  // (t, f, s, 0) of each nuclide of each material, packed by material, then
  // grid point, then the material's nuclides: a lookup reads one interval
  // of one material, which is one contiguous block of 2 * max_nuc * 32 bytes
  // (a layout by nuclide spreads it over one 64-byte piece per nuclide), and
  // a flight, which needs t and f only, one 16-byte load per nuclide and point
  const size_t MX = (size_t)d->max_nuc;
  std::vector<double> xs((size_t)d->n_mat * d->n_pts * MX * 4, 0.0);
  for (int m = 0; m < d->n_mat; ++m)
    for (int q = 0; q < d->n_pts; ++q)
      for (int k = 0; k < d->mat_n[m]; ++k) {
        const size_t src = (size_t)d->mat_nuc[m * d->max_nuc + k] * d->n_pts + q;
        double* e = &xs[(((size_t)m * d->n_pts + q) * MX + k) * 4];
        e[0] = d->sig_t[src];
        e[1] = d->sig_f[src];
        e[2] = d->sig_s[src];
      }
  if (c->batch) {
    c->has_geo = false;
    c->batch = false;
  }
  // the device holds the table as (t, f) pairs, which every lookup reads,
  // and s alone, which a collision needs for one nuclide (and an absorption
  // for all): less to cache than whole (t, f, s) entries
  std::vector<double> tf(xs.size() / 2), sv(xs.size() / 4);
  for (size_t e = 0; e < xs.size() / 4; ++e) {
    tf[2 * e] = xs[4 * e];
    tf[2 * e + 1] = xs[4 * e + 1];
    sv[e] = xs[4 * e + 2];
  }
  c->ce_tf = std::move(tf);
  c->ce_s = std::move(sv);
  c->ce_xs = std::move(xs);
  c->ce_grid.assign(d->e_grid, d->e_grid + d->n_pts);
  c->ce_awr.assign(d->awr, d->awr + d->n_nuc);
  c->ce_mat_n.assign(d->mat_n, d->mat_n + d->n_mat);
  c->ce_mat_nuc.assign(d->mat_nuc, d->mat_nuc + (size_t)d->n_mat * d->max_nuc);
  c->ce_dens.assign(d->mat_dens, d->mat_dens + (size_t)d->n_mat * d->max_nuc);
  c->ce_edges.assign(d->e_edges, d->e_edges + d->n_ebins + 1);
  c->ce_n_nuc = d->n_nuc;
  c->ce_n_pts = d->n_pts;
  c->ce_max_nuc = d->max_nuc;
  c->ce_n_ebins = d->n_ebins;
  c->ce_nu = d->nu;
  c->ce_watt_a = d->watt_a;
  c->ce_watt_b = d->watt_b;
  c->ce_e_max = d->e_max;
  c->ce_e_cut = d->e_cut;
  c->ce_src_energy = d->src_energy;
  c->ce_sigt_min = sigt_min;
  build_hash<double, uint64_t>(c->ce_grid, &c->ce_hash, &c->ce_hash_shift, &c->ce_hash_base);
  {
    std::vector<float> gf(c->ce_grid.size());
    for (size_t k = 0; k < gf.size(); ++k) gf[k] = (float)c->ce_grid[k];
    bool inc = true;
    for (size_t k = 1; k < gf.size(); ++k) inc = inc && gf[k - 1] < gf[k] && gf[k - 1] > 0.0f;
    if (inc) {
      build_hash<float, uint32_t>(gf, &c->ce_hash_f, &c->ce_hash_shift_f, &c->ce_hash_base_f);
    } else {
      c->ce_hash_f.clear();
    }
  }
  c->fissile = std::move(fis);
  c->n_mat = d->n_mat;
  c->G = d->n_ebins;
  // the multigroup tables are not used
  c->sig_t.clear();
  c->nusf.clear();
  c->sst.clear();
  c->cum_s.clear();
  c->cum_chi.clear();
  c->last_s.clear();
  c->last_chi.clear();
  c->sig_t_f.clear();
  c->nusf_f.clear();
  c->sst_f.clear();
  c->cum_s_f.clear();
  c->cum_chi_f.clear();
  c->ce = true;
  c->has_xs = true;
  c->bound = false;
  return MCX_OK;
}

int mcx_load_time_grid(mcx_ctx* c, int32_t n_tbins, const double* t_edges, const double* speed,
                       int32_t n_grp) {
  if (!c) return MCX_EINVAL;
  c->bound = false;
  if (n_tbins == 0) {
    c->t_edges.clear();
    c->t_speed.clear();
    return MCX_OK;
  }
  // multigroup: one speed per group; continuous energy: no speeds (NULL, 0)
  if (n_tbins < 0 || n_tbins > 4096 || !t_edges || (speed && (n_grp < 1 || n_grp > 65535)) ||
      (!speed && n_grp != 0))
    return fail(c, MCX_EINVAL, "time grid sizes");
  if (!(t_edges[0] == 0.0)) return fail(c, MCX_EINVAL, "the time grid starts at 0");
  for (int k = 0; k < n_tbins; ++k)
    if (!(t_edges[k] < t_edges[k + 1]) || !std::isfinite(t_edges[k + 1]))
      return fail(c, MCX_EINVAL, "time edges must increase");
  for (int g = 0; g < n_grp; ++g)
    if (!(speed[g] > 0.0) || !std::isfinite(speed[g]))
      return fail(c, MCX_EINVAL, "group speeds must be positive");
  c->t_edges.assign(t_edges, t_edges + n_tbins + 1);
  if (speed)
    c->t_speed.assign(speed, speed + n_grp);
  else
    c->t_speed.clear();
  return MCX_OK;
}

int mcx_seed_source(mcx_ctx* c, const mcx_source* s) {
  if (!c || !s) return MCX_EINVAL;
  if (s->n_per_gen < 1 || s->n_per_gen > (int64_t(1) << 30))
    return fail(c, MCX_EINVAL, "n_per_gen out of range");
  if (s->ent_nx < 1 || s->ent_ny < 1 || (int64_t)s->ent_nx * s->ent_ny > (1 << 20))
    return fail(c, MCX_EINVAL, "entropy mesh");
  c->src = *s;
  c->has_src = true;
  c->bound = false;
  return MCX_OK;
}

// Carve the workspace (base == nullptr only measures it).
static size_t carve(const mcx_ctx* c, Dev& d, char* base, int n_gen_max) {
  Carver cv(base);
  const bool batch = c->batch;
  const size_t N = batch ? 0 : (size_t)c->src.n_per_gen;
  const int mr1 = c->max_rings + 1;
  const size_t MG = (size_t)c->n_mat * c->G;
  const int nt = c->t_edges.empty() ? 1 : (int)c->t_edges.size() - 1;
  const int nb = batch ? c->batch_bins : c->nx * c->ny * mr1 * c->G * nt;
  const uint64_t n_hist = batch ? c->batch_hist : (uint64_t)N;
  const bool async = c->opt.engine == MCX_ENGINE_ASYNC;
  // per-history outputs: the persistent and asynchronous engines
  const bool persistent = batch || c->opt.engine == MCX_ENGINE_PERSISTENT || async;
  // copies of the flux accumulators, spread over workgroups by index (up to
  // 64 copies in 1 Mi words; a batch's workgroups all work on the few
  // problems whose histories are in flight, so its few bins get every copy,
  // in up to 16 Mi words)
  const int stripe_words = batch ? (1 << 24) : (1 << 20);
  const int stripes = std::max(1, std::min(STRIPES, stripe_words / std::max(1, 2 * nb)));
  const uint32_t fis_cap = (uint32_t)std::min<size_t>(2 * N + 4096, 0xFFFFFFF0u);
  const size_t n_ent = (size_t)c->src.ent_nx * c->src.ent_ny;
  const size_t n_cnt_slots = (size_t)c->opt.max_events + 4;

  Tables& T = d.T;
  T.geo.pin_map = cv.take<int>(c->pin_map.size());
  T.geo.n_rings = cv.take<int>(c->n_rings.size());
  T.geo.radii = cv.take<double>(c->radii.size());
  T.geo.mats = cv.take<int>(c->mats.size());
  (void)MG;
  T.sig_t = cv.take<double>(c->sig_t.size());
  T.nusf = cv.take<double>(c->nusf.size());
  T.sst = cv.take<double>(c->sst.size());
  T.cum_s = cv.take<double>(c->cum_s.size());
  T.last_s = cv.take<int>(c->last_s.size());
  T.cum_chi = cv.take<double>(c->cum_chi.size());
  T.last_chi = cv.take<int>(c->last_chi.size());
  T.fissile = cv.take<int>(c->n_mat);
  T.sig_t_f = cv.take<float>(c->sig_t_f.size());
  T.nusf_f = cv.take<float>(c->nusf_f.size());
  T.sst_f = cv.take<float>(c->sst_f.size());
  T.cum_s_f = cv.take<float>(c->cum_s_f.size());
  T.cum_chi_f = cv.take<float>(c->cum_chi_f.size());
  const bool ce = c->ce;
  T.ce = ce ? 1 : 0;
  T.e_grid = cv.take<double>(c->ce_grid.size());
  T.ce_tf = cv.take<double>(c->ce_tf.size());
  T.ce_s = cv.take<double>(c->ce_s.size());
  T.awr = cv.take<double>(c->ce_awr.size());
  T.mat_n = cv.take<int>(c->ce_mat_n.size());
  T.mat_nuc = cv.take<int>(c->ce_mat_nuc.size());
  T.mat_dens = cv.take<double>(c->ce_dens.size());
  T.e_edges = cv.take<double>(c->ce_edges.size());
  T.time = c->t_edges.empty() ? 0 : 1;
  T.nt = nt;
  T.t_edges = c->t_edges.empty() ? nullptr : cv.take<double>(c->t_edges.size());
  T.speed = c->t_edges.empty() ? nullptr : cv.take<double>(c->t_speed.size());
  T.t_max = c->t_edges.empty() ? 0.0 : c->t_edges.back();
  const bool fp32 = c->opt.precision == MCX_FP32_MIXED;
  const bool ce32 = ce && fp32;
  T.e_grid_f = cv.take<float>(ce32 ? c->ce_grid.size() : 0);
  T.ce_tf_f = cv.take<float>(ce32 ? c->ce_tf.size() : 0);
  T.ce_s_f = cv.take<float>(ce32 ? c->ce_s.size() : 0);
  T.awr_f = cv.take<float>(ce32 ? c->ce_awr.size() : 0);
  T.mat_dens_f = cv.take<float>(ce32 ? c->ce_dens.size() : 0);
  T.e_edges_f = cv.take<float>(ce32 ? c->ce_edges.size() : 0);
  T.e_hash = cv.take<int>(c->ce_hash.size());
  T.e_hash_f = cv.take<int>(ce32 ? c->ce_hash_f.size() : 0);
  for (int b = 0; b < 3; ++b) {
    Bank& k = d.bank[b];
    k.x = cv.take<double>(N);
    k.y = cv.take<double>(N);
    if (fp32) {
      k.u = cv.take<float>(N);
      k.v = cv.take<float>(N);
    } else {
      k.u = cv.take<double>(N);
      k.v = cv.take<double>(N);
    }
    k.cell = cv.take<uint32_t>(N);
    k.gs = cv.take<uint32_t>(N);
    k.ctr = cv.take<uint32_t>(N);
    k.id = cv.take<uint32_t>(N);
    k.nseg = cv.take<uint32_t>(N);
    k.t = c->t_edges.empty() ? nullptr : cv.take<double>(N);
    if (fp32) {
      k.w = cv.take<float>(ce ? N : 0);
      k.e = cv.take<float>(ce ? N : 0);
    } else {
      k.w = cv.take<double>(ce ? N : 0);
      k.e = cv.take<double>(ce ? N : 0);
    }
    const size_t nx = (ce && b == 2) ? N : 0;  // lookups handed to the collision kernel
    k.xgi = cv.take<int32_t>(nx);
    if (fp32) {
      k.xf = cv.take<float>(nx);
      k.xst = cv.take<float>(nx);
      k.xsf = cv.take<float>(nx);
    } else {
      k.xf = cv.take<double>(nx);
      k.xst = cv.take<double>(nx);
      k.xsf = cv.take<double>(nx);
    }
  }
  d.src_x = cv.take<double>(N);
  d.src_y = cv.take<double>(N);
  d.src_g = cv.take<int32_t>(N);
  d.src_e = ce ? cv.take<double>(N) : nullptr;
  Accum& A = d.A;
  A.fis.x = cv.take<double>(fis_cap);
  A.fis.y = cv.take<double>(fis_cap);
  A.fis.g = cv.take<int32_t>(fis_cap);
  A.fis.parent = cv.take<uint32_t>(fis_cap);
  A.fis.seq = cv.take<uint32_t>(fis_cap);
  A.fis.e = ce ? cv.take<double>(fis_cap) : nullptr;
  A.fis_cap = fis_cap;
  d.can_x = cv.take<double>(fis_cap);
  d.can_y = cv.take<double>(fis_cap);
  d.can_g = cv.take<int32_t>(fis_cap);
  d.can_e = ce ? cv.take<double>(fis_cap) : nullptr;
  const bool keig = !batch && !c->src.fixed_source;
  const size_t n_bk = keig ? bank_buckets(N) : 0;
  if (keig) {
    const size_t n_st = fis_cap;
    d.st.mg = ce ? nullptr : cv.take<StSite>(n_st);
    d.st.ce = ce ? cv.take<StSiteCE>(n_st) : nullptr;
  }
  A.nsite_id = cv.take<uint32_t>(std::max<size_t>(N, n_hist));
  if (persistent) {
    d.h_kcol = cv.take<unsigned long long>(2 * n_hist);
    d.h_kabs = cv.take<unsigned long long>(n_hist);
    d.h_cnt = cv.take<uint32_t>((size_t)7 * n_hist);
  }
  d.n_hist = n_hist;
  if (async) {
    AsyncBufs& B = d.ab;
    B.x = cv.take<double>(n_hist);
    B.y = cv.take<double>(n_hist);
    if (fp32) {
      B.u = cv.take<float>(n_hist);
      B.v = cv.take<float>(n_hist);
    } else {
      B.u = cv.take<double>(n_hist);
      B.v = cv.take<double>(n_hist);
    }
    B.cell = cv.take<uint32_t>(n_hist);
    B.gs = cv.take<uint32_t>(n_hist);
    B.ctr = cv.take<uint32_t>(n_hist);
    B.prob = cv.take<uint32_t>(n_hist);
    uint64_t cap = 64;
    while (cap < n_hist) cap <<= 1;
    B.mask = (uint32_t)(cap - 1);
    B.slot[0] = cv.take<uint32_t>(cap);
    B.slot[1] = cv.take<uint32_t>(cap);
    B.ctl = cv.take<unsigned long long>(ASYNC_CTL_WORDS);
  }
  if (batch) {
    d.probs = cv.take<ProbDesc>(c->n_probs);
    d.prob_kres = cv.take<double>((size_t)3 * c->n_probs);
    d.b_flux = cv.take<double>(nb);
    d.b_prod = cv.take<double>(nb);
  }
  d.offs = cv.take<uint32_t>(N);
  d.chunk_sum = cv.take<uint32_t>(scan_chunks((uint32_t)N) + 1);
  d.scan_total = cv.take<uint32_t>(1);
  d.gen_status = cv.take<uint32_t>((size_t)n_gen_max + 1);  // cleared in 8-byte words
  A.status = d.gen_status;
  d.cnt_live = cv.take<uint32_t>(n_cnt_slots);
  d.cnt_col = cv.take<uint32_t>(n_cnt_slots);
  // per-generation accumulators, zeroed together
  const size_t w_tally = (size_t)stripes * 2 * nb;
  const size_t w_tally_t = (size_t)stripes * 2 * nb;
  const size_t w_k = 3 * STRIPES * 2;
  const size_t w_cnt = (size_t)N_CNT_ALL * STRIPES;
  const size_t w_misc = 2 + (n_ent + 1) / 2 + (n_bk + 1) / 2;
  const size_t w_prob = batch ? (size_t)c->n_probs * (N_CNT + 4) : 0;
  // continuous-energy time-dependent mode: the density accumulators
  const size_t w_dens = (ce && !c->t_edges.empty()) ? w_tally + w_tally_t : 0;
  d.acc_words = w_tally + w_tally_t + w_k + w_cnt + w_prob + w_misc + w_dens;
  d.acc_base = cv.take<unsigned long long>(d.acc_words);
  if (base) {
    A.tally = d.acc_base;
    A.tally_t = A.tally + w_tally;
    A.k = A.tally_t + w_tally_t;
    A.cnt = A.k + w_k;
    unsigned long long* pw = A.cnt + w_cnt;
    if (batch) {
      d.prob_cnt = pw;
      d.prob_k = pw + (size_t)c->n_probs * N_CNT;
    }
    pw += w_prob;
    A.n_fis = reinterpret_cast<uint32_t*>(pw);
    d.work = reinterpret_cast<uint32_t*>(pw + 1);
    d.ent_hist = reinterpret_cast<uint32_t*>(pw + 2);
    d.bk_fill = n_bk ? reinterpret_cast<uint32_t*>(pw + 2 + (n_ent + 1) / 2) : nullptr;
    pw += w_misc;
    A.dens = w_dens ? pw : nullptr;
    A.dens_t = w_dens ? pw + w_tally : nullptr;
  }
  // results
  d.gen_k = cv.take<double>((size_t)3 * n_gen_max);
  d.gen_h = cv.take<double>(n_gen_max);
  d.gen_cnt = cv.take<unsigned long long>((size_t)N_CNT_ALL * n_gen_max);
  d.gen_m = cv.take<uint32_t>(n_gen_max);
  d.gen_tal = cv.take<double>((size_t)2 * nb * n_gen_max);
  d.tal_stat = cv.take<double>((size_t)4 * nb);
  d.tl_part = cv.take<double>((size_t)2 * std::max(1, gen_tally_blocks(nb)));
  d.k_stat = cv.take<double>(6);
  d.k_used = cv.take<double>(1);
  d.xi0 = cv.take<double>(1);
  A.k_used = d.k_used;
  // per-history records
  if (c->opt.record_histories) {
    Records& R = d.R;
    for (int pass = 0; pass < 2; ++pass) {
      // pass 0 measures the record block, pass 1 carves it
      Carver rc(pass ? reinterpret_cast<char*>(d.rec_base) : nullptr);
      R.n_seg = rc.take<int32_t>(N);
      R.n_col = rc.take<int32_t>(N);
      R.n_cross = rc.take<int32_t>(N);
      R.n_refl = rc.take<int32_t>(N);
      R.fate = rc.take<int32_t>(N);
      R.g_final = rc.take<int32_t>(N);
      R.ctr_final = rc.take<uint32_t>(N);
      R.tl_sum = rc.take<double>(N);
      R.kcol_sum = rc.take<double>(N);
      R.x_final = rc.take<double>(N);
      R.y_final = rc.take<double>(N);
      R.e_final = rc.take<double>(N);
      R.t_final = rc.take<double>(N);
      R.ev_cap = c->opt.event_log;
      R.ev = c->opt.event_log > 0 ? rc.take<EvEntry>(N * (size_t)c->opt.event_log) : nullptr;
      if (pass == 0) {
        d.rec_words = (rc.off + 7) / 8;
        d.rec_base = cv.take<unsigned long long>(d.rec_words);
        if (!base) break;
      }
    }
  } else {
    d.R = Records{};
    d.rec_base = nullptr;
    d.rec_words = 0;
  }
  d.N = (uint32_t)N;
  d.fis_cap = fis_cap;
  d.n_bins = nb;
  d.stripes = stripes;
  d.n_cnt_slots = n_cnt_slots;
  return cv.off + 256;
}

static bool loaded(const mcx_ctx* c) {
  return c->batch ? (c->has_geo && c->has_xs) : (c->has_geo && c->has_xs && c->has_src);
}

int mcx_workspace_size(mcx_ctx* c, int32_t n_gen_max, size_t* bytes) {
  if (!c || !bytes || n_gen_max < 1) return MCX_EINVAL;
  if (!loaded(c)) return fail(c, MCX_ESTATE, "load and seed first");
  Dev scratch;
  *bytes = carve(c, scratch, nullptr, n_gen_max);
  return MCX_OK;
}

int mcx_bind_workspace(mcx_ctx* c, void* ptr, size_t bytes, int32_t n_gen_max) {
  if (!c || !ptr || n_gen_max < 1) return MCX_EINVAL;
  c->bound = false;
  c->ran = false;
  c->can_continue = false;
  c->batch_ran = false;
  if (c->graph_exec) {
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  if (c->graph) {
    (void)hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
  if (!loaded(c)) return fail(c, MCX_ESTATE, "load and seed first");
  if ((uintptr_t)ptr % 256) return fail(c, MCX_EINVAL, "workspace must be 256-byte aligned");
  const bool launch_per_event =
      c->opt.engine == MCX_ENGINE_EVENT || c->opt.engine == MCX_ENGINE_MONOLITHIC;
  if (c->ce && !launch_per_event)
    return fail(c, MCX_EINVAL, "continuous energy runs on the event or monolithic engine");
  if (!c->t_edges.empty() &&
      (c->batch || !c->src.fixed_source || !launch_per_event ||
       (c->ce ? !c->t_speed.empty() : (int)c->t_speed.size() != c->G)))
    return fail(c, MCX_EINVAL,
                "the time-dependent mode runs fixed-source problems on the event or monolithic "
                "engine, with one speed per group (multigroup) or none (continuous energy)");
  if (c->ce && c->opt.precision == MCX_FP32_MIXED && c->ce_hash_f.empty())
    return fail(c, MCX_EINVAL, "the energy grid is not strictly increasing in binary32");
  // materials referenced by the geometry must exist (batches: checked per problem)
  if (!c->batch)
    for (int u = 0; u < c->n_univ; ++u)
      for (int k = 0; k <= c->n_rings[u]; ++k)
        if (c->mats[(size_t)u * (c->max_rings + 1) + k] >= c->n_mat)
          return fail(c, MCX_EINVAL, "geometry references a missing material");
  Dev scratch;
  const size_t need = carve(c, scratch, nullptr, n_gen_max);
  if (bytes < need) return fail(c, MCX_ENOMEM, "workspace too small");
  HIP_TRY(c, hipSetDevice(c->opt.device));
  c->ws = (char*)ptr;
  c->ws_bytes = bytes;
  c->n_gen_max = n_gen_max;
  carve(c, c->d, c->ws, n_gen_max);

  // fixed-point scales of the exact accumulators
  const double ln_max = 36.8;  // -ln of the smallest uniform draw, 2^-53
  double d_max = 0, kc_max = 0, ka_max = 0;
  for (size_t mg = 0; mg < c->sig_t.size(); ++mg) {
    const double d = ln_max / c->sig_t[mg];
    d_max = std::max(d_max, d);
    kc_max = std::max(kc_max, c->nusf[mg] / c->sig_t[mg]);
    if (c->nusf[mg] > 0.0) ka_max = std::max(ka_max, c->nusf[mg] / (c->sig_t[mg] - c->sst[mg]));
  }
  double ktl_max = 0.0;
  if (c->ce) {
    // nu Sigma_f <= nu Sigma_t and nu Sigma_f <= nu Sigma_a (sigma_t = sigma_s +
    // capture + fission pointwise), so every k term is at most nu and a
    // track-length term d nu Sigma_f at most ln_max nu
    d_max = ln_max / c->ce_sigt_min;
    kc_max = ka_max = c->ce_nu;
    ktl_max = ln_max * c->ce_nu;
  }
  Tables& T = c->d.T;
  T.geo.nx = c->nx;
  T.geo.ny = c->ny;
  T.n_univ = c->n_univ;
  T.geo.max_rings = c->max_rings;
  T.geo.mr1 = c->max_rings + 1;
  T.geo.pitch = c->pitch;
  T.geo.x0 = c->x0;
  T.geo.y0 = c->y0;
  T.geo.width = (double)c->nx * c->pitch;
  T.geo.height = (double)c->ny * c->pitch;
  for (int k = 0; k < 4; ++k) T.geo.bc[k] = c->bc[k];
  T.geo.bin_base = 0;
  T.probs = nullptr;
  T.n_probs = 0;
  T.n_hist_total = c->d.n_hist;
  T.n_mat = c->n_mat;
  T.G = c->G;
  T.seed = c->src.seed;
  T.prob = c->src.problem_id;
  T.fixed_source = c->src.fixed_source ? 1 : 0;
  T.ent_nx = c->src.ent_nx;
  T.ent_ny = c->src.ent_ny;
  std::vector<ProbDesc> pd;
  if (c->batch) {
    // each problem's lattice points into the concatenated tables
    pd.resize(c->n_probs);
    for (int p = 0; p < c->n_probs; ++p) {
      const mcx_ctx::BProb& b = c->bprobs[p];
      Geo& L = pd[p].geo;
      L.nx = b.nx;
      L.ny = b.ny;
      L.max_rings = b.max_rings;
      L.mr1 = b.max_rings + 1;
      L.pitch = b.pitch;
      L.x0 = b.x0;
      L.y0 = b.y0;
      L.width = (double)b.nx * b.pitch;
      L.height = (double)b.ny * b.pitch;
      for (int k = 0; k < 4; ++k) L.bc[k] = b.bc[k];
      L.pin_map = T.geo.pin_map + b.pin_base;
      L.n_rings = T.geo.n_rings + b.univ_base;
      L.radii = T.geo.radii + b.radii_base;
      L.mats = T.geo.mats + b.mats_base;
      L.bin_base = b.bin_base;
      pd[p].seed = b.seed;
      pd[p].prob = b.prob;
      pd[p].hist_base = b.hist_base;
      pd[p].n_hist = b.n_hist;
      pd[p].n_bins = b.n_bins;
    }
    const Geo first = pd[0].geo;
    T.geo = first;
    T.probs = c->d.probs;
    T.n_probs = c->n_probs;
    T.seed = 0;
    T.prob = 0;
    T.fixed_source = 1;
    T.ent_nx = T.ent_ny = 0;
  }
  T.n_bins = c->d.n_bins;
  T.tally_stripes = c->d.stripes;
  // binary32 terms can exceed the binary64 bound by a few ulp: 1% headroom
  d_max *= 1.01;
  kc_max *= 1.01;
  ka_max *= 1.01;
  T.q_flux = fixed_point_scale(d_max);
  T.q_kcol = fixed_point_scale(kc_max);
  T.q_kabs = fixed_point_scale(ka_max);
  T.q_ktl = fixed_point_scale(ktl_max * 1.01);
  // a density term is the time spent in one time bin, at most the census time
  T.q_dens = fixed_point_scale(c->t_edges.empty() ? 1.0 : c->t_edges.back() * 1.01);
  T.src_energy = c->ce_src_energy;
  T.max_events = c->opt.max_events;
  T.n_pts = c->ce_n_pts;
  T.max_nuc = c->ce_max_nuc;
  T.n_ebins = c->ce_n_ebins;
  T.nu = c->ce_nu;
  T.watt_a = c->ce_watt_a;
  T.watt_b = c->ce_watt_b;
  T.e_max = c->ce_e_max;
  T.e_cut = c->ce_e_cut;
  T.n_hash = c->ce_hash.empty() ? 0 : (int)c->ce_hash.size() - 1;
  T.hash_shift = c->ce_hash_shift;
  T.hash_base = c->ce_hash_base;
  T.n_hash_f = c->ce_hash_f.empty() ? 0 : (int)c->ce_hash_f.size() - 1;
  T.hash_shift_f = c->ce_hash_shift_f;
  T.hash_base_f = c->ce_hash_base_f;

  hipStream_t s = c->stream;
  auto up = [&](const void* dst, const void* srcp, size_t n) {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(const_cast<void*>(dst), srcp, n, hipMemcpyHostToDevice, s);
  };
  HIP_TRY(c, up(T.geo.pin_map, c->pin_map.data(), c->pin_map.size() * sizeof(int)));
  HIP_TRY(c, up(T.geo.n_rings, c->n_rings.data(), c->n_rings.size() * sizeof(int)));
  HIP_TRY(c, up(T.geo.radii, c->radii.data(), c->radii.size() * sizeof(double)));
  HIP_TRY(c, up(T.geo.mats, c->mats.data(), c->mats.size() * sizeof(int)));
  HIP_TRY(c, up(T.sig_t, c->sig_t.data(), c->sig_t.size() * sizeof(double)));
  HIP_TRY(c, up(T.nusf, c->nusf.data(), c->nusf.size() * sizeof(double)));
  HIP_TRY(c, up(T.sst, c->sst.data(), c->sst.size() * sizeof(double)));
  HIP_TRY(c, up(T.cum_s, c->cum_s.data(), c->cum_s.size() * sizeof(double)));
  HIP_TRY(c, up(T.last_s, c->last_s.data(), c->last_s.size() * sizeof(int)));
  HIP_TRY(c, up(T.cum_chi, c->cum_chi.data(), c->cum_chi.size() * sizeof(double)));
  HIP_TRY(c, up(T.last_chi, c->last_chi.data(), c->last_chi.size() * sizeof(int)));
  HIP_TRY(c, up(T.fissile, c->fissile.data(), c->fissile.size() * sizeof(int)));
  HIP_TRY(c, up(T.sig_t_f, c->sig_t_f.data(), c->sig_t_f.size() * sizeof(float)));
  HIP_TRY(c, up(T.nusf_f, c->nusf_f.data(), c->nusf_f.size() * sizeof(float)));
  HIP_TRY(c, up(T.sst_f, c->sst_f.data(), c->sst_f.size() * sizeof(float)));
  HIP_TRY(c, up(T.cum_s_f, c->cum_s_f.data(), c->cum_s_f.size() * sizeof(float)));
  HIP_TRY(c, up(T.cum_chi_f, c->cum_chi_f.data(), c->cum_chi_f.size() * sizeof(float)));
  if (c->batch) HIP_TRY(c, up(c->d.probs, pd.data(), pd.size() * sizeof(ProbDesc)));
  if (T.t_edges) {
    HIP_TRY(c, up(T.t_edges, c->t_edges.data(), c->t_edges.size() * sizeof(double)));
    HIP_TRY(c, up(T.speed, c->t_speed.data(), c->t_speed.size() * sizeof(double)));
  }
  if (c->ce) {
    HIP_TRY(c, up(T.e_grid, c->ce_grid.data(), c->ce_grid.size() * sizeof(double)));
    HIP_TRY(c, up(T.ce_tf, c->ce_tf.data(), c->ce_tf.size() * sizeof(double)));
    HIP_TRY(c, up(T.ce_s, c->ce_s.data(), c->ce_s.size() * sizeof(double)));
    HIP_TRY(c, up(T.awr, c->ce_awr.data(), c->ce_awr.size() * sizeof(double)));
    HIP_TRY(c, up(T.mat_n, c->ce_mat_n.data(), c->ce_mat_n.size() * sizeof(int)));
    HIP_TRY(c, up(T.mat_nuc, c->ce_mat_nuc.data(), c->ce_mat_nuc.size() * sizeof(int)));
    HIP_TRY(c, up(T.mat_dens, c->ce_dens.data(), c->ce_dens.size() * sizeof(double)));
    HIP_TRY(c, up(T.e_edges, c->ce_edges.data(), c->ce_edges.size() * sizeof(double)));
    HIP_TRY(c, up(T.e_hash, c->ce_hash.data(), c->ce_hash.size() * sizeof(int)));
    if (c->opt.precision == MCX_FP32_MIXED) {
      HIP_TRY(c, up(T.e_hash_f, c->ce_hash_f.data(), c->ce_hash_f.size() * sizeof(int)));
      // binary32 copies, each value rounded once
      auto to_f = [](const std::vector<double>& v) {
        std::vector<float> f(v.size());
        for (size_t k = 0; k < v.size(); ++k) f[k] = (float)v[k];
        return f;
      };
      c->ce_f32[0] = to_f(c->ce_grid);
      c->ce_f32[1] = to_f(c->ce_tf);
      c->ce_f32[2] = to_f(c->ce_awr);
      c->ce_f32[3] = to_f(c->ce_dens);
      c->ce_f32[4] = to_f(c->ce_edges);
      c->ce_f32[5] = to_f(c->ce_s);
      const float* dst[6] = {T.e_grid_f, T.ce_tf_f, T.awr_f, T.mat_dens_f, T.e_edges_f,
                             T.ce_s_f};
      for (int k = 0; k < 6; ++k)
        HIP_TRY(c, up(dst[k], c->ce_f32[k].data(), c->ce_f32[k].size() * sizeof(float)));
    }
  }
  const double one = 1.0;
  HIP_TRY(c, up(c->d.k_used, &one, sizeof(double)));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->bound = true;
  c->ran = false;
  return MCX_OK;
}

// Enqueue a timing event pair around a launch when kernel timing is on.
static hipError_t time_mark(mcx_ctx* c, int kind, bool begin) {
  if (!c->opt.time_kernels || (c->opt.time_kernels == 2 && kind != 0) || !c->time_gen)
    return hipSuccess;
  if (begin) c->ev_kind.push_back(kind);
  const size_t k = (c->ev_kind.size() - 1) * 2 + (begin ? 0 : 1);
  while (c->ev_pool.size() <= k) {
    hipEvent_t e;
    // device-scope release: a timing mark must not flush caches to the
    // system between two kernels (the default system-scope release does)
    hipError_t r = hipEventCreateWithFlags(&e, hipEventReleaseToDevice);
    if (r != hipSuccess) return r;
    c->ev_pool.push_back(e);
  }
  return hipEventRecord(c->ev_pool[k], c->stream);
}

static int collect_kernel_times(mcx_ctx* c) {
  for (size_t p = 0; p < c->ev_kind.size(); ++p) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_pool[2 * p], c->ev_pool[2 * p + 1]));
    if (c->ev_kind[p] == 0) {
      c->timing.advance_ms += ms;
      c->timing.n_advance += 1;
    } else if (c->ev_kind[p] == 1) {
      c->timing.collide_ms += ms;
      c->timing.n_collide += 1;
    } else if (c->ev_kind[p] == 2) {
      c->timing.tail_ms += ms;
    } else {
      c->timing.persistent_ms += ms;
      c->timing.n_persistent += 1;
    }
  }
  c->ev_kind.clear();
  return MCX_OK;
}

static int generation_end(mcx_ctx* c, int gen);

static int run_generation(mcx_ctx* c, int gen) {
  c->time_gen = c->opt.time_stride <= 1 || gen % c->opt.time_stride == 0;
  hipStream_t s = c->stream;
  const Tables& T = c->d.T;
  Accum& A = c->d.A;
  const bool rec = c->opt.record_histories != 0;
  const uint32_t N = c->d.N;
  A.status = c->d.gen_status + gen;
  HIP_TRY(c, launch_fill_u64(c->d.acc_base, c->d.acc_words, 0ull, s));
  HIP_TRY(c, launch_fill_u64(reinterpret_cast<unsigned long long*>(A.nsite_id), (N + 1) / 2,
                             0ull, s));
  if (rec) HIP_TRY(c, launch_fill_u64(c->d.rec_base, c->d.rec_words, 0ull, s));
  const int prec = c->opt.precision == MCX_FP32_MIXED ? 1 : 0;
  if (c->opt.engine == MCX_ENGINE_PERSISTENT) {
    // one launch per generation; a fixed source is sampled inside it
    const bool keig = !T.fixed_source;
    if (gen == 0 && keig)
      HIP_TRY(c, launch_source(T, gen, N, c->d.src_x, c->d.src_y, c->d.src_g, A.status, s));
    HIP_TRY(c, time_mark(c, 3, true));
    HIP_TRY(c, launch_persistent(prec, c->pcfg, T, gen, A, c->d.h_kcol, c->d.h_kabs, c->d.h_cnt,
                                 c->d.work, keig ? c->d.src_x : nullptr,
                                 keig ? c->d.src_y : nullptr, keig ? c->d.src_g : nullptr,
                                 gen > 0 ? c->d.gen_status + gen - 1 : nullptr, s));
    HIP_TRY(c, time_mark(c, 3, false));
    HIP_TRY(c, launch_hist_reduce(T, 1, c->d.h_kcol, c->d.h_kabs, c->d.h_cnt, A, nullptr, nullptr,
                                  s));
    return generation_end(c, gen);
  }
  if (c->opt.engine == MCX_ENGINE_ASYNC) {
    // one launch per generation; workgroups pull from the global queues
    const bool keig = !T.fixed_source;
    if (gen == 0 && keig)
      HIP_TRY(c, launch_source(T, gen, N, c->d.src_x, c->d.src_y, c->d.src_g, A.status, s));
    HIP_TRY(c, launch_async_init(c->d.ab, c->d.n_hist, s));
    HIP_TRY(c, time_mark(c, 3, true));
    HIP_TRY(c, launch_async(prec, c->pcfg.grid, T, gen, A, c->d.h_kcol, c->d.h_kabs, c->d.h_cnt,
                            c->d.ab, (uint32_t)c->opt.flights, ASYNC_SPIN_LIMIT,
                            keig ? c->d.src_x : nullptr, keig ? c->d.src_y : nullptr,
                            keig ? c->d.src_g : nullptr,
                            gen > 0 ? c->d.gen_status + gen - 1 : nullptr, s));
    HIP_TRY(c, time_mark(c, 3, false));
    HIP_TRY(c, launch_async_status(c->d.ab, A.status, s));
    HIP_TRY(c, launch_hist_reduce(T, 1, c->d.h_kcol, c->d.h_kabs, c->d.h_cnt, A, nullptr, nullptr,
                                  s));
    return generation_end(c, gen);
  }
  const bool ce = T.ce != 0;
  const uint32_t* prev_st = gen > 0 ? c->d.gen_status + gen - 1 : nullptr;
  if (ce) {
    if (gen == 0 || T.fixed_source)
      HIP_TRY(c, launch_ce_source(prec, T, gen, N, c->d.src_x, c->d.src_y, c->d.src_e, A.status, s));
    HIP_TRY(c, launch_ce_birth(prec, T, gen, N, c->d.src_x, c->d.src_y, c->d.src_e, c->d.bank[0],
                               c->d.cnt_live, c->d.cnt_col, prev_st, A.status, s));
  } else {
    if (gen == 0 || T.fixed_source)
      HIP_TRY(c, launch_source(T, gen, N, c->d.src_x, c->d.src_y, c->d.src_g, A.status, s));
    HIP_TRY(c, launch_birth(prec, T, gen, N, c->d.src_x, c->d.src_y, c->d.src_g, c->d.bank[0],
                            c->d.cnt_live, c->d.cnt_col, prev_st, A.status, s));
  }

  // event iterations; `bound` is the live count of iteration `known`, an
  // upper bound for every later iteration
  uint32_t bound = N;
  int64_t known = 0, it = 0;
  // live counts on their way to the host: (iteration, ring slot)
  std::deque<std::pair<int64_t, int>> pending;
  int64_t n_sent = 0;
  // the monolithic engine runs its one-segment kernel until every history
  // has ended (no history-based tail)
  const bool mono = c->opt.engine == MCX_ENGINE_MONOLITHIC;
  const int64_t tail = mono ? 0
                            : c->opt.tail_threshold != 0
                                  ? (int64_t)c->opt.tail_threshold
                                  : std::min<int64_t>(DEFAULT_TAIL_MAX,
                                                      std::max<int64_t>(DEFAULT_TAIL, (int64_t)N / 8));
  int cur = 0;
  // default block: 512 threads for the multigroup event kernels (the
  // collision kernel's bank reservations), 256 for the continuous-energy ones
  const int block = c->opt.block_size ? c->opt.block_size : ce ? DEFAULT_BLOCK_CE : DEFAULT_BLOCK;
  // the LDS-staged advance kernel: multigroup tables in LDS plus 16 B per
  // tally bin in one block's LDS; as many LT_BLOCK-thread blocks as are resident
  int lt_grid = 0;
  if (!ce && !mono && c->opt.lds_tally_min > 0) {
    const size_t lb = advance_lt_lds_bytes(prec, T);
    if (lb > 0 && lb <= c->lds_block_max)
      lt_grid = c->dev_cus * advance_lt_blocks_per_cu(prec, rec, LT_BLOCK, lb);
  }
  // the collision kernel walks its bank with as many blocks as are resident
  const int col_grid = ce || mono ? 0 : c->dev_cus * collide_blocks_per_cu(prec, rec, T, block);
  for (;;) {
    if (bound == 0) break;
    // every live particle makes at least one flight per iteration, so after
    // iteration max_events the guard has ended every history (the host's
    // count lags a few iterations behind the device)
    if (it > c->opt.max_events) break;
    if ((size_t)it + 3 >= c->d.n_cnt_slots) return fail(c, MCX_EDEVICE, "iteration slots exhausted");
    if (tail > 0 && bound <= (uint32_t)tail) {
      HIP_TRY(c, time_mark(c, 2, true));
      if (ce)
        HIP_TRY(c, launch_ce_tail(prec, rec, T, gen, c->d.bank[cur], c->d.cnt_live + it, A, c->d.R,
                                  bound, s));
      else
        HIP_TRY(c, launch_tail(prec, rec, T, gen, c->d.bank[cur], c->d.cnt_live + it, A, c->d.R,
                               bound, s));
      HIP_TRY(c, time_mark(c, 2, false));
      c->timing.n_tail_launches += 1;
      break;
    }
    if (mono) {
      HIP_TRY(c, time_mark(c, 0, true));
      if (ce)
        HIP_TRY(c, launch_ce_mono(prec, rec, T, gen, c->d.bank[cur], c->d.cnt_live + it,
                                  c->d.bank[1 - cur], c->d.cnt_live + it + 1, A, c->d.R,
                                  c->d.cnt_live + it + 2, bound, block, s));
      else
        HIP_TRY(c, launch_mono(prec, rec, T, gen, c->d.bank[cur], c->d.cnt_live + it,
                               c->d.bank[1 - cur], c->d.cnt_live + it + 1, A, c->d.R,
                               c->d.cnt_live + it + 2, bound, block, s));
      HIP_TRY(c, time_mark(c, 0, false));
    } else {
    HIP_TRY(c, time_mark(c, 0, true));
    const uint32_t fl = (uint32_t)c->opt.flights;
    if (ce)
      HIP_TRY(c, launch_ce_advance(prec, rec, T, gen, fl, c->d.bank[cur], c->d.cnt_live + it,
                                   c->d.bank[1 - cur], c->d.cnt_live + it + 1, c->d.bank[2],
                                   c->d.cnt_col + it, A, c->d.R, c->d.cnt_live + it + 2,
                                   c->d.cnt_col + it + 1, bound, block, s));
    else if (lt_grid > 0 && (int64_t)bound >= (int64_t)c->opt.lds_tally_min)
      HIP_TRY(c, launch_advance_lt(prec, rec, T, gen, (uint32_t)c->opt.lt_flights, c->d.bank[cur],
                                   c->d.cnt_live + it,
                                   c->d.bank[1 - cur], c->d.cnt_live + it + 1, c->d.bank[2],
                                   c->d.cnt_col + it, A, c->d.R, c->d.cnt_live + it + 2,
                                   c->d.cnt_col + it + 1, bound, LT_BLOCK, lt_grid, s));
    else if (c->opt.rounds > 1)
      HIP_TRY(c, launch_advance_refill(prec, rec, T, gen, fl, (uint32_t)c->opt.rounds,
                                       c->d.bank[cur], c->d.cnt_live + it, c->d.bank[1 - cur],
                                       c->d.cnt_live + it + 1, c->d.bank[2], c->d.cnt_col + it, A,
                                       c->d.R, c->d.cnt_live + it + 2, c->d.cnt_col + it + 1,
                                       bound, block, s));
    else
      HIP_TRY(c, launch_advance(prec, rec, T, gen, fl, c->d.bank[cur], c->d.cnt_live + it,
                                c->d.bank[1 - cur], c->d.cnt_live + it + 1, c->d.bank[2],
                                c->d.cnt_col + it, A, c->d.R, c->d.cnt_live + it + 2,
                                c->d.cnt_col + it + 1, bound, block, s));
    HIP_TRY(c, time_mark(c, 0, false));
    HIP_TRY(c, time_mark(c, 1, true));
    if (ce)
      HIP_TRY(c, launch_ce_collide(prec, rec, T, gen, c->d.bank[2], c->d.cnt_col + it,
                                   c->d.bank[1 - cur], c->d.cnt_live + it + 1, A, c->d.R, bound,
                                   block, s));
    else
      HIP_TRY(c, launch_collide(prec, rec, T, gen, c->d.bank[2], c->d.cnt_col + it,
                                c->d.bank[1 - cur], c->d.cnt_live + it + 1, A, c->d.R, bound,
                                block, col_grid, s));
    HIP_TRY(c, time_mark(c, 1, false));
    }
    cur = 1 - cur;
    ++it;
    c->timing.n_iterations += 1;
    // The count goes to the host every other iteration while the tail is far
    // (each copy and its event delay the next launch a few microseconds), and
    // every iteration near it.  Counts never grow within a generation, so an
    // older count is an upper bound for every later iteration.
    if (it % 2 == 0 || (tail > 0 && (int64_t)bound <= 2 * tail)) {
      const int slot = (int)(n_sent++ % RING);
      HIP_TRY(c, hipMemcpyAsync(&c->h_pin[slot], c->d.cnt_live + it, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, s));
      HIP_TRY(c, hipEventRecord(c->ev_ring[slot], s));
      pending.emplace_back(it, slot);
    }
    while (!pending.empty()) {
      hipEvent_t e = c->ev_ring[pending.front().second];
      hipError_t q = hipEventQuery(e);
      if (q == hipErrorNotReady && it - known >= c->opt.lookahead) {
        HIP_TRY(c, hipEventSynchronize(e));
        q = hipSuccess;
      }
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return hip_fail(c, q, "hipEventQuery");
      known = pending.front().first;
      bound = c->h_pin[pending.front().second];
      pending.pop_front();
    }
  }

  return generation_end(c, gen);
}

// Generation end: estimators, tallies, canonical bank, entropy, combing.
static int generation_end(mcx_ctx* c, int gen) {
  hipStream_t s = c->stream;
  const Tables& T = c->d.T;
  Accum& A = c->d.A;
  const bool rec = c->opt.record_histories != 0;
  const uint32_t N = c->d.N;
  HIP_TRY(c, launch_gen_tallies(T, gen, N, A, c->d.gen_tal, c->d.tl_part, s));
  HIP_TRY(c, launch_gen_totals(T, gen, N, A, c->d.tl_part, c->d.gen_k, c->d.gen_cnt, c->d.gen_m,
                               c->d.k_used, c->d.xi0, s));
  if (!T.fixed_source) {
    HIP_TRY(c, launch_scan(A.nsite_id, N, c->d.chunk_sum, c->d.offs, c->d.scan_total, s));
    HIP_TRY(c, launch_gen_check(T, A.n_fis, c->d.scan_total, A.status, s));
    // the canonical bank is kept for mcx_get_bank: written out in the run's
    // last generation only
    const bool keep = gen == c->run_last_gen;
    HIP_TRY(c, launch_bank_end(T, gen, A.fis, A.n_fis, c->d.offs, c->d.scan_total, N,
                               c->d.fis_cap, c->d.bk_fill, c->d.st, N, c->d.xi0, keep ? c->d.can_x : nullptr,
                               keep ? c->d.can_y : nullptr, keep ? c->d.can_g : nullptr,
                               keep ? c->d.can_e : nullptr, c->d.src_x, c->d.src_y, c->d.src_g,
                               c->d.src_e, c->d.ent_hist, c->d.gen_h, A.status, s));
  } else {
    HIP_TRY(c, launch_fill_u64(reinterpret_cast<unsigned long long*>(c->d.gen_h + gen), 1, 0ull, s));
  }
  // per-history records: copied back after every generation
  if (rec) {
    HIP_TRY(c, hipStreamSynchronize(s));
    std::vector<char> tmp((size_t)c->d.rec_words * 8);
    HIP_TRY(c, hipMemcpy(tmp.data(), c->d.rec_base, tmp.size(), hipMemcpyDeviceToHost));
    std::vector<uint32_t> ns(N);
    HIP_TRY(c, hipMemcpy(ns.data(), A.nsite_id, N * sizeof(uint32_t), hipMemcpyDeviceToHost));
    // the record arrays were carved in order from rec_base with 256-byte alignment
    Carver rc(tmp.data());
    int32_t* n_seg = rc.take<int32_t>(N);
    int32_t* n_col = rc.take<int32_t>(N);
    int32_t* n_cross = rc.take<int32_t>(N);
    int32_t* n_refl = rc.take<int32_t>(N);
    int32_t* fate = rc.take<int32_t>(N);
    int32_t* g_final = rc.take<int32_t>(N);
    uint32_t* ctr = rc.take<uint32_t>(N);
    double* tl = rc.take<double>(N);
    double* kc = rc.take<double>(N);
    double* xf = rc.take<double>(N);
    double* yf = rc.take<double>(N);
    double* ef = rc.take<double>(N);
    double* tf = rc.take<double>(N);
    mcx_record* out = c->h_rec.data() + (size_t)gen * N;
    for (uint32_t i = 0; i < N; ++i) {
      out[i] = mcx_record{n_seg[i], n_col[i], n_cross[i], n_refl[i], fate[i], (int32_t)ns[i],
                          g_final[i], ctr[i], tl[i], kc[i], xf[i], yf[i], ef[i], tf[i]};
    }
    if (c->opt.event_log > 0) {
      const size_t ne = (size_t)N * c->opt.event_log;
      EvEntry* ev = rc.take<EvEntry>(ne);
      static_assert(sizeof(EvEntry) == sizeof(mcx_event), "event layout");
      std::memcpy(c->h_ev.data() + (size_t)gen * ne, ev, ne * sizeof(EvEntry));
    }
  }
  return MCX_OK;
}

static int status_error(mcx_ctx* c, uint32_t st) {
  if (st & ST_SOURCE) return fail(c, MCX_ELOST, "source sampling found no fissile point");
  if (st & ST_OVERFLOW) return fail(c, MCX_EOVERFLOW, "fission bank overflow");
  if (st & ST_TALLY) return fail(c, MCX_EOVERFLOW, "2^32 or more flights in one generation");
  if (st & ST_ASYNC)
    return fail(c, MCX_EDEVICE, "the asynchronous engine gave up a wait past its bound");
  if (st & (ST_SITE_SEQ | ST_SCAN)) return fail(c, MCX_EDEVICE, "inconsistent fission bank");
  if (st & ST_EXTINCT) return fail(c, MCX_EEXTINCT, "fission bank is empty");
  return fail(c, MCX_EDEVICE, "generation skipped");
}

// Statistics over the completed generations [0, ng) and their host copies.
static int finish_results(mcx_ctx* c, int ng, int n_inactive) {
  hipStream_t s = c->stream;
  const int ni = std::min(n_inactive, ng - 1);
  HIP_TRY(c, launch_stats(2 * c->d.n_bins, ng, ni, c->d.gen_tal, c->d.tal_stat,
                          c->d.tal_stat + 2 * c->d.n_bins, c->d.gen_k, c->d.k_stat, s));
  c->h_gen_k.resize((size_t)3 * ng);
  c->h_gen_h.resize(ng);
  c->h_gen_cnt.resize((size_t)N_CNT_ALL * ng);
  c->h_gen_m.resize(ng);
  c->h_kstat.resize(6);
  HIP_TRY(c, hipMemcpyAsync(c->h_gen_k.data(), c->d.gen_k, c->h_gen_k.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_gen_h.data(), c->d.gen_h, c->h_gen_h.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_gen_cnt.data(), c->d.gen_cnt, c->h_gen_cnt.size() * 8,
                            hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_gen_m.data(), c->d.gen_m, c->h_gen_m.size() * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_kstat.data(), c->d.k_stat, 6 * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->last_n_gen = ng;
  c->last_n_inactive = ni;
  c->ran = true;
  return MCX_OK;
}

// Generations [g0, g1) of the power iteration (g0 = 0 starts it, g0 > 0
// continues from the source and k_used the previous generation left).
static int run_range(mcx_ctx* c, int g0, int g1, int n_inactive) {
  HIP_TRY(c, hipSetDevice(c->opt.device));
  hipStream_t s = c->stream;
  c->timing = mcx_timing{};
  c->ran = false;
  c->can_continue = false;
  c->req_n_inactive = n_inactive;
  if (c->opt.record_histories) c->h_rec.resize((size_t)g1 * c->d.N, mcx_record{});
  if (c->opt.event_log > 0) c->h_ev.resize((size_t)g1 * c->d.N * c->opt.event_log, mcx_event{});
  if (g0 == 0) {
    const double one = 1.0;
    HIP_TRY(c, hipMemcpyAsync(c->d.k_used, &one, sizeof(double), hipMemcpyHostToDevice, s));
  }
  // the status words of the earlier generations are zero (only a fully
  // successful run can be continued)
  HIP_TRY(c, launch_fill_u64(reinterpret_cast<unsigned long long*>(c->d.gen_status),
                             ((size_t)g1 + 1) / 2, 0ull, s));
  HIP_TRY(c, hipEventRecord(c->ev_start, s));
  // generations are enqueued back to back; each one's status is checked
  // once the run has finished (a failed generation makes the later ones run
  // empty)
  int rc = MCX_OK;
  c->run_last_gen = g1 - 1;
  for (int g = g0; g < g1; ++g) {
    rc = run_generation(c, g);
    if (rc != MCX_OK) break;
  }
  HIP_TRY(c, hipEventRecord(c->ev_stop, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (rc != MCX_OK) return rc;
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_start, c->ev_stop));
  c->timing.run_ms = ms;
  if (c->opt.time_kernels) {
    int trc = collect_kernel_times(c);
    if (trc) return trc;
  }
  std::vector<uint32_t> st(g1);
  HIP_TRY(c, hipMemcpy(st.data(), c->d.gen_status, g1 * sizeof(uint32_t), hipMemcpyDeviceToHost));
  int done = g1;
  for (int g = g0; g < g1; ++g)
    if (st[g]) {
      rc = status_error(c, st[g]);
      done = g;
      break;
    }
  if (done == 0) return rc;
  const int frc = finish_results(c, done, n_inactive);
  if (frc != MCX_OK) return frc;
  for (int g = g0; g < done; ++g) {
    c->timing.advance_items += (int64_t)c->h_gen_cnt[(size_t)g * N_CNT_ALL + CNT_ADV_ITEMS];
    c->timing.collide_items += (int64_t)c->h_gen_cnt[(size_t)g * N_CNT_ALL + CNT_COL_ITEMS];
    c->timing.advance_segments += (int64_t)c->h_gen_cnt[(size_t)g * N_CNT_ALL + CNT_ADV_SEGS];
  }
  if (rc != MCX_OK) return rc;
  c->can_continue = true;
  for (int g = g0; g < done; ++g)
    if (c->h_gen_cnt[(size_t)g * N_CNT_ALL + CNT_KILLED] > 0)
      return fail(c, MCX_EGUARD, "histories reached the event guard");
  return MCX_OK;
}

int mcx_run_generations(mcx_ctx* c, int32_t n_gen, int32_t n_inactive) {
  if (!c) return MCX_EINVAL;
  if (!c->bound) return fail(c, MCX_ESTATE, "bind a workspace first");
  if (c->batch) return fail(c, MCX_ESTATE, "a batch is loaded: use mcx_run_batch");
  if (n_gen < 1 || n_gen > c->n_gen_max || n_inactive < 0 || n_inactive >= n_gen)
    return fail(c, MCX_EINVAL, "generation counts");
  return run_range(c, 0, n_gen, n_inactive);
}

int mcx_continue_generations(mcx_ctx* c, int32_t n_more) {
  if (!c) return MCX_EINVAL;
  if (!c->bound || !c->can_continue)
    return fail(c, MCX_ESTATE, "no completed run (or restored checkpoint) to continue");
  if (n_more < 1 || (int64_t)c->last_n_gen + n_more > c->n_gen_max)
    return fail(c, MCX_EINVAL, "generation count beyond n_gen_max");
  return run_range(c, c->last_n_gen, c->last_n_gen + n_more, c->req_n_inactive);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free runs: the workspace in a static device array
//
// For callers that cannot allocate device memory, the library holds one
// MCX_SCRATCH_BYTES array per GPU (a file-scope __device__ variable, which
// each device keeps until the process ends).  In host code `scratch` names a
// host-side stand-in, not device memory: its device address comes from
// hipGetSymbolAddress, once per device with that device current, and only
// that address is handed to the kernels and copies.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[MCX_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
}  // namespace

// Device address of this device's scratch array (the device must be current).
static int scratch_address(mcx_ctx* c, void** out) {
  const int dev = c->opt.device;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(c, MCX_EINVAL, "device ordinal");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MCX_OK;
}

extern "C" {

int mcx_run_generations_noalloc(mcx_ctx* c, int32_t n_gen, int32_t n_inactive) {
  if (!c) return MCX_EINVAL;
  if (c->batch) return fail(c, MCX_ESTATE, "a batch is loaded: use mcx_run_batch");
  if (c->opt.time_kernels)
    return fail(c, MCX_EINVAL, "kernel timing creates HIP events: turn time_kernels off");
  if (n_gen < 1 || n_inactive < 0 || n_inactive >= n_gen)
    return fail(c, MCX_EINVAL, "generation counts");
  if (!loaded(c)) return fail(c, MCX_ESTATE, "load and seed first");
  HIP_TRY(c, hipSetDevice(c->opt.device));
  void* ptr = nullptr;
  int rc = scratch_address(c, &ptr);
  if (rc != MCX_OK) return rc;
  Dev layout;
  const size_t need = carve(c, layout, nullptr, n_gen);
  if (need > MCX_SCRATCH_BYTES) {
    char msg[160];
    std::snprintf(msg, sizeof msg,
                  "the run needs %zu bytes of workspace; the static scratch holds %zu",
                  need, (size_t)MCX_SCRATCH_BYTES);
    return fail(c, MCX_ENOMEM, msg);
  }
  rc = mcx_bind_workspace(c, ptr, MCX_SCRATCH_BYTES, n_gen);
  if (rc != MCX_OK) return rc;
  return mcx_run_generations(c, n_gen, n_inactive);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// checkpoints: the state a continued run needs (next source, k_used) and the
// per-generation results so far, tied to the problem by a fingerprint
// ---------------------------------------------------------------------------

namespace {

struct CkptHeader {
  char magic[8];
  uint32_t version, ce;
  int32_t precision;
  uint32_t n;
  int32_t n_bins, n_gen, n_inactive, n_cnt;
  uint64_t fingerprint;
};

template <class T>
void fnv(uint64_t* h, const T* p, size_t n) {
  const unsigned char* b = reinterpret_cast<const unsigned char*>(p);
  for (size_t k = 0; k < n * sizeof(T); ++k) {
    *h ^= b[k];
    *h *= 1099511628211ull;
  }
}

uint64_t fingerprint(const mcx_ctx* c) {
  uint64_t h = 1469598103934665603ull;
  const int32_t ints[] = {c->nx, c->ny, c->n_univ, c->max_rings, c->bc[0], c->bc[1], c->bc[2],
                          c->bc[3], c->n_mat, c->G, c->opt.precision, c->ce ? 1 : 0};
  fnv(&h, ints, sizeof(ints) / sizeof(ints[0]));
  const double dbl[] = {c->pitch,    c->x0,        c->y0,        (double)c->opt.max_events,
                        c->ce_nu,    c->ce_watt_a, c->ce_watt_b, c->ce_e_max,
                        c->ce_e_cut, c->ce_src_energy};
  fnv(&h, dbl, sizeof(dbl) / sizeof(dbl[0]));
  fnv(&h, c->pin_map.data(), c->pin_map.size());
  fnv(&h, c->n_rings.data(), c->n_rings.size());
  fnv(&h, c->radii.data(), c->radii.size());
  fnv(&h, c->mats.data(), c->mats.size());
  fnv(&h, c->sig_t.data(), c->sig_t.size());
  fnv(&h, c->nusf.data(), c->nusf.size());
  fnv(&h, c->cum_s.data(), c->cum_s.size());
  fnv(&h, c->cum_chi.data(), c->cum_chi.size());
  fnv(&h, c->ce_grid.data(), c->ce_grid.size());
  fnv(&h, c->ce_xs.data(), c->ce_xs.size());
  fnv(&h, c->ce_awr.data(), c->ce_awr.size());
  fnv(&h, c->ce_dens.data(), c->ce_dens.size());
  fnv(&h, c->ce_mat_nuc.data(), c->ce_mat_nuc.size());
  fnv(&h, c->ce_edges.data(), c->ce_edges.size());
  fnv(&h, c->t_edges.data(), c->t_edges.size());
  fnv(&h, c->t_speed.data(), c->t_speed.size());
  const uint64_t src[] = {c->src.seed, (uint64_t)c->src.n_per_gen, (uint64_t)c->src.fixed_source,
                          c->src.problem_id, (uint64_t)c->src.ent_nx, (uint64_t)c->src.ent_ny};
  fnv(&h, src, 6);
  return h;
}

// Byte layout of a checkpoint: header, k_used, source (x, y, g[, e]), then
// per generation k, entropy, counters, bank size and tallies.
size_t ckpt_size(const mcx_ctx* c, int ng) {
  const size_t N = c->d.N, nb = (size_t)c->d.n_bins;
  size_t b = sizeof(CkptHeader) + 8 + N * (8 + 8 + 4) + (c->ce ? N * 8 : 0);
  b += (size_t)ng * (3 * 8 + 8 + N_CNT_ALL * 8 + 4 + 2 * nb * 8);
  return b;
}

}  // namespace

extern "C" {

int mcx_checkpoint(mcx_ctx* c, void* buf, size_t* len) {
  if (!c || !len) return MCX_EINVAL;
  if (!c->bound || !c->can_continue || c->batch)
    return fail(c, MCX_ESTATE, "no completed run to checkpoint");
  const int ng = c->last_n_gen;
  const size_t need = ckpt_size(c, ng);
  if (!buf) {
    *len = need;
    return MCX_OK;
  }
  if (*len < need) {
    *len = need;
    return fail(c, MCX_ENOMEM, "checkpoint buffer too small");
  }
  HIP_TRY(c, hipSetDevice(c->opt.device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  char* p = static_cast<char*>(buf);
  CkptHeader hd{};
  std::memcpy(hd.magic, "MCXCKPT1", 8);
  hd.version = 1;
  hd.ce = c->ce ? 1u : 0u;
  hd.precision = c->opt.precision;
  hd.n = c->d.N;
  hd.n_bins = c->d.n_bins;
  hd.n_gen = ng;
  hd.n_inactive = c->req_n_inactive;
  hd.n_cnt = N_CNT_ALL;
  hd.fingerprint = fingerprint(c);
  std::memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  const size_t N = c->d.N, nb = (size_t)c->d.n_bins;
  auto down = [&](const void* d, size_t n) {
    hipError_t e = hipMemcpy(p, d, n, hipMemcpyDeviceToHost);
    p += n;
    return e;
  };
  HIP_TRY(c, down(c->d.k_used, 8));
  HIP_TRY(c, down(c->d.src_x, N * 8));
  HIP_TRY(c, down(c->d.src_y, N * 8));
  HIP_TRY(c, down(c->d.src_g, N * 4));
  if (c->ce) HIP_TRY(c, down(c->d.src_e, N * 8));
  HIP_TRY(c, down(c->d.gen_k, (size_t)3 * ng * 8));
  HIP_TRY(c, down(c->d.gen_h, (size_t)ng * 8));
  HIP_TRY(c, down(c->d.gen_cnt, (size_t)N_CNT_ALL * ng * 8));
  HIP_TRY(c, down(c->d.gen_m, (size_t)ng * 4));
  HIP_TRY(c, down(c->d.gen_tal, (size_t)2 * nb * ng * 8));
  *len = need;
  return MCX_OK;
}

int mcx_restore(mcx_ctx* c, const void* buf, size_t len) {
  if (!c || !buf) return MCX_EINVAL;
  if (!c->bound || c->batch) return fail(c, MCX_ESTATE, "bind a workspace for the problem first");
  CkptHeader hd{};
  if (len < sizeof hd) return fail(c, MCX_EINVAL, "checkpoint too short");
  std::memcpy(&hd, buf, sizeof hd);
  if (std::memcmp(hd.magic, "MCXCKPT1", 8) != 0 || hd.version != 1 || hd.n_cnt != N_CNT_ALL)
    return fail(c, MCX_EINVAL, "not a checkpoint of this library");
  if (hd.fingerprint != fingerprint(c) || hd.n != c->d.N || hd.n_bins != c->d.n_bins ||
      hd.ce != (c->ce ? 1u : 0u) || hd.precision != c->opt.precision)
    return fail(c, MCX_EINVAL, "checkpoint of a different problem or precision");
  if (hd.n_gen < 1 || hd.n_gen > c->n_gen_max || hd.n_inactive < 0)
    return fail(c, MCX_EINVAL, "checkpoint generation count beyond n_gen_max");
  if (len < ckpt_size(c, hd.n_gen)) return fail(c, MCX_EINVAL, "checkpoint truncated");
  HIP_TRY(c, hipSetDevice(c->opt.device));
  const int ng = hd.n_gen;
  const char* p = static_cast<const char*>(buf) + sizeof hd;
  const size_t N = c->d.N, nb = (size_t)c->d.n_bins;
  auto up = [&](void* d, size_t n) {
    hipError_t e = hipMemcpy(d, p, n, hipMemcpyHostToDevice);
    p += n;
    return e;
  };
  HIP_TRY(c, up(c->d.k_used, 8));
  HIP_TRY(c, up(c->d.src_x, N * 8));
  HIP_TRY(c, up(c->d.src_y, N * 8));
  HIP_TRY(c, up(c->d.src_g, N * 4));
  if (c->ce) HIP_TRY(c, up(c->d.src_e, N * 8));
  HIP_TRY(c, up(c->d.gen_k, (size_t)3 * ng * 8));
  HIP_TRY(c, up(c->d.gen_h, (size_t)ng * 8));
  HIP_TRY(c, up(c->d.gen_cnt, (size_t)N_CNT_ALL * ng * 8));
  HIP_TRY(c, up(c->d.gen_m, (size_t)ng * 4));
  HIP_TRY(c, up(c->d.gen_tal, (size_t)2 * nb * ng * 8));
  std::vector<uint32_t> zero((size_t)ng + 1, 0u);
  HIP_TRY(c, hipMemcpy(c->d.gen_status, zero.data(), zero.size() * 4, hipMemcpyHostToDevice));
  c->timing = mcx_timing{};
  if (c->opt.record_histories) c->h_rec.assign((size_t)ng * c->d.N, mcx_record{});
  const int frc = finish_results(c, ng, hd.n_inactive);
  if (frc != MCX_OK) return frc;
  c->req_n_inactive = hd.n_inactive;
  c->can_continue = true;
  return MCX_OK;
}

int mcx_get_keff(mcx_ctx* c, double* mean3, double* sigma3, double* per_gen) {
  if (!c) return MCX_EINVAL;
  if (!c->ran) return fail(c, MCX_ESTATE, "no completed run");
  for (int e = 0; e < 3; ++e) {
    if (mean3) mean3[e] = c->h_kstat[e];
    if (sigma3) sigma3[e] = c->h_kstat[3 + e];
  }
  if (per_gen) std::memcpy(per_gen, c->h_gen_k.data(), c->h_gen_k.size() * sizeof(double));
  return MCX_OK;
}

int mcx_get_generation_stats(mcx_ctx* c, double* entropy, int64_t* counts) {
  if (!c) return MCX_EINVAL;
  if (!c->ran) return fail(c, MCX_ESTATE, "no completed run");
  const int ng = c->last_n_gen;
  if (entropy) std::memcpy(entropy, c->h_gen_h.data(), (size_t)ng * sizeof(double));
  if (counts)
    for (int g = 0; g < ng; ++g)
      for (int k = 0; k < MCX_N_CNT; ++k)
        counts[(size_t)g * MCX_N_CNT + k] = (int64_t)c->h_gen_cnt[(size_t)g * N_CNT_ALL + k];
  return MCX_OK;
}

int mcx_get_tallies(mcx_ctx* c, double* fm, double* fs, double* pm, double* ps, int64_t n_bins) {
  if (!c) return MCX_EINVAL;
  if (!c->ran) return fail(c, MCX_ESTATE, "no completed run");
  if (n_bins != c->d.n_bins) return fail(c, MCX_EINVAL, "n_bins mismatch");
  const size_t nb = (size_t)c->d.n_bins;
  double* dst[4] = {fm, pm, fs, ps};
  for (int k = 0; k < 4; ++k)
    if (dst[k]) HIP_TRY(c, hipMemcpy(dst[k], c->d.tal_stat + k * nb, nb * 8, hipMemcpyDeviceToHost));
  return MCX_OK;
}

int mcx_get_generation_tallies(mcx_ctx* c, int32_t gen, double* flux, double* prod,
                               int64_t n_bins) {
  if (!c) return MCX_EINVAL;
  if (!c->ran) return fail(c, MCX_ESTATE, "no completed run");
  if (gen < 0 || gen >= c->last_n_gen) return fail(c, MCX_EINVAL, "generation index");
  if (n_bins != c->d.n_bins) return fail(c, MCX_EINVAL, "n_bins mismatch");
  const size_t nb = (size_t)c->d.n_bins;
  const double* g0 = c->d.gen_tal + (size_t)gen * 2 * nb;
  if (flux) HIP_TRY(c, hipMemcpy(flux, g0, nb * 8, hipMemcpyDeviceToHost));
  if (prod) HIP_TRY(c, hipMemcpy(prod, g0 + nb, nb * 8, hipMemcpyDeviceToHost));
  return MCX_OK;
}

int mcx_get_records(mcx_ctx* c, int32_t gen, mcx_record* out, int64_t n) {
  if (!c || !out) return MCX_EINVAL;
  if (!c->ran) return fail(c, MCX_ESTATE, "no completed run");
  if (!c->opt.record_histories) return fail(c, MCX_ESTATE, "records were not kept");
  if (gen < 0 || gen >= c->last_n_gen || n != (int64_t)c->d.N)
    return fail(c, MCX_EINVAL, "generation index or length");
  std::memcpy(out, c->h_rec.data() + (size_t)gen * c->d.N, (size_t)n * sizeof(mcx_record));
  return MCX_OK;
}

int mcx_get_event_log(mcx_ctx* c, int32_t gen, mcx_event* out, int64_t n) {
  if (!c || !out) return MCX_EINVAL;
  if (!c->ran) return fail(c, MCX_ESTATE, "no completed run");
  if (c->opt.event_log <= 0) return fail(c, MCX_ESTATE, "no event log was kept");
  const size_t ne = (size_t)c->d.N * c->opt.event_log;
  if (gen < 0 || gen >= c->last_n_gen || n != (int64_t)ne)
    return fail(c, MCX_EINVAL, "generation index or length");
  std::memcpy(out, c->h_ev.data() + (size_t)gen * ne, ne * sizeof(mcx_event));
  return MCX_OK;
}

int mcx_get_bank(mcx_ctx* c, double* xyg, int64_t cap, int64_t* len) {
  if (!c || !len) return MCX_EINVAL;
  if (!c->ran) return fail(c, MCX_ESTATE, "no completed run");
  const uint32_t m = c->d.T.fixed_source ? 0u : c->h_gen_m[c->last_n_gen - 1];
  *len = m;
  const size_t n = (size_t)std::min<int64_t>(cap, m);
  if (!xyg || n == 0) return MCX_OK;
  std::vector<double> x(n), y(n), e(c->d.can_e ? n : 0);
  std::vector<int32_t> g(n);
  HIP_TRY(c, hipMemcpy(x.data(), c->d.can_x, n * 8, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(y.data(), c->d.can_y, n * 8, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(g.data(), c->d.can_g, n * 4, hipMemcpyDeviceToHost));
  if (c->d.can_e) HIP_TRY(c, hipMemcpy(e.data(), c->d.can_e, n * 8, hipMemcpyDeviceToHost));
  for (size_t k = 0; k < n; ++k) {
    xyg[3 * k] = x[k];
    xyg[3 * k + 1] = y[k];
    xyg[3 * k + 2] = c->d.can_e ? e[k] : (double)g[k];
  }
  return MCX_OK;
}

int mcx_get_timing(mcx_ctx* c, mcx_timing* out) {
  if (!c || !out) return MCX_EINVAL;
  *out = c->timing;
  return MCX_OK;
}

int mcx_diag_math(mcx_ctx* c, int32_t which, const double* d_in, double* d_out, int64_t n) {
  if (!c || which < 0 || which > 3 || n < 0 || (n > 0 && (!d_in || !d_out))) return MCX_EINVAL;
  HIP_TRY(c, hipSetDevice(c->opt.device));
  HIP_TRY(c, launch_diag_math(which, d_in, d_out, n, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCX_OK;
}

int mcx_host_math(int32_t which, const double* in, double* out, int64_t n) {
  if (which < 0 || which > 3 || n < 0 || (n > 0 && (!in || !out))) return MCX_EINVAL;
  host_math(which, in, out, n);
  return MCX_OK;
}

int mcx_diag_philox(mcx_ctx* c, const uint64_t* d_in, uint64_t* d_out, int64_t n) {
  if (!c || n < 0 || (n > 0 && (!d_in || !d_out))) return MCX_EINVAL;
  HIP_TRY(c, hipSetDevice(c->opt.device));
  HIP_TRY(c, launch_diag_philox(d_in, d_out, n, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCX_OK;
}

// ---------------------------------------------------------------------------
// batches of fixed-source problems
// ---------------------------------------------------------------------------

int mcx_load_batch(mcx_ctx* c, int32_t n_probs, const mcx_problem* probs) {
  if (!c || !probs || n_probs < 1 || n_probs > 65535) return MCX_EINVAL;
  c->bound = false;
  // each problem goes through the single-problem validators, then is
  // appended to the concatenated tables
  std::vector<int> n_rings, mats, pin_map, last_s, last_chi, fissile;
  std::vector<double> radii, sig_t, nusf, sst, cum_s, cum_chi;
  std::vector<float> sig_t_f, nusf_f, sst_f, cum_s_f, cum_chi_f;
  std::vector<mcx_ctx::BProb> bp(n_probs);
  uint64_t hist = 0;
  int64_t bins = 0;
  int G = 0, n_mat = 0, n_univ = 0, max_rings = 0;
  auto app = [](auto& dst, const auto& src) { dst.insert(dst.end(), src.begin(), src.end()); };
  int rc = MCX_OK;
  for (int p = 0; p < n_probs && rc == MCX_OK; ++p) {
    const mcx_problem& q = probs[p];
    rc = mcx_load_geometry(c, &q.geo);
    if (rc == MCX_OK) rc = mcx_load_mg_xs(c, q.n_mat, q.n_grp, q.sig_t, q.sig_s, q.nu_sig_f, q.chi);
    if (rc != MCX_OK) {
      c->err = "problem " + std::to_string(p) + ": " + c->err;
      break;
    }
    if (p > 0 && q.n_grp != G) {
      rc = fail(c, MCX_EINVAL, "problem " + std::to_string(p) + ": group counts differ");
      break;
    }
    if (q.n_hist < 1) {
      rc = fail(c, MCX_EINVAL, "problem " + std::to_string(p) + ": n_hist < 1");
      break;
    }
    for (int u = 0; u < c->n_univ && rc == MCX_OK; ++u)
      for (int k = 0; k <= c->n_rings[u]; ++k)
        if (c->mats[(size_t)u * (c->max_rings + 1) + k] >= c->n_mat) {
          rc = fail(c, MCX_EINVAL,
                    "problem " + std::to_string(p) + ": geometry references a missing material");
          break;
        }
    if (rc != MCX_OK) break;
    G = q.n_grp;
    mcx_ctx::BProb& b = bp[p];
    b.nx = c->nx;
    b.ny = c->ny;
    b.max_rings = c->max_rings;
    b.pin_base = (int)pin_map.size();
    b.univ_base = (int)n_rings.size();
    b.radii_base = (int)radii.size();
    b.mats_base = (int)mats.size();
    b.bin_base = (int)bins;
    b.n_bins = c->nx * c->ny * (c->max_rings + 1) * G;
    b.pitch = c->pitch;
    b.x0 = c->x0;
    b.y0 = c->y0;
    for (int k = 0; k < 4; ++k) b.bc[k] = c->bc[k];
    b.seed = q.seed;
    b.prob = q.problem_id;
    b.hist_base = hist;
    b.n_hist = (uint32_t)std::min<int64_t>(q.n_hist, 0xFFFFFFFFll);
    hist += (uint64_t)q.n_hist;
    bins += b.n_bins;
    if (hist >= (uint64_t(1) << 32) || bins >= (int64_t(1) << 30)) {
      rc = fail(c, MCX_EINVAL, "batch too large (histories or tally bins)");
      break;
    }
    app(pin_map, c->pin_map);
    app(n_rings, c->n_rings);
    app(radii, c->radii);
    for (int m : c->mats) mats.push_back(m + n_mat);
    app(sig_t, c->sig_t);
    app(nusf, c->nusf);
    app(sst, c->sst);
    app(cum_s, c->cum_s);
    app(cum_chi, c->cum_chi);
    app(last_s, c->last_s);
    app(last_chi, c->last_chi);
    app(fissile, c->fissile);
    app(sig_t_f, c->sig_t_f);
    app(nusf_f, c->nusf_f);
    app(sst_f, c->sst_f);
    app(cum_s_f, c->cum_s_f);
    app(cum_chi_f, c->cum_chi_f);
    n_mat += c->n_mat;
    n_univ += c->n_univ;
    max_rings = std::max(max_rings, c->max_rings);
  }
  if (rc != MCX_OK) {
    c->has_geo = c->has_xs = false;
    c->batch = false;
    c->bound = false;
    return rc;
  }
  c->pin_map = std::move(pin_map);
  c->n_rings = std::move(n_rings);
  c->radii = std::move(radii);
  c->mats = std::move(mats);
  c->sig_t = std::move(sig_t);
  c->nusf = std::move(nusf);
  c->sst = std::move(sst);
  c->cum_s = std::move(cum_s);
  c->cum_chi = std::move(cum_chi);
  c->last_s = std::move(last_s);
  c->last_chi = std::move(last_chi);
  c->fissile = std::move(fissile);
  c->sig_t_f = std::move(sig_t_f);
  c->nusf_f = std::move(nusf_f);
  c->sst_f = std::move(sst_f);
  c->cum_s_f = std::move(cum_s_f);
  c->cum_chi_f = std::move(cum_chi_f);
  c->n_mat = n_mat;
  c->n_univ = n_univ;
  c->max_rings = max_rings;
  c->G = G;
  c->bprobs = std::move(bp);
  c->n_probs = n_probs;
  c->batch_hist = hist;
  c->batch_bins = (int)bins;
  c->batch = true;
  c->has_geo = c->has_xs = true;
  c->bound = false;
  c->batch_ran = false;
  c->ran = false;
  return MCX_OK;
}

// Enqueue one batch: clear the accumulators, transport every history,
// reduce per problem.  Kernels only (no memset or copy nodes), so the
// sequence can be recorded as a graph.
static hipError_t enqueue_batch(mcx_ctx* c, hipStream_t s) {
  Dev& d = c->d;
  Accum A = d.A;
  A.status = d.gen_status;
  const int prec = c->opt.precision == MCX_FP32_MIXED ? 1 : 0;
  hipError_t e = launch_fill_u64(d.acc_base, d.acc_words, 0ull, s);
  if (e == hipSuccess)
    e = launch_fill_u64(reinterpret_cast<unsigned long long*>(d.gen_status), 1, 0ull, s);
  if (e == hipSuccess) {
    if (c->opt.engine == MCX_ENGINE_ASYNC) {
      e = launch_async_init(d.ab, d.n_hist, s);
      if (e == hipSuccess)
        e = launch_async(prec, c->pcfg.grid, d.T, 0, A, d.h_kcol, d.h_kabs, d.h_cnt, d.ab,
                         (uint32_t)c->opt.flights, ASYNC_SPIN_LIMIT, nullptr, nullptr, nullptr,
                         nullptr, s);
      if (e == hipSuccess) e = launch_async_status(d.ab, A.status, s);
    } else {
      e = launch_persistent(prec, c->pcfg, d.T, 0, A, d.h_kcol, d.h_kabs, d.h_cnt, d.work, nullptr,
                            nullptr, nullptr, nullptr, s);
    }
  }
  if (e == hipSuccess)
    e = launch_hist_reduce(d.T, c->n_probs, d.h_kcol, d.h_kabs, d.h_cnt, A, d.prob_cnt, d.prob_k, s);
  if (e == hipSuccess)
    e = launch_batch_results(d.T, c->n_probs, A, d.prob_k, d.b_flux, d.b_prod, d.prob_kres, s);
  return e;
}

static void drop_graph(mcx_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

static int build_batch_graph(mcx_ctx* c) {
  drop_graph(c);
  if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  const hipError_t e = enqueue_batch(c, c->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(c->cap_stream, &g);
  if (e != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(c, e != hipSuccess ? e : ee, "recording the batch graph");
  }
  c->graph = g;
  HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
  return MCX_OK;
}

int mcx_run_batch(mcx_ctx* c) {
  if (c) c->time_gen = true;
  if (!c) return MCX_EINVAL;
  if (!c->batch) return fail(c, MCX_ESTATE, "no batch loaded");
  if (!c->bound) return fail(c, MCX_ESTATE, "bind a workspace first");
  HIP_TRY(c, hipSetDevice(c->opt.device));
  c->batch_ran = false;
  c->timing = mcx_timing{};
  if (!c->graph_exec) {
    const int rc = build_batch_graph(c);
    if (rc != MCX_OK) return rc;
  }
  hipStream_t s = c->stream;
  HIP_TRY(c, hipEventRecord(c->ev_start, s));
  HIP_TRY(c, hipGraphLaunch(c->graph_exec, s));
  HIP_TRY(c, hipEventRecord(c->ev_stop, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_start, c->ev_stop));
  c->timing.run_ms = ms;
  c->timing.persistent_ms = ms;
  c->timing.n_persistent = 1;
  uint32_t st = 0;
  HIP_TRY(c, hipMemcpy(&st, c->d.gen_status, sizeof(uint32_t), hipMemcpyDeviceToHost));
  c->h_bk.resize((size_t)3 * c->n_probs);
  c->h_bcnt.resize((size_t)N_CNT * c->n_probs);
  HIP_TRY(c, hipMemcpy(c->h_bk.data(), c->d.prob_kres, c->h_bk.size() * 8, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(c->h_bcnt.data(), c->d.prob_cnt, c->h_bcnt.size() * 8, hipMemcpyDeviceToHost));
  uint64_t flights = 0;
  for (int p = 0; p < c->n_probs; ++p) flights += c->h_bcnt[(size_t)p * N_CNT + CNT_SEG];
  if (flights >= (1ull << 32)) st |= ST_TALLY;
  if (st) return status_error(c, st);
  c->batch_ran = true;
  for (int p = 0; p < c->n_probs; ++p)
    if (c->h_bcnt[(size_t)p * N_CNT + CNT_KILLED] > 0)
      return fail(c, MCX_EGUARD, "histories reached the event guard");
  return MCX_OK;
}

int mcx_get_batch_results(mcx_ctx* c, double* k, int64_t* counts) {
  if (!c) return MCX_EINVAL;
  if (!c->batch_ran) return fail(c, MCX_ESTATE, "no completed batch");
  if (k) std::memcpy(k, c->h_bk.data(), c->h_bk.size() * sizeof(double));
  if (counts)
    for (size_t e = 0; e < c->h_bcnt.size(); ++e) counts[e] = (int64_t)c->h_bcnt[e];
  return MCX_OK;
}

int mcx_get_batch_tallies(mcx_ctx* c, int32_t p, double* flux, double* prod, int64_t n_bins) {
  if (!c) return MCX_EINVAL;
  if (!c->batch_ran) return fail(c, MCX_ESTATE, "no completed batch");
  if (p < 0 || p >= c->n_probs) return fail(c, MCX_EINVAL, "problem index");
  const mcx_ctx::BProb& b = c->bprobs[p];
  if (n_bins != b.n_bins) return fail(c, MCX_EINVAL, "n_bins mismatch");
  if (flux)
    HIP_TRY(c, hipMemcpy(flux, c->d.b_flux + b.bin_base, (size_t)n_bins * 8, hipMemcpyDeviceToHost));
  if (prod)
    HIP_TRY(c, hipMemcpy(prod, c->d.b_prod + b.bin_base, (size_t)n_bins * 8, hipMemcpyDeviceToHost));
  return MCX_OK;
}

// ---------------------------------------------------------------------------
// autotuner of the persistent engine
// ---------------------------------------------------------------------------

static std::string tune_key(mcx_ctx* c) {
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, c->opt.device) == hipSuccess)
    dev = std::string(prop.gcnArchName) + "x" + std::to_string(prop.multiProcessorCount);
  // the shape of the workload: problems, histories, bins, materials, groups
  char buf[256];
  std::snprintf(buf, sizeof buf,
                "dev=%s eng=%d prec=%d batch=%d probs=%d hist=%llu bins=%d mat=%d grp=%d fixed=%d ce=%d",
                dev.c_str(), c->batch ? (int)MCX_ENGINE_PERSISTENT : c->opt.engine,
                c->opt.precision, c->batch ? 1 : 0, c->batch ? c->n_probs : 1,
                (unsigned long long)c->d.n_hist, c->d.n_bins, c->n_mat, c->G,
                c->batch ? 1 : (c->src.fixed_source ? 1 : 0), c->ce ? 1 : 0);
  for (char* q = buf; *q; ++q)
    if (*q == '\n' || *q == '\t') *q = ' ';
  return buf;
}

static bool tune_lookup(const char* path, const std::string& key, mcx_tune* t) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool hit = false;
  while (std::fgets(line, sizeof line, f)) {
    const char* bar = std::strstr(line, " | ");
    if (!bar || std::string(line, bar - line) != key) continue;
    mcx_tune v{};
    if (std::sscanf(bar + 3, "block=%d slots=%d grid=%d tau=%lf sort=%d ms=%lf", &v.block,
                    &v.slots, &v.grid, &v.tau, &v.sort, &v.ms) == 6 &&
        persistent_config_valid(v.block, v.slots) && v.grid >= 1 && v.tau > 0.0 && v.tau <= 1.0 &&
        (v.sort == 0 || v.sort == 1)) {
      *t = v;  // the last matching line wins
      hit = true;
    } else if (std::sscanf(bar + 3, "event block=%d flights=%d lt_flights=%d tail=%d ms=%lf",
                           &v.block, &v.flights, &v.lt_flights, &v.tail, &v.ms) == 5 &&
               v.block >= 64 && v.block <= 1024 && v.block % 64 == 0 && v.flights >= 1 &&
               v.flights <= 65536 && v.lt_flights >= 1 && v.lt_flights <= 65536 && v.tail > 0) {
      *t = v;
      hit = true;
    }
  }
  std::fclose(f);
  return hit;
}

// One timed run of the bound workload with configuration cfg.
static int tune_trial(mcx_ctx* c, const PersistentCfg& cfg, double* ms) {
  c->pcfg = cfg;
  drop_graph(c);
  int rc;
  if (c->batch) {
    rc = mcx_run_batch(c);  // records the graph, then a first replay
    if (rc == MCX_OK || rc == MCX_EGUARD) rc = mcx_run_batch(c);
  } else {
    rc = mcx_run_generations(c, 1, 0);
  }
  if (rc != MCX_OK && rc != MCX_EGUARD) return rc;
  *ms = c->timing.run_ms;
  return MCX_OK;
}

// Event engine: the block size, flights per advance launch, flights of the
// LDS-staged launches and the tail threshold with the shortest run of two
// generations.
static int autotune_event(mcx_ctx* c, const char* cache_path, const std::string& key,
                          mcx_tune* best) {
  mcx_tune t{};
  if (cache_path && tune_lookup(cache_path, key, &t) && t.flights > 0) {
    c->opt.block_size = t.block;
    c->opt.flights = t.flights;
    c->opt.lt_flights = t.lt_flights;
    c->opt.tail_threshold = t.tail;
    if (best) *best = t;
    return MCX_OK;
  }
  const int64_t N = c->d.N;
  auto clamp_tail = [&](int64_t v) {
    return (int)std::min<int64_t>(std::max<int64_t>(v, DEFAULT_TAIL), 1 << 20);
  };
  const int blocks[] = {256, 512};
  const int flights[] = {6, 8};
  const int lts[] = {3, 4, 5, 6};
  const int tails[] = {clamp_tail(std::min<int64_t>(N / 16, DEFAULT_TAIL_MAX / 2)),
                       clamp_tail(std::min<int64_t>(N / 8, DEFAULT_TAIL_MAX)),
                       clamp_tail(std::min<int64_t>(N / 4, 2 * (int64_t)DEFAULT_TAIL_MAX))};
  const mcx_options keep = c->opt;
  double best_ms = 1e300;
  mcx_tune win{};
  for (int b : blocks)
    for (int f : flights)
      for (int lt : lts)
        for (int tl : tails) {
          c->opt.block_size = b;
          c->opt.flights = f;
          c->opt.lt_flights = lt;
          c->opt.tail_threshold = tl;
          // two generations per candidate (the first has its own source and
          // k_used = 1), timed together
          const int rc = mcx_run_generations(c, std::min(2, c->n_gen_max), 0);
          if (rc != MCX_OK && rc != MCX_EGUARD) {
            c->opt = keep;
            return rc;
          }
          if (c->timing.run_ms < best_ms) {
            best_ms = c->timing.run_ms;
            win = mcx_tune{b, 0, 0, 0.0, best_ms, 0, f, lt, tl};
          }
        }
  c->opt.block_size = win.block;
  c->opt.flights = win.flights;
  c->opt.lt_flights = win.lt_flights;
  c->opt.tail_threshold = win.tail;
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s | event block=%d flights=%d lt_flights=%d tail=%d ms=%.4f\n",
                   key.c_str(), win.block, win.flights, win.lt_flights, win.tail, win.ms);
      std::fclose(f);
    }
  }
  if (best) *best = win;
  return MCX_OK;
}

int mcx_autotune(mcx_ctx* c, const char* cache_path, mcx_tune* best) {
  if (!c) return MCX_EINVAL;
  if (!c->bound) return fail(c, MCX_ESTATE, "bind a workspace first");
  const bool event = !c->batch && c->opt.engine == MCX_ENGINE_EVENT;
  if (!event && (c->opt.engine == MCX_ENGINE_ASYNC ||
                 (!c->batch && c->opt.engine != MCX_ENGINE_PERSISTENT)))
    return fail(c, MCX_ESTATE, "the autotuner configures the event and persistent engines");
  HIP_TRY(c, hipSetDevice(c->opt.device));
  const std::string key = tune_key(c);
  if (event) return autotune_event(c, cache_path, key, best);
  mcx_tune t{};
  if (cache_path && tune_lookup(cache_path, key, &t)) {
    c->pcfg = PersistentCfg{t.block, t.slots, t.grid, t.tau, t.sort};
    drop_graph(c);
    if (best) *best = t;
    return MCX_OK;
  }
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->opt.device) == hipSuccess) cus = prop.multiProcessorCount;
  const int blocks[] = {128, 256};
  const int slots[] = {256, 512};
  const int per_cu[] = {1, 2, 3, 4};
  const double taus[] = {0.5, 0.75, 0.9};
  const PersistentCfg keep = c->pcfg;
  double best_ms = 1e300;
  PersistentCfg win = keep;
  for (int b : blocks)
    for (int sl : slots)
      for (int m : per_cu)
        for (double tau : taus) {
          PersistentCfg cfg{b, sl, m * cus, tau, 0};
          double ms = 0;
          const int rc = tune_trial(c, cfg, &ms);
          if (rc != MCX_OK) {
            c->pcfg = keep;
            drop_graph(c);
            return rc;
          }
          if (ms < best_ms) {
            best_ms = ms;
            win = cfg;
          }
        }
  // then the collide-list ordering at the winning launch shape
  {
    PersistentCfg cfg = win;
    cfg.sort = 1;
    double ms = 0;
    const int rc = tune_trial(c, cfg, &ms);
    if (rc != MCX_OK) {
      c->pcfg = keep;
      drop_graph(c);
      return rc;
    }
    if (ms < best_ms) {
      best_ms = ms;
      win = cfg;
    }
  }
  c->pcfg = win;
  drop_graph(c);
  t = mcx_tune{win.block, win.slots, win.grid, win.tau, best_ms, win.sort, 0, 0, 0};
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s | block=%d slots=%d grid=%d tau=%.4f sort=%d ms=%.4f\n", key.c_str(),
                   t.block, t.slots, t.grid, t.tau, t.sort, t.ms);
      std::fclose(f);
    }
  }
  if (best) *best = t;
  return MCX_OK;
}

}  // extern "C"
