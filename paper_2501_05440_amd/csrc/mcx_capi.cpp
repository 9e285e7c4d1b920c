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
#include <vector>

#include "mcx.h"
#include "mcx_launch.hpp"

using namespace mcx;

namespace {

constexpr int RING = 64;
constexpr int DEFAULT_TAIL = 4096;
constexpr int DEFAULT_LOOKAHEAD = 4;
constexpr int64_t DEFAULT_MAX_EVENTS = 100000;

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
  double *src_x = nullptr, *src_y = nullptr;
  int32_t* src_g = nullptr;
  double *can_x = nullptr, *can_y = nullptr;
  int32_t* can_g = nullptr;
  uint32_t *offs = nullptr, *chunk_sum = nullptr, *scan_total = nullptr;
  uint32_t *cnt_live = nullptr, *cnt_col = nullptr;
  double *gen_k = nullptr, *gen_h = nullptr, *gen_tal = nullptr;
  unsigned long long* gen_cnt = nullptr;
  uint32_t* gen_m = nullptr;
  double *k_used = nullptr, *xi0 = nullptr, *k_stat = nullptr;
  double *tal_stat = nullptr;  // [mean flux | mean prod | sigma flux | sigma prod]
  uint32_t* ent_hist = nullptr;
  double* ent_term = nullptr;
  uint32_t* gen_status = nullptr;  // [n_gen_max] status bits per generation
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

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int n_gen_max = 0;
  Dev d;

  // results of the last run
  int last_n_gen = 0, last_n_inactive = 0;
  bool ran = false;
  std::vector<double> h_gen_k, h_gen_h, h_kstat;
  std::vector<unsigned long long> h_gen_cnt;
  std::vector<uint32_t> h_gen_m;
  std::vector<mcx_record> h_rec;
  mcx_timing timing{};

  // host-side synchronisation helpers
  uint32_t* h_pin = nullptr;  // [RING] live counts + [RING..] status words
  hipEvent_t ev_ring[RING]{};
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  std::vector<hipEvent_t> ev_pool;
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
  if (c->opt.block_size == 0) c->opt.block_size = 256;
  if (c->opt.block_size < 64 || c->opt.block_size > 1024 || c->opt.block_size % 64) {
    delete c;
    return MCX_EINVAL;
  }
  if (c->opt.precision != MCX_FP64 && c->opt.precision != MCX_FP32_MIXED) {
    delete c;
    return MCX_EINVAL;
  }
  // tail_threshold == 0: N / 8, at least DEFAULT_TAIL (resolved per run)
  if (c->opt.lookahead <= 0) c->opt.lookahead = DEFAULT_LOOKAHEAD;
  if (c->opt.lookahead > RING - 2) c->opt.lookahead = RING - 2;
  if (c->opt.max_events <= 0) c->opt.max_events = DEFAULT_MAX_EVENTS;
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
      sst_f[mg] = run;
      if (run > sig_t_f[mg]) return fail(c, MCX_EINVAL, "scattering exceeds sig_t in binary32");
      cchi += (float)chi[mg];
      cum_chi_f[mg] = cchi;
    }
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
  c->bound = false;
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
  const size_t N = (size_t)c->src.n_per_gen;
  const int mr1 = c->max_rings + 1;
  const size_t MG = (size_t)c->n_mat * c->G;
  const int nb = c->nx * c->ny * mr1 * c->G;
  const int stripes = std::max(1, std::min(STRIPES, 65536 / std::max(1, 2 * nb)));
  const uint32_t fis_cap = (uint32_t)std::min<size_t>(2 * N + 4096, 0xFFFFFFF0u);
  const size_t n_ent = (size_t)c->src.ent_nx * c->src.ent_ny;
  const size_t n_cnt_slots = (size_t)c->opt.max_events + 4;

  Tables& T = d.T;
  T.pin_map = cv.take<int>((size_t)c->nx * c->ny);
  T.n_rings = cv.take<int>(c->n_univ);
  T.radii = cv.take<double>((size_t)c->n_univ * c->max_rings);
  T.mats = cv.take<int>((size_t)c->n_univ * mr1);
  T.sig_t = cv.take<double>(MG);
  T.nusf = cv.take<double>(MG);
  T.sst = cv.take<double>(MG);
  T.cum_s = cv.take<double>(MG * c->G);
  T.last_s = cv.take<int>(MG);
  T.cum_chi = cv.take<double>(MG);
  T.last_chi = cv.take<int>(c->n_mat);
  T.fissile = cv.take<int>(c->n_mat);
  T.sig_t_f = cv.take<float>(MG);
  T.nusf_f = cv.take<float>(MG);
  T.sst_f = cv.take<float>(MG);
  T.cum_s_f = cv.take<float>(MG * c->G);
  T.cum_chi_f = cv.take<float>(MG);
  const bool fp32 = c->opt.precision == MCX_FP32_MIXED;
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
  }
  d.src_x = cv.take<double>(N);
  d.src_y = cv.take<double>(N);
  d.src_g = cv.take<int32_t>(N);
  Accum& A = d.A;
  A.fis.x = cv.take<double>(fis_cap);
  A.fis.y = cv.take<double>(fis_cap);
  A.fis.g = cv.take<int32_t>(fis_cap);
  A.fis.parent = cv.take<uint32_t>(fis_cap);
  A.fis.seq = cv.take<uint32_t>(fis_cap);
  A.fis_cap = fis_cap;
  d.can_x = cv.take<double>(fis_cap);
  d.can_y = cv.take<double>(fis_cap);
  d.can_g = cv.take<int32_t>(fis_cap);
  A.nsite_id = cv.take<uint32_t>(N);
  d.offs = cv.take<uint32_t>(N);
  d.chunk_sum = cv.take<uint32_t>(scan_chunks((uint32_t)N) + 1);
  d.scan_total = cv.take<uint32_t>(1);
  d.gen_status = cv.take<uint32_t>(n_gen_max);
  A.status = d.gen_status;
  d.cnt_live = cv.take<uint32_t>(n_cnt_slots);
  d.cnt_col = cv.take<uint32_t>(n_cnt_slots);
  // per-generation accumulators, zeroed together
  const size_t w_tally = (size_t)stripes * 2 * nb;
  const size_t w_tally_t = (size_t)2 * nb;
  const size_t w_k = 3 * STRIPES * 2;
  const size_t w_cnt = (size_t)N_CNT_ALL * STRIPES;
  const size_t w_misc = 1 + (n_ent + 1) / 2;
  d.acc_words = w_tally + w_tally_t + w_k + w_cnt + w_misc;
  d.acc_base = cv.take<unsigned long long>(d.acc_words);
  if (base) {
    A.tally = d.acc_base;
    A.tally_t = A.tally + w_tally;
    A.k = A.tally_t + w_tally_t;
    A.cnt = A.k + w_k;
    A.n_fis = reinterpret_cast<uint32_t*>(A.cnt + w_cnt);
    d.ent_hist = reinterpret_cast<uint32_t*>(A.cnt + w_cnt + 1);
  }
  // results
  d.gen_k = cv.take<double>((size_t)3 * n_gen_max);
  d.gen_h = cv.take<double>(n_gen_max);
  d.gen_cnt = cv.take<unsigned long long>((size_t)N_CNT_ALL * n_gen_max);
  d.gen_m = cv.take<uint32_t>(n_gen_max);
  d.gen_tal = cv.take<double>((size_t)2 * nb * n_gen_max);
  d.tal_stat = cv.take<double>((size_t)4 * nb);
  d.ent_term = cv.take<double>(n_ent);
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

int mcx_workspace_size(mcx_ctx* c, int32_t n_gen_max, size_t* bytes) {
  if (!c || !bytes || n_gen_max < 1) return MCX_EINVAL;
  if (!c->has_geo || !c->has_xs || !c->has_src) return fail(c, MCX_ESTATE, "load and seed first");
  Dev scratch;
  *bytes = carve(c, scratch, nullptr, n_gen_max);
  return MCX_OK;
}

int mcx_bind_workspace(mcx_ctx* c, void* ptr, size_t bytes, int32_t n_gen_max) {
  if (!c || !ptr || n_gen_max < 1) return MCX_EINVAL;
  c->bound = false;
  c->ran = false;
  if (!c->has_geo || !c->has_xs || !c->has_src) return fail(c, MCX_ESTATE, "load and seed first");
  if ((uintptr_t)ptr % 256) return fail(c, MCX_EINVAL, "workspace must be 256-byte aligned");
  // materials referenced by the geometry must exist
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
  Tables& T = c->d.T;
  T.nx = c->nx;
  T.ny = c->ny;
  T.n_univ = c->n_univ;
  T.max_rings = c->max_rings;
  T.mr1 = c->max_rings + 1;
  T.pitch = c->pitch;
  T.x0 = c->x0;
  T.y0 = c->y0;
  T.width = (double)c->nx * c->pitch;
  T.height = (double)c->ny * c->pitch;
  for (int k = 0; k < 4; ++k) T.bc[k] = c->bc[k];
  T.n_mat = c->n_mat;
  T.G = c->G;
  T.seed = c->src.seed;
  T.prob = c->src.problem_id;
  T.fixed_source = c->src.fixed_source ? 1 : 0;
  T.ent_nx = c->src.ent_nx;
  T.ent_ny = c->src.ent_ny;
  T.n_bins = c->d.n_bins;
  T.tally_stripes = c->d.stripes;
  // binary32 terms can exceed the binary64 bound by a few ulp: 1% headroom
  d_max *= 1.01;
  kc_max *= 1.01;
  ka_max *= 1.01;
  T.q_flux = fixed_point_scale(d_max);
  T.q_kcol = fixed_point_scale(kc_max);
  T.q_kabs = fixed_point_scale(ka_max);
  T.max_events = c->opt.max_events;

  hipStream_t s = c->stream;
  auto up = [&](const void* dst, const void* srcp, size_t n) {
    return hipMemcpyAsync(const_cast<void*>(dst), srcp, n, hipMemcpyHostToDevice, s);
  };
  HIP_TRY(c, up(T.pin_map, c->pin_map.data(), c->pin_map.size() * sizeof(int)));
  HIP_TRY(c, up(T.n_rings, c->n_rings.data(), c->n_rings.size() * sizeof(int)));
  HIP_TRY(c, up(T.radii, c->radii.data(), c->radii.size() * sizeof(double)));
  HIP_TRY(c, up(T.mats, c->mats.data(), c->mats.size() * sizeof(int)));
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
  HIP_TRY(c, hipStreamSynchronize(s));
  c->bound = true;
  c->ran = false;
  return MCX_OK;
}

// Enqueue a timing event pair around a launch when kernel timing is on.
static hipError_t time_mark(mcx_ctx* c, int kind, bool begin) {
  if (!c->opt.time_kernels) return hipSuccess;
  if (begin) c->ev_kind.push_back(kind);
  const size_t k = (c->ev_kind.size() - 1) * 2 + (begin ? 0 : 1);
  while (c->ev_pool.size() <= k) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
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
    } else {
      c->timing.tail_ms += ms;
    }
  }
  c->ev_kind.clear();
  return MCX_OK;
}

static int run_generation(mcx_ctx* c, int gen) {
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
  if (gen == 0 || T.fixed_source)
    HIP_TRY(c, launch_source(T, gen, N, c->d.src_x, c->d.src_y, c->d.src_g, A.status, s));
  const int prec = c->opt.precision == MCX_FP32_MIXED ? 1 : 0;
  HIP_TRY(c, launch_birth(prec, T, gen, N, c->d.src_x, c->d.src_y, c->d.src_g, c->d.bank[0], c->d.cnt_live,
                          c->d.cnt_col, gen > 0 ? c->d.gen_status + gen - 1 : nullptr, A.status,
                          s));

  // event iterations; `bound` is the live count of iteration `known`, an
  // upper bound for every later iteration
  uint32_t bound = N;
  int64_t known = 0, it = 0;
  const int64_t tail = c->opt.tail_threshold != 0
                           ? (int64_t)c->opt.tail_threshold
                           : std::max<int64_t>(DEFAULT_TAIL, (int64_t)N / 8);
  int cur = 0;
  const int block = c->opt.block_size;
  for (;;) {
    if (bound == 0) break;
    if ((size_t)it + 3 >= c->d.n_cnt_slots) return fail(c, MCX_EDEVICE, "iteration slots exhausted");
    if (tail > 0 && bound <= (uint32_t)tail) {
      HIP_TRY(c, time_mark(c, 2, true));
      HIP_TRY(c, launch_tail(prec, rec, T, gen, (uint32_t)it, c->d.bank[cur], c->d.cnt_live + it, A, c->d.R,
                             bound, s));
      HIP_TRY(c, time_mark(c, 2, false));
      c->timing.n_tail_launches += 1;
      break;
    }
    HIP_TRY(c, time_mark(c, 0, true));
    HIP_TRY(c, launch_advance(prec, rec, T, gen, (uint32_t)it, c->d.bank[cur], c->d.cnt_live + it,
                              c->d.bank[1 - cur], c->d.cnt_live + it + 1, c->d.bank[2],
                              c->d.cnt_col + it, A, c->d.R, c->d.cnt_live + it + 2, c->d.cnt_col + it + 1,
                              bound, block, s));
    HIP_TRY(c, time_mark(c, 0, false));
    HIP_TRY(c, time_mark(c, 1, true));
    HIP_TRY(c, launch_collide(prec, rec, T, gen, c->d.bank[2], c->d.cnt_col + it, c->d.bank[1 - cur],
                              c->d.cnt_live + it + 1, A, c->d.R, bound, block, s));
    HIP_TRY(c, time_mark(c, 1, false));
    cur = 1 - cur;
    ++it;
    c->timing.n_iterations += 1;
    HIP_TRY(c, hipMemcpyAsync(&c->h_pin[it % RING], c->d.cnt_live + it, sizeof(uint32_t),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipEventRecord(c->ev_ring[it % RING], s));
    while (known < it) {
      hipEvent_t e = c->ev_ring[(known + 1) % RING];
      hipError_t q = hipEventQuery(e);
      if (q == hipErrorNotReady && it - known >= c->opt.lookahead) {
        HIP_TRY(c, hipEventSynchronize(e));
        q = hipSuccess;
      }
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return hip_fail(c, q, "hipEventQuery");
      ++known;
      bound = c->h_pin[known % RING];
    }
  }

  // generation end
  HIP_TRY(c, launch_gen_totals(T, gen, N, A, c->d.gen_k, c->d.gen_cnt, c->d.gen_m, c->d.k_used, c->d.xi0, s));
  HIP_TRY(c, launch_gen_tallies(T, gen, N, A, c->d.gen_tal, c->d.gen_k, s));
  if (!T.fixed_source) {
    HIP_TRY(c, launch_scan(A.nsite_id, N, c->d.chunk_sum, c->d.offs, c->d.scan_total, s));
    HIP_TRY(c, launch_gen_check(T, A.n_fis, c->d.scan_total, A.status, s));
    HIP_TRY(c, launch_canon(A.fis, A.n_fis, c->d.offs, A.nsite_id, c->d.fis_cap, c->d.can_x, c->d.can_y,
                            c->d.can_g, A.status, c->d.fis_cap, s));
    HIP_TRY(c, launch_entropy(T, gen, c->d.can_x, c->d.can_y, A.n_fis, c->d.fis_cap, c->d.ent_hist,
                              c->d.ent_term, c->d.gen_h, c->d.fis_cap, s));
    HIP_TRY(c, launch_comb(N, A.n_fis, c->d.fis_cap, c->d.xi0, c->d.can_x, c->d.can_y, c->d.can_g, c->d.src_x, c->d.src_y,
                           c->d.src_g, s));
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
    mcx_record* out = c->h_rec.data() + (size_t)gen * N;
    for (uint32_t i = 0; i < N; ++i) {
      out[i] = mcx_record{n_seg[i], n_col[i], n_cross[i], n_refl[i], fate[i], (int32_t)ns[i],
                          g_final[i], ctr[i], tl[i], kc[i], xf[i], yf[i]};
    }
  }
  return MCX_OK;
}

static int status_error(mcx_ctx* c, uint32_t st) {
  if (st & ST_SOURCE) return fail(c, MCX_ELOST, "source sampling found no fissile point");
  if (st & ST_OVERFLOW) return fail(c, MCX_EOVERFLOW, "fission bank overflow");
  if (st & (ST_SITE_SEQ | ST_SCAN)) return fail(c, MCX_EDEVICE, "inconsistent fission bank");
  if (st & ST_EXTINCT) return fail(c, MCX_EEXTINCT, "fission bank is empty");
  return fail(c, MCX_EDEVICE, "generation skipped");
}

int mcx_run_generations(mcx_ctx* c, int32_t n_gen, int32_t n_inactive) {
  if (!c) return MCX_EINVAL;
  if (!c->bound) return fail(c, MCX_ESTATE, "bind a workspace first");
  if (n_gen < 1 || n_gen > c->n_gen_max || n_inactive < 0 || n_inactive >= n_gen)
    return fail(c, MCX_EINVAL, "generation counts");
  HIP_TRY(c, hipSetDevice(c->opt.device));
  hipStream_t s = c->stream;
  c->timing = mcx_timing{};
  c->ran = false;
  c->last_n_gen = n_gen;
  c->last_n_inactive = n_inactive;
  if (c->opt.record_histories) c->h_rec.assign((size_t)n_gen * c->d.N, mcx_record{});
  const double one = 1.0;
  HIP_TRY(c, hipMemcpyAsync(c->d.k_used, &one, sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(c, launch_fill_u64(reinterpret_cast<unsigned long long*>(c->d.gen_status),
                             ((size_t)n_gen + 1) / 2, 0ull, s));
  HIP_TRY(c, hipEventRecord(c->ev_start, s));
  // generations are enqueued back to back; each one's status is checked
  // once the run has finished (a failed generation makes the later ones run
  // empty)
  int rc = MCX_OK;
  for (int g = 0; g < n_gen; ++g) {
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
  std::vector<uint32_t> st(n_gen);
  HIP_TRY(c, hipMemcpy(st.data(), c->d.gen_status, n_gen * sizeof(uint32_t), hipMemcpyDeviceToHost));
  int done = n_gen;
  for (int g = 0; g < n_gen; ++g)
    if (st[g]) {
      rc = status_error(c, st[g]);
      done = g;
      break;
    }
  if (done == 0) return rc;
  const int ng = done;
  const int ni = std::min(n_inactive, ng - 1);
  HIP_TRY(c, launch_stats(2 * c->d.n_bins, ng, ni, c->d.gen_tal, c->d.tal_stat, c->d.tal_stat + 2 * c->d.n_bins,
                          c->d.gen_k, c->d.k_stat, s));
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
  for (int g = 0; g < ng; ++g) {
    c->timing.advance_items += (int64_t)c->h_gen_cnt[(size_t)g * N_CNT_ALL + CNT_ADV_ITEMS];
    c->timing.collide_items += (int64_t)c->h_gen_cnt[(size_t)g * N_CNT_ALL + CNT_COL_ITEMS];
  }
  if (rc != MCX_OK) return rc;
  for (int g = 0; g < ng; ++g)
    if (c->h_gen_cnt[(size_t)g * N_CNT_ALL + CNT_KILLED] > 0)
      return fail(c, MCX_EGUARD, "histories reached the event guard");
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

int mcx_get_bank(mcx_ctx* c, double* xyg, int64_t cap, int64_t* len) {
  if (!c || !len) return MCX_EINVAL;
  if (!c->ran) return fail(c, MCX_ESTATE, "no completed run");
  const uint32_t m = c->d.T.fixed_source ? 0u : c->h_gen_m[c->last_n_gen - 1];
  *len = m;
  const size_t n = (size_t)std::min<int64_t>(cap, m);
  if (!xyg || n == 0) return MCX_OK;
  std::vector<double> x(n), y(n);
  std::vector<int32_t> g(n);
  HIP_TRY(c, hipMemcpy(x.data(), c->d.can_x, n * 8, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(y.data(), c->d.can_y, n * 8, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(g.data(), c->d.can_g, n * 4, hipMemcpyDeviceToHost));
  for (size_t k = 0; k < n; ++k) {
    xyg[3 * k] = x[k];
    xyg[3 * k + 1] = y[k];
    xyg[3 * k + 2] = (double)g[k];
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

}  // extern "C"
