// mcx_kernels_common.hpp - per-particle transport operations shared by the
// event kernels (mcx_kernels.hip) and the persistent engine
// (mcx_persistent.hip): precision policy, particle state, one flight, one
// collision, source sampling, block scans and exact-sum conversions.
#pragma once

#include <type_traits>

#include "mcx_launch.hpp"

namespace mcx {

// ---------------------------------------------------------------------------
// precision policy
//
// FP64 (the paper's precision): every quantity in binary64, ln and cos/sin
// correctly rounded.  FP32-mixed (R = float): directions, the distance to
// collision, the plane distances (numerator differenced in FP64, then
// rounded), cross sections, the reaction and group comparisons and the
// direction sampling in binary32; positions, the cylinder quadratic, the
// comparison of the distances, the move, the tallies and the k and entropy
// estimators in binary64.
// ---------------------------------------------------------------------------

template <class R>
struct Prec;

template <>
struct Prec<double> {
  static __device__ __forceinline__ double xi(double u) { return u; }
  static __device__ __forceinline__ double dcol(double xi, double st,
                                               const double* lt = log_tab()) {
    return -cr_log(xi, lt) / st;
  }
  static __device__ __forceinline__ double plane(double x, double lo, double hi, double u) {
    return dist_plane(x, lo, hi, u);
  }
  static __device__ __forceinline__ void iso(double xm, double xp, double* u, double* v,
                                             const double* sct = sc_tab()) {
    isotropic_uv(xm, xp, u, v, sct);
  }
};

template <>
struct Prec<float> {
  // (float) of a draw may round up to 1; keep it in (0, 1)
  static __device__ __forceinline__ float xi(double u) {
    const float f = (float)u;
    return f < 1.0f ? f : 0x1.fffffep-1f;
  }
  static __device__ __forceinline__ float dcol(float xi, float st, const double* = nullptr) {
    return -logf(xi) / st;
  }
  static __device__ __forceinline__ float plane(double x, double lo, double hi, float u) {
    float t;
    if (u > 0.0f) {
      t = (float)(hi - x) / u;
    } else if (u < 0.0f) {
      t = (float)(lo - x) / u;
    } else {
      return __builtin_inff();
    }
    return t < 0.0f ? 0.0f : t;
  }
  static __device__ __forceinline__ void iso(float xm, float xp, float* u, float* v,
                                             const double* = nullptr) {
    const float w = 2.0f * xm - 1.0f;
    const float s2 = 1.0f - w * w;
    const float s = sqrtf(s2 > 0.0f ? s2 : 0.0f);
    float sn, cs;
    sincospif(2.0f * xp, &sn, &cs);
    *u = s * cs;
    *v = s * sn;
  }
};

// ---------------------------------------------------------------------------
// draw cache of a sparse tail wavefront
//
// Near the end of a generation a tail wavefront holds a few long histories
// and many idle lanes, and each history's flights are a serial chain whose
// largest links are the Philox block, the correctly rounded ln of the
// distance to collision and cos/sin of the scattering azimuth.  The transport
// stream of a history is fixed in advance (its draws depend only on the
// history id and the draw index), so when at most TC_SLOTS histories remain
// live the wavefront's lanes evaluate the next TC_WORDS draws of each one
// side by side: every lane one draw, with its uniform, ln and cos/sin of 2 pi
// times it, written to LDS.  The history then takes its draws from there and
// falls back to evaluating them itself past the end of its window.  The
// values are the ones the history would compute, so results do not change.
// ---------------------------------------------------------------------------

constexpr int TC_SLOTS = 4;    // histories served per wavefront
constexpr int TC_WORDS = 16;   // draws per history and refill (TC_SLOTS * TC_WORDS = 64)
constexpr int TC_LOW = 6;      // refill when fewer draws than this remain

struct DrawEntry {
  double u, ln, c, s;  // uniform, ln(u), cos(2 pi u), sin(2 pi u)
};

// The wavefront's windows (tail kernels run one wavefront per block).
static __shared__ DrawEntry tc_cache[TC_SLOTS * TC_WORDS];

struct CachedStream : Stream {
  uint32_t ebase;        // first entry of this history's window
  uint32_t cbase, clen;  // draw index of that entry, entries valid
  int last;              // entry of the last draw, or -1 if evaluated here

  __device__ CachedStream(const Stream& s)
      : Stream(s), ebase(0), cbase(0), clen(0), last(-1) {}

  __device__ double next() {
    const uint32_t o = draw - cbase;
    if (o < clen) {
      last = (int)(ebase + o);
      draw += 1u;
      return tc_cache[last].u;
    }
    last = -1;
    return Stream::next();
  }
};

// ---------------------------------------------------------------------------
// lockstep stream of the advance kernels
//
// A flight takes one draw, so a lane needs a new Philox block every fourth
// flight, and the lanes of a wavefront reach that point at different
// flights: with Stream the wavefront evaluates the block code at nearly
// every flight, each time for about a quarter of its lanes.  LockStream
// holds up to two blocks per lane, and top_up() (called by the active lanes
// before every flight) evaluates blocks only when some active lane has run
// dry, and then for every active lane that has room: the dry lanes take the
// block of their next draw, the others the block after the one they hold.
// The wavefront then evaluates the block code about once per four flights,
// with most of its lanes active.  Draw values and order are Stream's.
// ---------------------------------------------------------------------------

struct LockStream {
  uint64_t k0, k1, id, gen, prob;
  uint32_t draw;
  uint32_t b0;   // block of w[0..3] (draws 4 b0 .. 4 b0 + 3), ~0u = none
  bool has1;     // w[4..7] holds block b0 + 1
  uint64_t w[8];

  __device__ LockStream(uint64_t seed, uint64_t tag, uint64_t id_, uint64_t gen_, uint64_t prob_,
                        uint32_t draw_)
      : k0(seed), k1(tag), id(id_), gen(gen_), prob(prob_), draw(draw_), b0(~0u), has1(false) {}

  __device__ __forceinline__ void shift() {
    w[0] = w[4];
    w[1] = w[5];
    w[2] = w[6];
    w[3] = w[7];
    b0 += 1u;
    has1 = false;
  }

  // Every active lane of the wavefront must call it (lanes that have left
  // the flight loop do not).
  __device__ __forceinline__ void top_up() {
    const uint32_t b = draw >> 2;
    if (has1 && b == b0 + 1u) shift();
    const bool dry = b != b0;
    if (__ballot(dry) == 0ull) return;
    if (dry || !has1) {
      const uint32_t cb = dry ? b : b0 + 1u;
      const u64x4 v = philox4x64_10(cb, id, gen, prob, k0, k1);
      if (dry) {
        w[0] = v.v[0];
        w[1] = v.v[1];
        w[2] = v.v[2];
        w[3] = v.v[3];
        b0 = b;
        has1 = false;
      } else {
        w[4] = v.v[0];
        w[5] = v.v[1];
        w[6] = v.v[2];
        w[7] = v.v[3];
        has1 = true;
      }
    }
  }

  // With the block of the next draw held, also evaluate the one after it
  // (every active lane at once).
  __device__ __forceinline__ void fill_next() {
    if (!has1 && b0 == (draw >> 2)) {
      const u64x4 v = philox4x64_10(b0 + 1u, id, gen, prob, k0, k1);
      w[4] = v.v[0];
      w[5] = v.v[1];
      w[6] = v.v[2];
      w[7] = v.v[3];
      has1 = true;
    }
  }

  __device__ __forceinline__ double next() {
    const uint32_t b = draw >> 2;
    if (has1 && b == b0 + 1u) shift();
    if (b != b0) {  // not topped up (never on the advance kernels' flights)
      const u64x4 v = philox4x64_10(b, id, gen, prob, k0, k1);
      w[0] = v.v[0];
      w[1] = v.v[1];
      w[2] = v.v[2];
      w[3] = v.v[3];
      b0 = b;
      has1 = false;
    }
    const uint32_t k = draw & 3u;
    const uint64_t x = k == 0 ? w[0] : k == 1 ? w[1] : k == 2 ? w[2] : w[3];
    draw += 1u;
    return u01(x);
  }
};

// Distance to collision from the next draw.
template <class R, class S>
__device__ __forceinline__ R draw_dcol(S& rs, R st, const double* lt) {
  const R xi = Prec<R>::xi(rs.next());
  return Prec<R>::dcol(xi, st, lt);
}

template <>
__device__ __forceinline__ double draw_dcol<double, CachedStream>(CachedStream& rs, double st,
                                                                  const double* lt) {
  const double xi = rs.next();
  const double l = rs.last >= 0 ? tc_cache[rs.last].ln : cr_log(xi, lt);
  return -l / st;
}

// Isotropic direction from the next two draws.
template <class R, class S>
__device__ __forceinline__ void draw_iso(S& rs, R* u, R* v, const double* sct) {
  const R xm = Prec<R>::xi(rs.next());
  const R xp = Prec<R>::xi(rs.next());
  Prec<R>::iso(xm, xp, u, v, sct);
}

template <>
__device__ __forceinline__ void draw_iso<double, CachedStream>(CachedStream& rs, double* u,
                                                               double* v, const double* sct) {
  const double xm = rs.next();
  const double xp = rs.next();
  if (rs.last >= 0)
    isotropic_uv_cs(xm, tc_cache[rs.last].c, tc_cache[rs.last].s, u, v);
  else
    isotropic_uv(xm, xp, u, v, sct);
}

// Cross-section tables of the working precision.
template <class R>
struct XSView {
  const R* sig_t;
  const R* nusf;
  const R* sst;
  const R* cum_s;
  const R* cum_chi;
};

template <class R>
__device__ __forceinline__ XSView<R> xs_view(const Tables& T);

template <>
__device__ __forceinline__ XSView<double> xs_view<double>(const Tables& T) {
  return XSView<double>{T.sig_t, T.nusf, T.sst, T.cum_s, T.cum_chi};
}

template <>
__device__ __forceinline__ XSView<float> xs_view<float>(const Tables& T) {
  return XSView<float>{T.sig_t_f, T.nusf_f, T.sst_f, T.cum_s_f, T.cum_chi_f};
}

// ---------------------------------------------------------------------------
// LDS copies of the multigroup tables
//
// The lookups of a flight form a dependent chain: lattice cell -> universe ->
// ring material -> cross section, then the ln table, and at a collision the
// scattering row and the sin/cos table.  Through the cache hierarchy each
// link costs a vector-memory round trip, which is what bounds a lone history
// (the tail).  When the lattice and the working-precision cross sections fit
// in a few KB, every block of the event kernels first copies them into LDS
// and runs on the copies.
// ---------------------------------------------------------------------------

constexpr size_t LDS_TABLES_MAX = 32768;  // bytes per block

MCX_HD size_t lds_round8(size_t b) { return (b + 7) & ~(size_t)7; }

// Bytes of the LDS copy for element size rb of the working precision.
MCX_HD size_t lds_tables_bytes(const Tables& T, size_t rb) {
  const Geo& L = T.geo;
  const size_t nc = (size_t)L.nx * (size_t)L.ny, nu = (size_t)T.n_univ;
  const size_t mg = (size_t)T.n_mat * (size_t)T.G;
  return lds_round8(nc * 4) + lds_round8(nu * 4) + lds_round8(nu * (size_t)L.mr1 * 4) +
         lds_round8(nu * (size_t)L.max_rings * 8) + 4 * lds_round8(mg * rb) +
         lds_round8(mg * (size_t)T.G * rb) + lds_round8(mg * 4) + lds_round8((size_t)T.n_mat * 4) +
         (2 * MCX_LOG_TAB_N + 4 * MCX_SINCOS_TAB_N) * 8 +
         (T.time ? ((size_t)T.nt + 1 + (size_t)T.G) * 8 : 0);
}

__device__ __forceinline__ const void* lds_put(char* base, uint32_t* off, const void* src,
                                               size_t bytes, bool copy) {
  uint32_t* d = reinterpret_cast<uint32_t*>(base + *off);
  const uint32_t* s = static_cast<const uint32_t*>(src);
  const uint32_t n = copy ? (uint32_t)(bytes / 4) : 0u;
  for (uint32_t w = threadIdx.x; w < n; w += blockDim.x) d[w] = s[w];
  *off += (uint32_t)lds_round8(bytes);
  return d;
}

template <class R>
__device__ __forceinline__ void set_xs_view(Tables& T, const XSView<R>& X);

template <>
__device__ __forceinline__ void set_xs_view<double>(Tables& T, const XSView<double>& X) {
  T.sig_t = X.sig_t;
  T.nusf = X.nusf;
  T.sst = X.sst;
  T.cum_s = X.cum_s;
  T.cum_chi = X.cum_chi;
}

template <>
__device__ __forceinline__ void set_xs_view<float>(Tables& T, const XSView<float>& X) {
  T.sig_t_f = X.sig_t;
  T.nusf_f = X.nusf;
  T.sst_f = X.sst;
  T.cum_s_f = X.cum_s;
  T.cum_chi_f = X.cum_chi;
}

// The tables a kernel runs on: with LDS, copies made by the whole block
// (every thread of the block must call this, before any early exit; a block
// with no work passes copy = false and must then not read the tables);
// otherwise the arguments with the math tables of constant memory.
template <class R, bool LDS>
__device__ __forceinline__ Tables kernel_tables(const Tables& T0, bool copy = true) {
  Tables T = T0;
  if constexpr (!LDS) {
    T.lt = log_tab();
    T.sct = sc_tab();
  } else {
    extern __shared__ __align__(16) char lds_tab[];
    const Geo& L = T0.geo;
    const size_t nc = (size_t)L.nx * L.ny, nu = (size_t)T0.n_univ;
    const size_t mg = (size_t)T0.n_mat * T0.G, rb = sizeof(R);
    uint32_t off = 0;
    T.geo.pin_map = (const int*)lds_put(lds_tab, &off, L.pin_map, nc * 4, copy);
    T.geo.n_rings = (const int*)lds_put(lds_tab, &off, L.n_rings, nu * 4, copy);
    T.geo.mats = (const int*)lds_put(lds_tab, &off, L.mats, nu * L.mr1 * 4, copy);
    T.geo.radii = (const double*)lds_put(lds_tab, &off, L.radii, nu * L.max_rings * 8, copy);
    const XSView<R> X = xs_view<R>(T0);
    XSView<R> Y;
    Y.sig_t = (const R*)lds_put(lds_tab, &off, X.sig_t, mg * rb, copy);
    Y.nusf = (const R*)lds_put(lds_tab, &off, X.nusf, mg * rb, copy);
    Y.sst = (const R*)lds_put(lds_tab, &off, X.sst, mg * rb, copy);
    Y.cum_chi = (const R*)lds_put(lds_tab, &off, X.cum_chi, mg * rb, copy);
    Y.cum_s = (const R*)lds_put(lds_tab, &off, X.cum_s, mg * T0.G * rb, copy);
    set_xs_view<R>(T, Y);
    T.last_s = (const int*)lds_put(lds_tab, &off, T0.last_s, mg * 4, copy);
    T.last_chi = (const int*)lds_put(lds_tab, &off, T0.last_chi, (size_t)T0.n_mat * 4, copy);
    T.lt = (const double*)lds_put(lds_tab, &off, log_tab(), 2 * MCX_LOG_TAB_N * 8, copy);
    T.sct = (const double*)lds_put(lds_tab, &off, sc_tab(), 4 * MCX_SINCOS_TAB_N * 8, copy);
    // (without a time grid the pointers are set but never read, so that
    // every table access of the kernel stays an LDS access)
    const size_t nte = T0.time ? (size_t)T0.nt + 1 : 0, nsp = T0.time ? (size_t)T0.G : 0;
    T.t_edges = (const double*)lds_put(lds_tab, &off, T0.t_edges, nte * 8, copy);
    T.speed = (const double*)lds_put(lds_tab, &off, T0.speed, nsp * 8, copy);
    __syncthreads();
  }
  return T;
}

// ---------------------------------------------------------------------------
// particle state in registers
// ---------------------------------------------------------------------------

template <class R>
struct Part {
  double x, y;
  R u, v;
  int i, j, r, g;
  uint32_t nsite, ctr, id, nseg;
  double t;  // time since the source pulse (time-dependent mode)
};

template <class R>
__device__ __forceinline__ Part<R> load_part(const Bank& b, uint32_t k) {
  Part<R> p;
  p.x = b.x[k];
  p.y = b.y[k];
  p.u = static_cast<const R*>(b.u)[k];
  p.v = static_cast<const R*>(b.v)[k];
  const uint32_t c = b.cell[k];
  p.i = cell_i(c);
  p.j = cell_j(c);
  p.r = cell_r(c);
  const uint32_t gs = b.gs[k];
  p.g = (int)(gs & 0xFFFFu);
  p.nsite = gs >> 16;
  p.ctr = b.ctr[k];
  p.id = b.id[k];
  p.nseg = b.nseg[k];
  p.t = b.t ? b.t[k] : 0.0;
  return p;
}

template <class R>
__device__ __forceinline__ void store_part(const Bank& b, uint32_t k, const Part<R>& p) {
  b.x[k] = p.x;
  b.y[k] = p.y;
  static_cast<R*>(b.u)[k] = p.u;
  static_cast<R*>(b.v)[k] = p.v;
  b.cell[k] = pack_cell(p.i, p.j, p.r);
  b.gs[k] = (uint32_t)p.g | (p.nsite << 16);
  b.ctr[k] = p.ctr;
  b.id[k] = p.id;
  b.nseg[k] = p.nseg;
  if (b.t) b.t[k] = p.t;
}

enum : int { EV_NONE = 0, EV_COLLIDE = 1, EV_CROSS = 2, EV_LEAK = 3, EV_KILL = 4, EV_CENSUS = 5 };

template <class R, bool REC>
__device__ __forceinline__ void die(const Part<R>& p, int fate, const Accum& A,
                                    const Records& Rc) {
  A.nsite_id[p.id] = p.nsite;
  if (REC) {
    Rc.fate[p.id] = fate;
    Rc.g_final[p.id] = p.g;
    Rc.ctr_final[p.id] = p.ctr;
    Rc.x_final[p.id] = p.x;
    Rc.y_final[p.id] = p.y;
    Rc.t_final[p.id] = p.t;
  }
}

// The block's staged flux words in dynamic LDS (after the table copies):
// per bin the sums of the low and of the high 32-bit halves of its terms.
__device__ __forceinline__ unsigned long long* lds_tally(const Tables& T) {
  extern __shared__ __align__(16) char lds_tab[];
  return reinterpret_cast<unsigned long long*>(lds_tab + T.lds_tally_off);
}

// Zero the block's LDS flux words, lds_bin_n bins (every thread of the block
// calls it).
__device__ __forceinline__ void lds_tally_clear(const Tables& T) {
  unsigned long long* tw = lds_tally(T);
  for (uint32_t w = threadIdx.x; w < 2u * T.lds_bin_n; w += blockDim.x) tw[w] = 0ull;
  __syncthreads();
}

// Add each nonzero bin of the block's LDS flux words to the bin's 128-bit
// pair in the block's stripe of device memory: lo + hi 2^32 exactly, one
// add per bin (every thread of the block calls it).  zero: clear the words
// too (for a window that moves on).
__device__ __forceinline__ void lds_tally_flush(const Tables& T, const Accum& A,
                                                bool zero = false) {
  __syncthreads();
  unsigned long long* tw = lds_tally(T);
  unsigned long long* tb =
      A.tally + (size_t)(blockIdx.x % (unsigned)T.tally_stripes) * (size_t)(2 * T.n_bins) +
      2 * (size_t)T.lds_bin_lo;
  for (uint32_t b = threadIdx.x; b < T.lds_bin_n; b += blockDim.x) {
    const unsigned long long lo = tw[2 * b], hi = tw[2 * b + 1];
    if ((lo | hi) == 0ull) continue;
    const unsigned long long w0 = lo + (hi << 32);
    const unsigned long long w1 = (hi >> 32) + (w0 < lo ? 1ull : 0ull);
    acc_add128(tb + 2 * b, w0, w1);
    if (zero) {
      tw[2 * b] = 0ull;
      tw[2 * b + 1] = 0ull;
    }
  }
  if (zero) __syncthreads();
}

// One exact fixed-point flux term q (< 2^61) of bin `bin`.  TLDS: into the
// block's LDS words as two 32-bit halves (LDS atomics, flushed once per
// block) when the bin is in the block's window, else as below; HALVES: the same halves as two non-returning atomics on the global
// half words; otherwise one returning 64-bit atomic on a 128-bit pair with a
// carry word.
template <bool HALVES, bool TLDS>
__device__ __forceinline__ void flux_term(const Tables& T, unsigned long long* tb,
                                          unsigned long long* tt, int bin, uint64_t q) {
  if constexpr (TLDS) {
    const uint32_t b = (uint32_t)bin - T.lds_bin_lo;
    if (b < T.lds_bin_n) {
      if (q) {
        unsigned long long* w = lds_tally(T);
        atomicAdd(w + 2 * b, (unsigned long long)(q & 0xFFFFFFFFull));
        atomicAdd(w + 2 * b + 1, (unsigned long long)(q >> 32));
      }
    } else {
      acc_add(tb + 2 * bin, q);  // outside the block's window
    }
  } else if constexpr (HALVES) {
    if (q) {
      atomicAdd(tt + 2 * bin, (unsigned long long)(q & 0xFFFFFFFFull));
      atomicAdd(tt + 2 * bin + 1, (unsigned long long)(q >> 32));
    }
  } else {
    acc_add(tb + 2 * bin, q);
  }
}

// One flight: cross-section lookup, distance to collision, distance to the
// bounding surfaces, move, track-length tally, and the surface crossing if
// the boundary comes first.  Returns EV_COLLIDE, EV_CROSS or EV_LEAK.
// HALVES: add the flux term as two non-returning 32-bit-half atomics (the
// tail kernel, where a returning atomic's latency is not hidden by other
// waves); TLDS: into the block's LDS flux words; otherwise one returning
// 64-bit atomic with a carry word.
template <class R, bool REC, bool HALVES, class S = Stream, bool TLDS = false>
__device__ __forceinline__ int segment(const Tables& T, const Geo& L, Part<R>& p, S& rs,
                                       const Accum& A, const Records& Rc, bool* refl_out) {
  const XSView<R> X = xs_view<R>(T);
  const int c = p.j * L.nx + p.i;
  const int un = L.pin_map[c];
  const int nr = L.n_rings[un];
  const int m = L.mats[un * L.mr1 + p.r];
  const R st = X.sig_t[m * T.G + p.g];

  // distance to collision: exponential with mean 1 / sig_t
  const R d_col = draw_dcol<R>(rs, st, T.lt);

  // distance to boundary: the cell's planes ahead and the region's rings
  const double xlo = L.x0 + (double)p.i * L.pitch, xhi = L.x0 + (double)(p.i + 1) * L.pitch;
  const double ylo = L.y0 + (double)p.j * L.pitch, yhi = L.y0 + (double)(p.j + 1) * L.pitch;
  const R tx = Prec<R>::plane(p.x, xlo, xhi, p.u);
  const R ty = Prec<R>::plane(p.y, ylo, yhi, p.v);
  const double cx = L.x0 + ((double)p.i + 0.5) * L.pitch;
  const double cy = L.y0 + ((double)p.j + 0.5) * L.pitch;
  const double dx = p.x - cx, dy = p.y - cy;
  const double u = (double)p.u, v = (double)p.v;
  double t_out = __builtin_inf(), t_in = __builtin_inf();
  if (p.r < nr) t_out = dist_cylinder(dx, dy, u, v, L.radii[un * L.max_rings + p.r], true);
  if (p.r > 0) t_in = dist_cylinder(dx, dy, u, v, L.radii[un * L.max_rings + p.r - 1], false);
  double d_bnd = (double)tx;
  if ((double)ty < d_bnd) d_bnd = (double)ty;
  if (t_out < d_bnd) d_bnd = t_out;
  if (t_in < d_bnd) d_bnd = t_in;

  bool collide = (double)d_col < d_bnd;
  double d = collide ? (double)d_col : d_bnd;
  // time-dependent mode: the flight stops at the end of the time grid if
  // that comes first (census)
  bool census = false;
  double vg = 0.0;
  if (T.time) {
    vg = T.speed[p.g];
    const double d_cen = (T.t_max - p.t) * vg;
    if (d_cen < d) {
      d = d_cen;
      census = true;
      collide = false;
    }
  }
  p.x = p.x + d * u;
  p.y = p.y + d * v;

  // track-length flux tally of this bin (cell, region, group[, time bin]);
  // nu_sig_f is constant in a bin, so the production tally and the
  // track-length k estimator follow from the flux sums at the end of the
  // generation
  const int bin = L.bin_base + ((c * L.mr1 + p.r) * T.G + p.g) * T.nt;
  const size_t stripe_off = (size_t)(blockIdx.x % (unsigned)T.tally_stripes) * (size_t)(2 * T.n_bins);
  unsigned long long* tb = A.tally + stripe_off;
  unsigned long long* tt = A.tally_t + stripe_off;
  if (T.time) {
    // split the flight over the time bins it spans
    double t1 = census ? T.t_max : p.t + d / vg;
    if (t1 > T.t_max) t1 = T.t_max;
    int lo_b = 0, hi_b = T.nt;
    while (hi_b - lo_b > 1) {
      const int mid = lo_b + (hi_b - lo_b) / 2;
      if (T.t_edges[mid] <= p.t)
        lo_b = mid;
      else
        hi_b = mid;
    }
    for (int b = lo_b; b < T.nt; ++b) {
      const double e0 = T.t_edges[b], e1 = T.t_edges[b + 1];
      const double lo = e0 > p.t ? e0 : p.t;
      const double hi = e1 < t1 ? e1 : t1;
      if (hi > lo) {
        flux_term<HALVES, TLDS>(T, tb, tt, bin + b, quantize((hi - lo) * vg, T.q_flux));
      }
      if (e1 >= t1) break;
    }
    p.t = t1;
  } else {
    flux_term<HALVES, TLDS>(T, tb, tt, bin, quantize(d, T.q_flux));
  }
  int k_ev = 0;
  if (REC) {
    k_ev = Rc.n_seg[p.id];
    Rc.n_seg[p.id] += 1;
    Rc.tl_sum[p.id] += d;
  }
  *refl_out = false;
  if (census) {
    if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, 0.0, c, p.r, p.g, 4);
    return EV_CENSUS;
  }
  if (collide) {
    if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, 0.0, c, p.r, p.g, 1);
    return EV_COLLIDE;
  }

  if (REC) Rc.n_cross[p.id] += 1;
  const bool hit_x = (double)tx == d_bnd;
  const bool hit_y = (double)ty == d_bnd;
  if (hit_x || hit_y) {
    const bool out_x = hit_x && (p.u > R(0) ? p.i == L.nx - 1 : p.i == 0);
    const bool out_y = hit_y && (p.v > R(0) ? p.j == L.ny - 1 : p.j == 0);
    const int side_x = p.u > R(0) ? 1 : 0;
    const int side_y = p.v > R(0) ? 3 : 2;
    if ((out_x && L.bc[side_x] == BC_VACUUM) || (out_y && L.bc[side_y] == BC_VACUUM)) {
      if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, 0.0, c, p.r, p.g, 3);
      return EV_LEAK;
    }
    if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, 0.0, c, p.r, p.g, 2);
    bool refl = false;
    if (hit_x) {
      if (out_x) {
        p.u = -p.u;
        refl = true;
      } else {
        p.i += p.u > R(0) ? 1 : -1;
      }
    }
    if (hit_y) {
      if (out_y) {
        p.v = -p.v;
        refl = true;
      } else {
        p.j += p.v > R(0) ? 1 : -1;
      }
    }
    if (REC && refl) Rc.n_refl[p.id] += 1;
    *refl_out = refl;
    // a lattice face lies outside every ring
    p.r = L.n_rings[L.pin_map[p.j * L.nx + p.i]];
  } else {
    if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, 0.0, c, p.r, p.g, 2);
    p.r += t_out == d_bnd ? 1 : -1;
  }
  return EV_CROSS;
}

// Collision, first part: the collision estimator term and the number of
// fission sites floor(nu_sig_f / (sig_t k_used) + xi) (one draw, in fissile
// material of a k-eigenvalue run only).
template <class R>
struct ColXS {
  int m;
  R st, nusf;
};

template <class R>
__device__ __forceinline__ ColXS<R> col_xs(const Tables& T, const Geo& L, const Part<R>& p) {
  const XSView<R> X = xs_view<R>(T);
  const int un = L.pin_map[p.j * L.nx + p.i];
  const int m = L.mats[un * L.mr1 + p.r];
  return ColXS<R>{m, X.sig_t[m * T.G + p.g], X.nusf[m * T.G + p.g]};
}

template <class R, class S>
__device__ __forceinline__ uint32_t fission_count(const Tables& T, const ColXS<R>& x, S& rs,
                                                  double k_used) {
  if (T.fixed_source || !(x.nusf > R(0))) return 0u;
  const R xf = Prec<R>::xi(rs.next());
  const R f = floor(x.nusf / (x.st * (R)k_used) + xf);
  // a nonpositive k_used (only after a failed generation) must not loop forever
  return f < R(65536) ? (uint32_t)(int)f : 65536u;
}

// Collision, second part: write the nf sites reserved at slot, then scatter
// (probability sig_s / sig_t: new group from the scattering row, isotropic
// direction) or absorb.  Returns true if the particle scatters.
template <class R, bool REC, class S>
__device__ __forceinline__ bool collide_rest(const Tables& T, Part<R>& p, S& rs,
                                             const ColXS<R>& x, uint32_t nf, uint32_t slot,
                                             const Accum& A, uint64_t* q_kabs) {
  const XSView<R> X = xs_view<R>(T);
  const int G = T.G;
  for (uint32_t s = 0; s < nf; ++s) {
    const R xs = Prec<R>::xi(rs.next());
    const int gs = sample_cum(xs, X.cum_chi + x.m * G, G, T.last_chi[x.m]);
    const uint32_t k = slot + s;
    if (k < A.fis_cap) {
      A.fis.x[k] = p.x;
      A.fis.y[k] = p.y;
      A.fis.g[k] = gs;
      A.fis.parent[k] = p.id;
      A.fis.seq[k] = p.nsite + s;
    } else {
      atomicOr(A.status, ST_OVERFLOW);
    }
  }
  if (p.nsite + nf > 0xFFFFu) atomicOr(A.status, ST_OVERFLOW);
  p.nsite += nf;
  const R xr = Prec<R>::xi(rs.next());
  const R sst = X.sst[x.m * G + p.g];
  if (xr * x.st < sst) {
    const R xg = Prec<R>::xi(rs.next());
    const int row = x.m * G + p.g;
    p.g = sample_cum(xg, X.cum_s + (size_t)row * G, G, T.last_s[row]);
    draw_iso<R>(rs, &p.u, &p.v, T.sct);
    *q_kabs = 0;
    return true;
  }
  *q_kabs = x.nusf > R(0) ? quantize((double)(x.nusf / (x.st - sst)), T.q_kabs) : 0;
  return false;
}

__device__ __forceinline__ void wave_flag(unsigned long long* base, bool f) {
  const unsigned long long n = (unsigned long long)__popcll(__ballot(f));
  if (lane_id() == 0 && n) atomicAdd(base + (blockIdx.x % STRIPES), n);
}

// ---------------------------------------------------------------------------
// per-history outputs of the persistent and asynchronous engines, reduced
// per problem by k_hist_reduce
// ---------------------------------------------------------------------------

// The problem of global history index h (binary search of the batch).
__device__ __forceinline__ int problem_of(const ProbDesc* P, int n, uint64_t h) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (P[mid].hist_base <= h)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

struct HistOut {
  unsigned long long* kcol;  // [n][2]: sums of the low and high 32-bit halves of q_kcol
  unsigned long long* kabs;  // [n]: q_kabs of the absorption (0 if none)
  uint32_t* cnt;             // [n][HO_N]
};
enum { HO_SEG = 0, HO_COL, HO_CROSS, HO_REFL, HO_SCAT, HO_SITES, HO_FATE, HO_N };

// ---------------------------------------------------------------------------
// source and birth
// ---------------------------------------------------------------------------

// Source site of history id in batch gen: rejection in the lattice's bounding
// box until the point is in fissile material, then a fission-spectrum group
// (FP64 in both precisions).  Returns false (and the lattice corner) when no
// fissile point is found in 10^4 tries.
__device__ __forceinline__ bool sample_source(const Tables& T, const Geo& L, uint64_t seed,
                                              uint64_t prob, uint64_t id, uint32_t gen,
                                              double* sx, double* sy, int32_t* sg) {
  Stream s(seed, TAG_SRC, id, gen, prob, 0);
  for (int t = 0; t < 10000; ++t) {
    const double xa = s.next();
    const double ya = s.next();
    const double x = L.x0 + xa * L.width;
    const double y = L.y0 + ya * L.height;
    int i, j, r;
    locate(L, x, y, &i, &j, &r);
    const int m = L.mats[L.pin_map[j * L.nx + i] * L.mr1 + r];
    if (T.fissile[m]) {
      const double xi = s.next();
      *sx = x;
      *sy = y;
      *sg = sample_cum(xi, T.cum_chi + m * T.G, T.G, T.last_chi[m]);
      return true;
    }
  }
  *sx = L.x0;
  *sy = L.y0;
  *sg = 0;
  return false;
}


__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
  // lds: one slot per wave
  const uint32_t lane = lane_id();
  const uint32_t wid = threadIdx.x / 64u;
  const uint32_t nw = blockDim.x / 64u;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off);
    if ((int)lane >= off) incl += t;
  }
  if (lane == 63) lds[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      const uint32_t t = lds[w];
      lds[w] = run;
      run += t;
    }
    lds[nw] = run;
  }
  __syncthreads();
  const uint32_t r = lds[wid] + incl - v;
  *total = lds[nw];
  __syncthreads();
  return r;
}


// w1 * 2^64 + w0 correctly rounded to double.
__device__ __forceinline__ double u128_to_double(unsigned long long w0, unsigned long long w1) {
  if (w1 == 0) return (double)w0;  // u64 -> f64 conversion rounds to nearest
  // normalise the top 64 bits, fold the rest into a sticky bit
  const int lz = __clzll((long long)w1);
  const unsigned long long top = lz ? ((w1 << lz) | (w0 >> (64 - lz))) : w1;
  const unsigned long long rest = lz ? (w0 << lz) : w0;
  const unsigned long long m = top | (rest ? 1ull : 0ull);
  return ldexp((double)m, 64 - lz);
}

// Sum of striped 128-bit accumulators (hi * 2^64 + lo), correctly rounded
// to double.
__device__ __forceinline__ double stripes_to_double(const unsigned long long* pairs, int n_stripes,
                                    size_t stride) {
  unsigned long long w0 = 0, w1 = 0;  // value = w1 * 2^64 + w0
  for (int s = 0; s < n_stripes; ++s) {
    const unsigned long long lo = pairs[(size_t)s * stride + 0];
    const unsigned long long hi = pairs[(size_t)s * stride + 1];
    const unsigned long long t = w0 + lo;
    w1 += hi + ((t < w0) ? 1ull : 0ull);
    w0 = t;
  }
  return u128_to_double(w0, w1);
}

// Exact flux sum of one bin: the striped 128-bit pairs of the event kernels
// plus the striped (low-half sum, high-half sum) pairs of the tail kernels
// (exact while each of their words takes fewer than 2^32 terms, which the
// flight count of the generation bounds).
__device__ __forceinline__ double flux_total(const unsigned long long* pairs, int n_stripes,
                                             size_t stride, const unsigned long long* halves) {
  unsigned long long w0 = 0, w1 = 0;  // value = w1 * 2^64 + w0
  for (int s = 0; s < n_stripes; ++s) {
    const unsigned long long lo = pairs[(size_t)s * stride + 0];
    const unsigned long long hi = pairs[(size_t)s * stride + 1];
    unsigned long long t = w0 + lo;
    w1 += hi + ((t < w0) ? 1ull : 0ull);
    w0 = t;
    const unsigned long long a = halves[(size_t)s * stride + 0];  // a + b * 2^32
    const unsigned long long b = halves[(size_t)s * stride + 1];
    t = w0 + a;
    w1 += (t < w0) ? 1ull : 0ull;
    w0 = t;
    t = w0 + (b << 32);
    w1 += ((t < w0) ? 1ull : 0ull) + (b >> 32);
    w0 = t;
  }
  return u128_to_double(w0, w1);
}

}  // namespace mcx
