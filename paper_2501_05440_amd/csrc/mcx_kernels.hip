// mcx_kernels.hip - event kernels of one k-eigenvalue generation on gfx950.
//
// Birth, then iterations of {advance, collide} over compacted particle banks
// (the paper's to-be-processed / processed banks, Sec. 2), a history-based
// tail kernel for the last few particles, and the generation-end kernels:
// canonical fission bank, k estimators, Shannon entropy and combing.
//
// Layout: one lane per particle, 64-lane wavefronts.  Particle state is a
// structure of arrays; every event kernel reads a dense bank with coalesced
// loads and appends survivors to dense output banks through wave-aggregated
// atomics (ballot + popcount: one atomic per wave), so each kernel's lanes
// run the same event and no bank is ever read through an index list.
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
  static __device__ __forceinline__ double dcol(double xi, double st) {
    return -cr_log(xi, log_tab()) / st;
  }
  static __device__ __forceinline__ double plane(double x, double lo, double hi, double u) {
    return dist_plane(x, lo, hi, u);
  }
  static __device__ __forceinline__ void iso(double xm, double xp, double* u, double* v) {
    isotropic_uv(xm, xp, u, v);
  }
};

template <>
struct Prec<float> {
  // (float) of a draw may round up to 1; keep it in (0, 1)
  static __device__ __forceinline__ float xi(double u) {
    const float f = (float)u;
    return f < 1.0f ? f : 0x1.fffffep-1f;
  }
  static __device__ __forceinline__ float dcol(float xi, float st) { return -logf(xi) / st; }
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
  static __device__ __forceinline__ void iso(float xm, float xp, float* u, float* v) {
    const float w = 2.0f * xm - 1.0f;
    const float s2 = 1.0f - w * w;
    const float s = sqrtf(s2 > 0.0f ? s2 : 0.0f);
    float sn, cs;
    sincospif(2.0f * xp, &sn, &cs);
    *u = s * cs;
    *v = s * sn;
  }
};

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
// particle state in registers
// ---------------------------------------------------------------------------

template <class R>
struct Part {
  double x, y;
  R u, v;
  int i, j, r, g;
  uint32_t nsite, ctr, id;
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
}

enum : int { EV_NONE = 0, EV_COLLIDE = 1, EV_CROSS = 2, EV_LEAK = 3, EV_KILL = 4 };

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
  }
}

// One flight: cross-section lookup, distance to collision, distance to the
// bounding surfaces, move, track-length tally, and the surface crossing if
// the boundary comes first.  Returns EV_COLLIDE, EV_CROSS or EV_LEAK.
// HALVES: add the flux term as two non-returning 32-bit-half atomics (the
// tail kernel, where a returning atomic's latency is not hidden by other
// waves); otherwise one returning 64-bit atomic with a carry word.
template <class R, bool REC, bool HALVES>
__device__ __forceinline__ int segment(const Tables& T, Part<R>& p, Stream& rs, const Accum& A,
                                       const Records& Rc, bool* refl_out) {
  const XSView<R> X = xs_view<R>(T);
  const int c = p.j * T.nx + p.i;
  const int un = T.pin_map[c];
  const int nr = T.n_rings[un];
  const int m = T.mats[un * T.mr1 + p.r];
  const R st = X.sig_t[m * T.G + p.g];

  // distance to collision: exponential with mean 1 / sig_t
  const R xi = Prec<R>::xi(rs.next());
  const R d_col = Prec<R>::dcol(xi, st);

  // distance to boundary: the cell's planes ahead and the region's rings
  const double xlo = T.x0 + (double)p.i * T.pitch, xhi = T.x0 + (double)(p.i + 1) * T.pitch;
  const double ylo = T.y0 + (double)p.j * T.pitch, yhi = T.y0 + (double)(p.j + 1) * T.pitch;
  const R tx = Prec<R>::plane(p.x, xlo, xhi, p.u);
  const R ty = Prec<R>::plane(p.y, ylo, yhi, p.v);
  const double cx = T.x0 + ((double)p.i + 0.5) * T.pitch;
  const double cy = T.y0 + ((double)p.j + 0.5) * T.pitch;
  const double dx = p.x - cx, dy = p.y - cy;
  const double u = (double)p.u, v = (double)p.v;
  double t_out = __builtin_inf(), t_in = __builtin_inf();
  if (p.r < nr) t_out = dist_cylinder(dx, dy, u, v, T.radii[un * T.max_rings + p.r], true);
  if (p.r > 0) t_in = dist_cylinder(dx, dy, u, v, T.radii[un * T.max_rings + p.r - 1], false);
  double d_bnd = (double)tx;
  if ((double)ty < d_bnd) d_bnd = (double)ty;
  if (t_out < d_bnd) d_bnd = t_out;
  if (t_in < d_bnd) d_bnd = t_in;

  const bool collide = (double)d_col < d_bnd;
  const double d = collide ? (double)d_col : d_bnd;
  p.x = p.x + d * u;
  p.y = p.y + d * v;

  // track-length flux tally of this bin (cell, region, group); nu_sig_f is
  // constant in a bin, so the production tally and the track-length k
  // estimator follow from the flux sums at the end of the generation
  const int bin = (c * T.mr1 + p.r) * T.G + p.g;
  const uint64_t qf = quantize(d, T.q_flux);
  if (HALVES) {
    if (qf) {
      atomicAdd(A.tally_t + 2 * bin, (unsigned long long)(qf & 0xFFFFFFFFull));
      atomicAdd(A.tally_t + 2 * bin + 1, (unsigned long long)(qf >> 32));
    }
  } else {
    unsigned long long* tb =
        A.tally + (size_t)(blockIdx.x % (unsigned)T.tally_stripes) * (size_t)(2 * T.n_bins);
    acc_add(tb + 2 * bin, qf);
  }
  if (REC) {
    Rc.n_seg[p.id] += 1;
    Rc.tl_sum[p.id] += d;
  }
  *refl_out = false;
  if (collide) return EV_COLLIDE;

  if (REC) Rc.n_cross[p.id] += 1;
  const bool hit_x = (double)tx == d_bnd;
  const bool hit_y = (double)ty == d_bnd;
  if (hit_x || hit_y) {
    const bool out_x = hit_x && (p.u > R(0) ? p.i == T.nx - 1 : p.i == 0);
    const bool out_y = hit_y && (p.v > R(0) ? p.j == T.ny - 1 : p.j == 0);
    const int side_x = p.u > R(0) ? 1 : 0;
    const int side_y = p.v > R(0) ? 3 : 2;
    if ((out_x && T.bc[side_x] == BC_VACUUM) || (out_y && T.bc[side_y] == BC_VACUUM))
      return EV_LEAK;
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
    p.r = T.n_rings[T.pin_map[p.j * T.nx + p.i]];
  } else if (t_out == d_bnd) {
    p.r += 1;
  } else {
    p.r -= 1;
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
__device__ __forceinline__ ColXS<R> col_xs(const Tables& T, const Part<R>& p) {
  const XSView<R> X = xs_view<R>(T);
  const int un = T.pin_map[p.j * T.nx + p.i];
  const int m = T.mats[un * T.mr1 + p.r];
  return ColXS<R>{m, X.sig_t[m * T.G + p.g], X.nusf[m * T.G + p.g]};
}

template <class R>
__device__ __forceinline__ uint32_t fission_count(const Tables& T, const ColXS<R>& x, Stream& rs,
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
template <class R, bool REC>
__device__ __forceinline__ bool collide_rest(const Tables& T, Part<R>& p, Stream& rs,
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
    const R xm = Prec<R>::xi(rs.next());
    const R xp = Prec<R>::xi(rs.next());
    Prec<R>::iso(xm, xp, &p.u, &p.v);
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
// source and birth
// ---------------------------------------------------------------------------

// Source site of history id in batch gen: rejection in the lattice's bounding
// box until the point is in fissile material, then a fission-spectrum group
// (FP64 in both precisions).
__global__ void k_source(Tables T, uint32_t gen, uint32_t n, double* sx, double* sy,
                         int32_t* sg, uint32_t* status) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  Stream s(T.seed, TAG_SRC, id, gen, T.prob, 0);
  for (int t = 0; t < 10000; ++t) {
    const double xa = s.next();
    const double ya = s.next();
    const double x = T.x0 + xa * T.width;
    const double y = T.y0 + ya * T.height;
    int i, j, r;
    locate(T, x, y, &i, &j, &r);
    const int m = T.mats[T.pin_map[j * T.nx + i] * T.mr1 + r];
    if (T.fissile[m]) {
      const double xi = s.next();
      sx[id] = x;
      sy[id] = y;
      sg[id] = sample_cum(xi, T.cum_chi + m * T.G, T.G, T.last_chi[m]);
      return;
    }
  }
  atomicOr(status, ST_SOURCE);
  sx[id] = T.x0;
  sy[id] = T.y0;
  sg[id] = 0;
}

// Birth: isotropic direction (transport draws 0 and 1), cell location.
template <class R>
__global__ void k_birth(Tables T, uint32_t gen, uint32_t n, const double* sx, const double* sy,
                        const int32_t* sg, Bank out, uint32_t* cnt_live, uint32_t* cnt_col,
                        const uint32_t* prev_status, uint32_t* status) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  // after a failed generation every later one runs empty
  const bool skip = (prev_status && *prev_status != 0u) || (*status & ST_SOURCE);
  if (id == 0) {
    cnt_live[0] = skip ? 0u : n;
    cnt_live[1] = 0;
    cnt_col[0] = 0;
    if (skip) atomicOr(status, ST_SKIPPED);
  }
  if (skip || id >= n) return;
  Part<R> p;
  p.x = sx[id];
  p.y = sy[id];
  p.g = sg[id];
  Stream rs(T.seed, TAG_TRANSPORT, id, gen, T.prob, 0);
  const R xm = Prec<R>::xi(rs.next());
  const R xp = Prec<R>::xi(rs.next());
  Prec<R>::iso(xm, xp, &p.u, &p.v);
  locate(T, p.x, p.y, &p.i, &p.j, &p.r);
  p.nsite = 0;
  p.ctr = rs.draw;
  p.id = id;
  store_part(out, id, p);
}

// ---------------------------------------------------------------------------
// event kernels
// ---------------------------------------------------------------------------

// Advance every particle of the input bank by one flight.  Particles that
// cross a surface and stay inside go to the live bank of the next iteration,
// particles that collide go to the collision bank; leaks and guard kills end
// here.  Block 0 clears the counters the next iteration appends to.
template <class R, bool REC>
__global__ void __launch_bounds__(1024) k_advance(Tables T, uint32_t gen, uint32_t it, Bank in,
                                                  const uint32_t* __restrict__ n_in_p, Bank live,
                                                  uint32_t* n_live, Bank col, uint32_t* n_col,
                                                  Accum A, Records Rc, uint32_t* clr_live,
                                                  uint32_t* clr_col) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *clr_live = 0;
    *clr_col = 0;
  }
  const uint32_t n_in = *n_in_p;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  int ev = EV_NONE;
  bool refl = false;
  Part<R> p;
  if (k < n_in) {
    p = load_part<R>(in, k);
    if ((int64_t)it >= T.max_events) {
      ev = EV_KILL;
      die<R, REC>(p, FATE_KILLED, A, Rc);
    } else {
      Stream rs(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
      ev = segment<R, REC, false>(T, p, rs, A, Rc, &refl);
      p.ctr = rs.draw;
      if (ev == EV_LEAK) die<R, REC>(p, FATE_LEAKED, A, Rc);
    }
  }
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  uint32_t pl, pc;
  block_append2(ev == EV_CROSS, ev == EV_COLLIDE, n_live, n_col, lds, &pl, &pc);
  if (ev == EV_CROSS) store_part(live, pl, p);
  if (ev == EV_COLLIDE) store_part(col, pc, p);
  wave_flag(A.cnt + CNT_SEG * STRIPES, ev == EV_COLLIDE || ev == EV_CROSS || ev == EV_LEAK);
  wave_flag(A.cnt + CNT_CROSS * STRIPES, ev == EV_CROSS || ev == EV_LEAK);
  wave_flag(A.cnt + CNT_REFL * STRIPES, refl);
  wave_flag(A.cnt + CNT_LEAK * STRIPES, ev == EV_LEAK);
  wave_flag(A.cnt + CNT_KILLED * STRIPES, ev == EV_KILL);
  wave_flag(A.cnt + CNT_ADV_ITEMS * STRIPES, k < n_in);
}

// Process the collision bank: collision estimator, fission-bank append
// (block-aggregated reservation), scatter to the live bank or absorb.
template <class R, bool REC>
__global__ void __launch_bounds__(1024) k_collide(Tables T, uint32_t gen, Bank in,
                                                  const uint32_t* __restrict__ n_in_p, Bank live,
                                                  uint32_t* n_live, Accum A, Records Rc) {
  const uint32_t n_in = *n_in_p;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = k < n_in;
  const double k_used = *A.k_used;
  Part<R> p;
  ColXS<R> x{0, R(1), R(0)};
  uint32_t nf = 0;
  uint64_t q_kcol = 0;
  Stream rs(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
  if (valid) {
    p = load_part<R>(in, k);
    rs = Stream(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    x = col_xs(T, p);
    const double kc = (double)(x.nusf / x.st);
    q_kcol = quantize(kc, T.q_kcol);
    if (REC) {
      Rc.n_col[p.id] += 1;
      Rc.kcol_sum[p.id] += kc;
    }
    nf = fission_count(T, x, rs, k_used);
  }
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  const uint32_t slot = block_reserve(nf, A.n_fis, lds);
  bool alive = false;
  uint64_t q_kabs = 0;
  if (valid) {
    alive = collide_rest<R, REC>(T, p, rs, x, nf, slot, A, &q_kabs);
    p.ctr = rs.draw;
    if (!alive) die<R, REC>(p, FATE_ABSORBED, A, Rc);
  }
  const uint32_t pl = block_reserve(alive ? 1u : 0u, n_live, lds);
  if (alive) store_part(live, pl, p);
  wave_flag(A.cnt + CNT_COL * STRIPES, valid);
  wave_flag(A.cnt + CNT_COL_ITEMS * STRIPES, valid);
  wave_flag(A.cnt + CNT_SCAT * STRIPES, alive);
  wave_flag(A.cnt + CNT_ABS * STRIPES, valid && !alive);
  wave_count(A.cnt + CNT_SITES * STRIPES, nf);
  wave_acc(A.k + K_COL * STRIPES * 2, q_kcol);
  wave_acc(A.k + K_ABS * STRIPES * 2, q_kabs);
}

// History-based finish of the last live particles: one lane runs its
// particle's remaining flights and collisions to the end (the same
// operations as the event kernels, in the same order).
template <class R, bool REC>
__global__ void __launch_bounds__(256) k_tail(Tables T, uint32_t gen, uint32_t it0, Bank in,
                                              const uint32_t* __restrict__ n_in_p, Accum A,
                                              Records Rc) {
  const uint32_t n_in = *n_in_p;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long c_seg = 0, c_col = 0, c_cross = 0, c_refl = 0, c_leak = 0, c_abs = 0,
                     c_kill = 0, c_sites = 0, c_scat = 0;
  unsigned long long kcol[2] = {0, 0}, kabs[2] = {0, 0};
  if (k < n_in) {
    const double k_used = *A.k_used;
    Part<R> p = load_part<R>(in, k);
    Stream rs(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    int64_t nseg = it0;
    for (;;) {
      if (nseg >= T.max_events) {
        p.ctr = rs.draw;
        die<R, REC>(p, FATE_KILLED, A, Rc);
        ++c_kill;
        break;
      }
      bool refl = false;
      const int ev = segment<R, REC, true>(T, p, rs, A, Rc, &refl);
      ++nseg;
      ++c_seg;
      if (ev == EV_LEAK) {
        ++c_cross;
        ++c_leak;
        p.ctr = rs.draw;
        die<R, REC>(p, FATE_LEAKED, A, Rc);
        break;
      }
      if (ev == EV_CROSS) {
        ++c_cross;
        c_refl += refl ? 1 : 0;
        continue;
      }
      ++c_col;
      const ColXS<R> x = col_xs(T, p);
      const double kc = (double)(x.nusf / x.st);
      const uint64_t q = quantize(kc, T.q_kcol);
      kcol[0] += q & 0xFFFFFFFFull;
      kcol[1] += q >> 32;
      if (REC) {
        Rc.n_col[p.id] += 1;
        Rc.kcol_sum[p.id] += kc;
      }
      const uint32_t nf = fission_count(T, x, rs, k_used);
      const uint32_t slot = nf ? atomicAdd(A.n_fis, nf) : 0u;
      c_sites += nf;
      uint64_t qa = 0;
      const bool alive = collide_rest<R, REC>(T, p, rs, x, nf, slot, A, &qa);
      if (!alive) {
        kabs[0] += qa & 0xFFFFFFFFull;
        kabs[1] += qa >> 32;
        ++c_abs;
        p.ctr = rs.draw;
        die<R, REC>(p, FATE_ABSORBED, A, Rc);
        break;
      }
      ++c_scat;
    }
  }
  wave_count(A.cnt + CNT_SEG * STRIPES, c_seg);
  wave_count(A.cnt + CNT_COL * STRIPES, c_col);
  wave_count(A.cnt + CNT_CROSS * STRIPES, c_cross);
  wave_count(A.cnt + CNT_REFL * STRIPES, c_refl);
  wave_count(A.cnt + CNT_LEAK * STRIPES, c_leak);
  wave_count(A.cnt + CNT_ABS * STRIPES, c_abs);
  wave_count(A.cnt + CNT_KILLED * STRIPES, c_kill);
  wave_count(A.cnt + CNT_SITES * STRIPES, c_sites);
  wave_count(A.cnt + CNT_SCAT * STRIPES, c_scat);
  wave_acc_halves(A.k + K_COL * STRIPES * 2, kcol[0], kcol[1]);
  wave_acc_halves(A.k + K_ABS * STRIPES * 2, kabs[0], kabs[1]);
}

// ---------------------------------------------------------------------------
// generation end
// ---------------------------------------------------------------------------

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    p[k] = v;
}

// Exclusive scan of per-history site counts, in three passes over chunks of
// SCAN_CHUNK entries: chunk sums, a one-block scan of the chunk sums, and the
// per-chunk scan.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_PER_THREAD;

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

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_sums(const uint32_t* in, uint32_t n,
                                                            uint32_t* chunk_sum) {
  __shared__ uint32_t lds[SCAN_THREADS / 64 + 1];
  const size_t base = (size_t)blockIdx.x * SCAN_CHUNK;
  uint32_t s = 0;
  for (int e = 0; e < SCAN_PER_THREAD; ++e) {
    const size_t k = base + (size_t)e * SCAN_THREADS + threadIdx.x;
    if (k < n) s += in[k];
  }
  uint32_t total;
  block_excl_scan(s, lds, &total);
  if (threadIdx.x == 0) chunk_sum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024) k_scan_chunks(uint32_t* chunk_sum, uint32_t n_chunks,
                                                      uint32_t* grand_total) {
  __shared__ uint32_t lds[1024 / 64 + 1];
  uint32_t carry = 0;
  for (uint32_t b = 0; b < n_chunks; b += blockDim.x) {
    const uint32_t k = b + threadIdx.x;
    const uint32_t v = k < n_chunks ? chunk_sum[k] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan(v, lds, &total);
    if (k < n_chunks) chunk_sum[k] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *grand_total = carry;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_chunk(const uint32_t* in, uint32_t n,
                                                             const uint32_t* chunk_off,
                                                             uint32_t* out) {
  __shared__ uint32_t lds[SCAN_THREADS / 64 + 1];
  const size_t base = (size_t)blockIdx.x * SCAN_CHUNK;
  // each thread owns SCAN_PER_THREAD consecutive entries
  const size_t t0 = base + (size_t)threadIdx.x * SCAN_PER_THREAD;
  uint32_t v[SCAN_PER_THREAD];
  uint32_t s = 0;
  for (int e = 0; e < SCAN_PER_THREAD; ++e) {
    const size_t k = t0 + e;
    v[e] = k < n ? in[k] : 0u;
    s += v[e];
  }
  uint32_t total;
  uint32_t run = block_excl_scan(s, lds, &total) + chunk_off[blockIdx.x];
  for (int e = 0; e < SCAN_PER_THREAD; ++e) {
    const size_t k = t0 + e;
    if (k < n) out[k] = run;
    run += v[e];
  }
}

// Canonical bank: site s of history parent goes to offset[parent] + seq.
__global__ void k_canon(Sites fis, const uint32_t* n_fis_p, const uint32_t* offs,
                        const uint32_t* nsite_id, uint32_t cap, double* cx, double* cy,
                        int32_t* cg, uint32_t* status) {
  const uint32_t n = min(*n_fis_p, cap);
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    const uint32_t par = fis.parent[s];
    const uint32_t q = fis.seq[s];
    if (q >= nsite_id[par]) {
      atomicOr(status, ST_SITE_SEQ);
      continue;
    }
    const uint32_t pos = offs[par] + q;
    if (pos >= cap) {  // only after an overflow, which the host reports
      atomicOr(status, ST_OVERFLOW);
      continue;
    }
    cx[pos] = fis.x[s];
    cy[pos] = fis.y[s];
    cg[pos] = fis.g[s];
  }
}

// w1 * 2^64 + w0 correctly rounded to double.
__device__ double u128_to_double(unsigned long long w0, unsigned long long w1) {
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
__device__ double stripes_to_double(const unsigned long long* pairs, int n_stripes,
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
// plus the (low-half sum, high-half sum) pair of the tail kernel.
__device__ double flux_total(const unsigned long long* pairs, int n_stripes, size_t stride,
                             const unsigned long long* halves) {
  unsigned long long w0 = 0, w1 = 0;
  for (int s = 0; s < n_stripes; ++s) {
    const unsigned long long lo = pairs[(size_t)s * stride + 0];
    const unsigned long long hi = pairs[(size_t)s * stride + 1];
    const unsigned long long t = w0 + lo;
    w1 += hi + ((t < w0) ? 1ull : 0ull);
    w0 = t;
  }
  const unsigned long long a = halves[0], b = halves[1];  // a + b * 2^32
  unsigned long long t = w0 + a;
  w1 += (t < w0) ? 1ull : 0ull;
  w0 = t;
  t = w0 + (b << 32);
  w1 += ((t < w0) ? 1ull : 0ull) + (b >> 32);
  w0 = t;
  return u128_to_double(w0, w1);
}

// Generation totals: k estimators, counters, next k_used and combing offset.
__global__ void k_gen_totals(Tables T, uint32_t gen, uint32_t n, Accum A, double* gen_k,
                             unsigned long long* gen_cnt, uint32_t* gen_m, double* k_used,
                             double* xi0) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double inv_q[3] = {1.0 / T.q_kcol, 0.0, 1.0 / T.q_kabs};
  for (int e = 0; e < 3; e += 2) {
    const double v = stripes_to_double(A.k + (size_t)e * STRIPES * 2, STRIPES, 2) * inv_q[e];
    gen_k[3 * gen + e] = v / (double)n;
  }
  for (int c = 0; c < N_CNT_ALL; ++c) {
    unsigned long long s = 0;
    for (int t = 0; t < STRIPES; ++t) s += A.cnt[c * STRIPES + t];
    gen_cnt[(size_t)gen * N_CNT_ALL + c] = s;
  }
  gen_m[gen] = *A.n_fis;
  if (!T.fixed_source) *k_used = gen_k[3 * gen + 0];
  Stream rs(T.seed, TAG_RESAMPLE, 0, gen, T.prob, 0);
  *xi0 = rs.next();
}

// Generation tallies per source particle: flux from the exact sums, the
// production nu_sig_f(bin) * flux, and the track-length k estimator as the
// sum of the production over bins (compensated, fixed order; one block).
__global__ void __launch_bounds__(1024) k_gen_tallies(Tables T, uint32_t gen, uint32_t n, Accum A,
                                                      double* gen_tal, double* gen_k) {
  __shared__ double ps[1024], pc[1024];
  const int nb = T.n_bins;
  const int per_cell = T.mr1 * T.G;
  double s = 0.0, cmp = 0.0;  // Neumaier pair of this thread
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const double flux = flux_total(A.tally + 2 * (size_t)b, T.tally_stripes, 2 * (size_t)nb,
                                   A.tally_t + 2 * (size_t)b) /
                        T.q_flux;
    const int cell = b / per_cell;
    const int r = (b / T.G) % T.mr1;
    const int g = b % T.G;
    const int m = T.mats[T.pin_map[cell] * T.mr1 + r];
    const double prod = T.nusf[m * T.G + g] * flux;
    gen_tal[(size_t)gen * 2 * nb + b] = flux / (double)n;
    gen_tal[(size_t)gen * 2 * nb + nb + b] = prod / (double)n;
    const double t = s + prod;
    cmp += fabs(s) >= fabs(prod) ? (s - t) + prod : (prod - t) + s;
    s = t;
  }
  ps[threadIdx.x] = s;
  pc[threadIdx.x] = cmp;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, ac = 0.0;
    for (unsigned k = 0; k < blockDim.x; ++k) {
      const double parts[2] = {ps[k], pc[k]};
      for (int e = 0; e < 2; ++e) {
        const double x = parts[e];
        const double t = a + x;
        ac += fabs(a) >= fabs(x) ? (a - t) + x : (x - t) + a;
        a = t;
      }
    }
    gen_k[3 * gen + 1] = (a + ac) / (double)n;
  }
}

// Shannon entropy of the canonical bank over the entropy mesh: per-block
// histograms in LDS (meshes up to LDS_HIST bins), merged with one global
// atomic per nonzero bin and block.
constexpr int LDS_HIST = 8192;

__global__ void __launch_bounds__(256) k_entropy_hist(Tables T, const double* cx, const double* cy,
                                                     const uint32_t* n_p, uint32_t cap,
                                                     uint32_t* hist) {
  __shared__ uint32_t h[LDS_HIST];
  const int nb = T.ent_nx * T.ent_ny;
  const bool in_lds = nb <= LDS_HIST;
  if (in_lds)
    for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  const uint32_t n = min(*n_p, cap);
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    int bx = (int)floor((cx[s] - T.x0) / T.width * (double)T.ent_nx);
    int by = (int)floor((cy[s] - T.y0) / T.height * (double)T.ent_ny);
    bx = bx < 0 ? 0 : (bx > T.ent_nx - 1 ? T.ent_nx - 1 : bx);
    by = by < 0 ? 0 : (by > T.ent_ny - 1 ? T.ent_ny - 1 : by);
    if (in_lds)
      atomicAdd(&h[by * T.ent_nx + bx], 1u);
    else
      atomicAdd(&hist[by * T.ent_nx + bx], 1u);
  }
  __syncthreads();
  if (in_lds)
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
      if (h[b]) atomicAdd(&hist[b], h[b]);
}

// H = -sum_b p_b log2 p_b: the terms in parallel, the sum in bin order.
__global__ void __launch_bounds__(256) k_entropy_final(Tables T, uint32_t gen,
                                                      const uint32_t* hist, const uint32_t* n_p,
                                                      double* term, double* gen_h) {
  const uint32_t m = *n_p;
  const int nb = T.ent_nx * T.ent_ny;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    double t = 0.0;
    if (m > 0 && hist[b] > 0) {
      const double p = (double)hist[b] / (double)m;
      t = p * log2(p);
    }
    term[b] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double h = 0.0;
    for (int b = 0; b < nb; ++b) h -= term[b];
    gen_h[gen] = h;
  }
}

// Consistency of the generation's bank: scan total equals the number of
// appended sites, and a k-eigenvalue generation banked at least one site.
__global__ void k_gen_check(Tables T, const uint32_t* n_fis, const uint32_t* scan_total,
                            uint32_t* status) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  if (T.fixed_source) return;
  uint32_t st = 0;
  if (*scan_total != *n_fis) st |= ST_SCAN;
  if (*n_fis == 0) st |= ST_EXTINCT;
  if (st) atomicOr(status, st);
}

// Combing: source site i of the next generation is canonical entry
// floor((i + xi0) M / N), capped at M - 1.
__global__ void k_comb(uint32_t n, const uint32_t* m_p, uint32_t cap, const double* xi0_p,
                       const double* cx, const double* cy, const int32_t* cg, double* sx,
                       double* sy, int32_t* sg) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t m = min(*m_p, cap);  // m > cap only after an overflow
  if (m == 0) return;
  const double t = ((double)i + *xi0_p) * (double)m / (double)n;
  uint64_t k = (uint64_t)floor(t);
  if (k > m - 1) k = m - 1;
  sx[i] = cx[k];
  sy[i] = cy[k];
  sg[i] = cg[k];
}

// Active-generation mean and standard deviation of the mean, per bin, and
// of the three k estimators (block 0, thread 0).
__global__ void k_stats(int n_bins2, int n_gen, int n_inactive, const double* gen_tal,
                        double* tal_mean, double* tal_sigma, const double* gen_k,
                        double* k_stat) {
  const int A = n_gen - n_inactive;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n_bins2; b += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int g = n_inactive; g < n_gen; ++g) s += gen_tal[(size_t)g * n_bins2 + b];
    const double mean = s / (double)A;
    double v = 0.0;
    for (int g = n_inactive; g < n_gen; ++g) {
      const double d = gen_tal[(size_t)g * n_bins2 + b] - mean;
      v += d * d;
    }
    tal_mean[b] = mean;
    tal_sigma[b] = A > 1 ? sqrt(v / ((double)A * (double)(A - 1))) : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int e = 0; e < 3; ++e) {
      double s = 0.0;
      for (int g = n_inactive; g < n_gen; ++g) s += gen_k[3 * g + e];
      const double mean = s / (double)A;
      double v = 0.0;
      for (int g = n_inactive; g < n_gen; ++g) {
        const double d = gen_k[3 * g + e] - mean;
        v += d * d;
      }
      k_stat[e] = mean;
      k_stat[3 + e] = A > 1 ? sqrt(v / ((double)A * (double)(A - 1))) : 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// diagnostics
// ---------------------------------------------------------------------------

__global__ void k_diag_math(int which, const double* in, double* out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (which == 0) {
    out[i] = cr_log(in[i], log_tab());
  } else if (which == 1) {
    cr_cossin_2pi(in[i], sc_tab(), &out[2 * i], &out[2 * i + 1]);
  } else if (which == 2) {
    out[i] = sqrt(in[i]);
  } else {
    out[i] = u01((uint64_t)__double_as_longlong(in[i]));
  }
}

__global__ void k_diag_philox(const uint64_t* in, uint64_t* out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t* c = in + 6 * i;
  const u64x4 r = philox4x64_10(c[0], c[1], c[2], c[3], c[4], c[5]);
  for (int k = 0; k < 4; ++k) out[4 * i + k] = r.v[k];
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------

static inline unsigned nblk(uint64_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<uint64_t>(nblk(n, 256), 4096);
  hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_source(const Tables& T, uint32_t gen, uint32_t n, double* sx, double* sy,
                         int32_t* sg, uint32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_source, dim3(nblk(n, 256)), dim3(256), 0, s, T, gen, n, sx, sy, sg,
                     status);
  return hipGetLastError();
}

hipError_t launch_birth(int prec, const Tables& T, uint32_t gen, uint32_t n, const double* sx,
                        const double* sy, const int32_t* sg, const Bank& out, uint32_t* cnt_live,
                        uint32_t* cnt_col, const uint32_t* prev_status, uint32_t* status,
                        hipStream_t s) {
  if (prec == 0)
    hipLaunchKernelGGL(k_birth<double>, dim3(nblk(n, 256)), dim3(256), 0, s, T, gen, n, sx, sy,
                       sg, out, cnt_live, cnt_col, prev_status, status);
  else
    hipLaunchKernelGGL(k_birth<float>, dim3(nblk(n, 256)), dim3(256), 0, s, T, gen, n, sx, sy, sg,
                       out, cnt_live, cnt_col, prev_status, status);
  return hipGetLastError();
}

template <class R, bool REC>
static void advance_k(dim3 g, dim3 b, hipStream_t s, const Tables& T, uint32_t gen, uint32_t it,
                      const Bank& in, const uint32_t* n_in, const Bank& live, uint32_t* n_live,
                      const Bank& col, uint32_t* n_col, const Accum& A, const Records& Rc,
                      uint32_t* clr_live, uint32_t* clr_col) {
  hipLaunchKernelGGL((k_advance<R, REC>), g, b, 0, s, T, gen, it, in, n_in, live, n_live, col,
                     n_col, A, Rc, clr_live, clr_col);
}

hipError_t launch_advance(int prec, bool rec, const Tables& T, uint32_t gen, uint32_t it,
                          const Bank& in, const uint32_t* n_in, const Bank& live,
                          uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                          const Records& Rc, uint32_t* clr_live, uint32_t* clr_col,
                          uint32_t bound, int block, hipStream_t s) {
  const dim3 g(std::max(1u, nblk(bound, block))), b(block);
  if (prec == 0) {
    if (rec)
      advance_k<double, true>(g, b, s, T, gen, it, in, n_in, live, n_live, col, n_col, A, Rc,
                              clr_live, clr_col);
    else
      advance_k<double, false>(g, b, s, T, gen, it, in, n_in, live, n_live, col, n_col, A, Rc,
                               clr_live, clr_col);
  } else {
    if (rec)
      advance_k<float, true>(g, b, s, T, gen, it, in, n_in, live, n_live, col, n_col, A, Rc,
                             clr_live, clr_col);
    else
      advance_k<float, false>(g, b, s, T, gen, it, in, n_in, live, n_live, col, n_col, A, Rc,
                              clr_live, clr_col);
  }
  return hipGetLastError();
}

hipError_t launch_collide(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                          const uint32_t* n_in, const Bank& live, uint32_t* n_live,
                          const Accum& A, const Records& Rc, uint32_t bound, int block,
                          hipStream_t s) {
  const dim3 g(std::max(1u, nblk(bound, block))), b(block);
  if (prec == 0) {
    if (rec)
      hipLaunchKernelGGL((k_collide<double, true>), g, b, 0, s, T, gen, in, n_in, live, n_live, A,
                         Rc);
    else
      hipLaunchKernelGGL((k_collide<double, false>), g, b, 0, s, T, gen, in, n_in, live, n_live,
                         A, Rc);
  } else {
    if (rec)
      hipLaunchKernelGGL((k_collide<float, true>), g, b, 0, s, T, gen, in, n_in, live, n_live, A,
                         Rc);
    else
      hipLaunchKernelGGL((k_collide<float, false>), g, b, 0, s, T, gen, in, n_in, live, n_live, A,
                         Rc);
  }
  return hipGetLastError();
}

hipError_t launch_tail(int prec, bool rec, const Tables& T, uint32_t gen, uint32_t it0,
                       const Bank& in, const uint32_t* n_in, const Accum& A, const Records& Rc,
                       uint32_t bound, hipStream_t s) {
  const dim3 g(std::max(1u, nblk(bound, 64))), b(64);
  if (prec == 0) {
    if (rec)
      hipLaunchKernelGGL((k_tail<double, true>), g, b, 0, s, T, gen, it0, in, n_in, A, Rc);
    else
      hipLaunchKernelGGL((k_tail<double, false>), g, b, 0, s, T, gen, it0, in, n_in, A, Rc);
  } else {
    if (rec)
      hipLaunchKernelGGL((k_tail<float, true>), g, b, 0, s, T, gen, it0, in, n_in, A, Rc);
    else
      hipLaunchKernelGGL((k_tail<float, false>), g, b, 0, s, T, gen, it0, in, n_in, A, Rc);
  }
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* in, uint32_t n, uint32_t* chunk_sum, uint32_t* out,
                       uint32_t* total, hipStream_t s) {
  const uint32_t nc = nblk(n, SCAN_CHUNK);
  hipLaunchKernelGGL(k_scan_sums, dim3(nc), dim3(SCAN_THREADS), 0, s, in, n, chunk_sum);
  hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, s, chunk_sum, nc, total);
  hipLaunchKernelGGL(k_scan_chunk, dim3(nc), dim3(SCAN_THREADS), 0, s, in, n, chunk_sum, out);
  return hipGetLastError();
}

uint32_t scan_chunks(uint32_t n) { return nblk(n, SCAN_CHUNK); }

hipError_t launch_gen_check(const Tables& T, const uint32_t* n_fis, const uint32_t* scan_total,
                            uint32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_check, dim3(1), dim3(64), 0, s, T, n_fis, scan_total, status);
  return hipGetLastError();
}

hipError_t launch_canon(const Sites& fis, const uint32_t* n_fis, const uint32_t* offs,
                        const uint32_t* nsite_id, uint32_t cap, double* cx, double* cy,
                        int32_t* cg, uint32_t* status, uint32_t bound, hipStream_t s) {
  const unsigned g = std::max(1u, std::min(nblk(bound, 256), 8192u));
  hipLaunchKernelGGL(k_canon, dim3(g), dim3(256), 0, s, fis, n_fis, offs, nsite_id, cap, cx, cy,
                     cg, status);
  return hipGetLastError();
}

hipError_t launch_gen_totals(const Tables& T, uint32_t gen, uint32_t n, const Accum& A,
                             double* gen_k, unsigned long long* gen_cnt, uint32_t* gen_m,
                             double* k_used, double* xi0, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_totals, dim3(1), dim3(64), 0, s, T, gen, n, A, gen_k, gen_cnt, gen_m,
                     k_used, xi0);
  return hipGetLastError();
}

hipError_t launch_gen_tallies(const Tables& T, uint32_t gen, uint32_t n, const Accum& A,
                              double* gen_tal, double* gen_k, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_tallies, dim3(1), dim3(1024), 0, s, T, gen, n, A, gen_tal, gen_k);
  return hipGetLastError();
}

hipError_t launch_entropy(const Tables& T, uint32_t gen, const double* cx, const double* cy,
                          const uint32_t* n_p, uint32_t cap, uint32_t* hist, double* term,
                          double* gen_h, uint32_t bound, hipStream_t s) {
  const unsigned g = std::max(1u, std::min(nblk(bound, 256 * 16), 1024u));
  hipLaunchKernelGGL(k_entropy_hist, dim3(g), dim3(256), 0, s, T, cx, cy, n_p, cap, hist);
  hipLaunchKernelGGL(k_entropy_final, dim3(1), dim3(256), 0, s, T, gen, hist, n_p, term, gen_h);
  return hipGetLastError();
}

hipError_t launch_comb(uint32_t n, const uint32_t* m_p, uint32_t cap, const double* xi0,
                       const double* cx, const double* cy, const int32_t* cg, double* sx,
                       double* sy, int32_t* sg, hipStream_t s) {
  hipLaunchKernelGGL(k_comb, dim3(nblk(n, 256)), dim3(256), 0, s, n, m_p, cap, xi0, cx, cy, cg,
                     sx, sy, sg);
  return hipGetLastError();
}

hipError_t launch_stats(int n_bins2, int n_gen, int n_inactive, const double* gen_tal,
                        double* tal_mean, double* tal_sigma, const double* gen_k, double* k_stat,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_stats, dim3(std::max(1u, nblk(n_bins2, 256))), dim3(256), 0, s, n_bins2,
                     n_gen, n_inactive, gen_tal, tal_mean, tal_sigma, gen_k, k_stat);
  return hipGetLastError();
}

hipError_t launch_diag_math(int which, const double* in, double* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_math, dim3(nblk(n, 256)), dim3(256), 0, s, which, in, out, n);
  return hipGetLastError();
}

hipError_t launch_diag_philox(const uint64_t* in, uint64_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_philox, dim3(nblk(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

void host_math(int which, const double* in, double* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    if (which == 0) {
      out[i] = cr_log(in[i], log_tab());
    } else if (which == 1) {
      cr_cossin_2pi(in[i], sc_tab(), &out[2 * i], &out[2 * i + 1]);
    } else if (which == 2) {
      out[i] = sqrt(in[i]);
    } else {
      out[i] = u01(as_u64(in[i]));
    }
  }
}

}  // namespace mcx
