// mcx_ce.hip - continuous-energy event kernels (FP64 and FP32-mixed).
//
// The continuous-energy form of the method's physics (Sec. 1 lists it among
// the capabilities; Sec. 4 runs a continuous-energy pin cell; Sec. 5 notes
// that cross-section lookup and interpolation dominate it).  The kernels
// keep the event structure of the multigroup path (source, birth, advance
// with up to `flights` flights, collide, history-based tail) and change the
// physics:
//   lookup   the interval of the shared energy grid (the index a bisection
//            returns, found from a bucket of the energy's bit pattern and a
//            short bisection inside it), then Sigma_x(E) = sum over the
//            material's nuclides of N_k (s_k(E_i) + f (s_k(E_i+1) - s_k(E_i))),
//            f the clipped interpolation fraction; the flights read (sig_t,
//            sig_f) pairs packed by [material][grid point][nuclide], so one
//            lookup of a material is one contiguous block, and a collision
//            reads sig_s of the sampled nuclide from a separate table in the
//            same order;
//   flight   d_col = -ln(xi) / Sigma_t(E); flux tallied per (cell, region,
//            energy bin); the track-length k term d nu Sigma_f(E) summed
//            exactly;
//   collide  fission sites with Watt energies, the nuclide by its share of
//            Sigma_t, elastic scattering off it at rest (centre-of-mass
//            isotropic) with the direction turned about itself, or
//            absorption; a scatter below the cutoff energy ends the history.
// In FP64 every operation repeats the CPU oracle's, in the same order, so
// histories are identical.  In FP32-mixed (R = float) the energy, the
// directions, the cross sections and their interpolation, the distance to
// collision and the plane distances, the reaction comparisons and the Watt
// and scattering kinematics are binary32; positions, the cylinder quadratic,
// the move, the tallies and the estimators stay binary64.
#include "mcx_kernels_common.hpp"

namespace mcx {

template <class R>
struct PartCE {
  double x, y;
  R u, v, w, e;
  int i, j, r;
  uint32_t nsite, ctr, id, nseg;
  double t;  // time since the source pulse (time-dependent mode)
};

// Speed (cm/s) of a neutron of kinetic energy e (eV): c sqrt(2 e / m c^2),
// c = 2.99792458e10 cm/s, m c^2 = 939.56542052e6 eV (binary64 in both
// precisions, like the time it advances).
__device__ __forceinline__ double neutron_speed(double e) {
  return 2.99792458e10 * sqrt(2.0 * e / 939.56542052e6);
}

template <class R>
__device__ __forceinline__ PartCE<R> load_ce(const Bank& b, uint32_t k) {
  PartCE<R> p;
  p.x = b.x[k];
  p.y = b.y[k];
  p.u = static_cast<const R*>(b.u)[k];
  p.v = static_cast<const R*>(b.v)[k];
  p.w = static_cast<const R*>(b.w)[k];
  p.e = static_cast<const R*>(b.e)[k];
  const uint32_t c = b.cell[k];
  p.i = cell_i(c);
  p.j = cell_j(c);
  p.r = cell_r(c);
  p.nsite = b.gs[k] >> 16;
  p.ctr = b.ctr[k];
  p.id = b.id[k];
  p.nseg = b.nseg[k];
  p.t = b.t ? b.t[k] : 0.0;
  return p;
}

template <class R>
__device__ __forceinline__ void store_ce(const Bank& b, uint32_t k, const PartCE<R>& p) {
  b.x[k] = p.x;
  b.y[k] = p.y;
  static_cast<R*>(b.u)[k] = p.u;
  static_cast<R*>(b.v)[k] = p.v;
  static_cast<R*>(b.w)[k] = p.w;
  static_cast<R*>(b.e)[k] = p.e;
  b.cell[k] = pack_cell(p.i, p.j, p.r);
  b.gs[k] = p.nsite << 16;
  b.ctr[k] = p.ctr;
  b.id[k] = p.id;
  b.nseg[k] = p.nseg;
  if (b.t) b.t[k] = p.t;
}

// Precision policy of the continuous-energy path: the tables and the
// transcendental functions of the working precision.
template <class R>
struct CEP;

template <>
struct CEP<double> {
  static __device__ __forceinline__ const double* grid(const Tables& T) { return T.e_grid; }
  static __device__ __forceinline__ const double* edges(const Tables& T) { return T.e_edges; }
  static __device__ __forceinline__ const double* dens(const Tables& T) { return T.mat_dens; }
  static __device__ __forceinline__ const double* awr(const Tables& T) { return T.awr; }
  static __device__ __forceinline__ double log(double x) { return cr_log(x, log_tab()); }
  static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ void cossin_2pi(double t, double* c, double* s) {
    cr_cossin_2pi(t, sc_tab(), c, s);
  }
  // one interval of nuclide k of material m: t and f at both ends (one
  // 16-byte load per grid point), interpolated
  static __device__ __forceinline__ void micro_tf(const Tables& T, int m, int k, int gi, double f,
                                                  double* t, double* fi) {
    const size_t e = ((size_t)m * T.n_pts + gi) * T.max_nuc + k;
    const double2* a = reinterpret_cast<const double2*>(T.ce_tf) + e;
    const double2 tf0 = a[0], tf1 = a[T.max_nuc];
    *t = tf0.x + f * (tf1.x - tf0.x);
    *fi = tf0.y + f * (tf1.y - tf0.y);
  }
  // the same for s
  static __device__ __forceinline__ double micro_s(const Tables& T, int m, int k, int gi,
                                                   double f) {
    const size_t e = ((size_t)m * T.n_pts + gi) * T.max_nuc + k;
    const double s0 = T.ce_s[e], s1 = T.ce_s[e + T.max_nuc];
    return s0 + f * (s1 - s0);
  }
  static constexpr double rot_eps = 1e-10;
};

template <>
struct CEP<float> {
  static __device__ __forceinline__ const float* grid(const Tables& T) { return T.e_grid_f; }
  static __device__ __forceinline__ const float* edges(const Tables& T) { return T.e_edges_f; }
  static __device__ __forceinline__ const float* dens(const Tables& T) { return T.mat_dens_f; }
  static __device__ __forceinline__ const float* awr(const Tables& T) { return T.awr_f; }
  static __device__ __forceinline__ float log(float x) { return logf(x); }
  static __device__ __forceinline__ float sqrt(float x) { return sqrtf(x); }
  static __device__ __forceinline__ void cossin_2pi(float t, float* c, float* s) {
    sincospif(2.0f * t, s, c);
  }
  static __device__ __forceinline__ void micro_tf(const Tables& T, int m, int k, int gi, float f,
                                                  float* t, float* fi) {
    const size_t e = ((size_t)m * T.n_pts + gi) * T.max_nuc + k;
    const float2* a = reinterpret_cast<const float2*>(T.ce_tf_f) + e;
    const float2 p0 = a[0], p1 = a[T.max_nuc];
    *t = p0.x + f * (p1.x - p0.x);
    *fi = p0.y + f * (p1.y - p0.y);
  }
  static __device__ __forceinline__ float micro_s(const Tables& T, int m, int k, int gi, float f) {
    const size_t e = ((size_t)m * T.n_pts + gi) * T.max_nuc + k;
    const float s0 = T.ce_s_f[e], s1 = T.ce_s_f[e + T.max_nuc];
    return s0 + f * (s1 - s0);
  }
  // binary32 loses 1 - w^2 to cancellation much earlier than binary64
  static constexpr float rot_eps = 1e-4f;
};

// Largest i with grid[i] <= e, within [0, n - 2] (bisection; the index is
// unique, so in FP64 it equals the CPU oracle's).
template <class R>
__device__ __forceinline__ int ce_interval(const R* __restrict__ grid, int n, R e) {
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

// The grid interval of e found from the bucket of its bit pattern: for
// positive floating-point numbers the bit pattern increases with the value,
// so bucket (bits(e) - bits(E_0)) >> shift brackets the interval between two
// precomputed start points and a short bisection finishes it.  Returns the
// same index as the bisection over the whole grid.
template <class R>
struct Bits;
template <>
struct Bits<double> {
  static __device__ __forceinline__ uint64_t of(double x) { return (uint64_t)__double_as_longlong(x); }
};
template <>
struct Bits<float> {
  static __device__ __forceinline__ uint64_t of(float x) { return (uint64_t)(uint32_t)__float_as_uint(x); }
};

template <class R>
__device__ __forceinline__ int ce_interval_hashed(const R* __restrict__ grid, int n, R e,
                                                  const int* __restrict__ hash, int n_hash,
                                                  int shift, uint64_t base) {
  if (!(e > grid[0])) return 0;
  uint64_t key = (Bits<R>::of(e) - base) >> shift;
  if (key > (uint64_t)(n_hash - 1)) key = (uint64_t)(n_hash - 1);
  int lo = hash[key];
  int hi = hash[key + 1] + 1;
  if (hi > n - 1) hi = n - 1;
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (grid[mid] <= e)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <class R>
__device__ __forceinline__ int grid_interval(const Tables& T, R e);
template <>
__device__ __forceinline__ int grid_interval<double>(const Tables& T, double e) {
  return ce_interval_hashed<double>(T.e_grid, T.n_pts, e, T.e_hash, T.n_hash, T.hash_shift,
                                    T.hash_base);
}
template <>
__device__ __forceinline__ int grid_interval<float>(const Tables& T, float e) {
  return ce_interval_hashed<float>(T.e_grid_f, T.n_pts, e, T.e_hash_f, T.n_hash_f,
                                   T.hash_shift_f, T.hash_base_f);
}

template <class R>
struct CEXS {
  R st, sf;      // macroscopic total, fission
  int gi;        // grid interval
  R f;           // interpolation fraction
};

// Grid interval of e and the interpolation fraction in it.
template <class R>
__device__ __forceinline__ void ce_locate(const Tables& T, R e, int* gi, R* fr) {
  const R* grid = CEP<R>::grid(T);
  *gi = grid_interval<R>(T, e);
  const R e0 = grid[*gi], e1 = grid[*gi + 1];
  R f = (e - e0) / (e1 - e0);
  if (f < R(0)) f = R(0);
  if (f > R(1)) f = R(1);
  *fr = f;
}

// Macroscopic total and fission cross sections of material m at (gi, f).
template <class R>
__device__ __forceinline__ void ce_sums(const Tables& T, int m, int gi, R fr, R* st_out,
                                        R* sf_out) {
  R st = R(0), sf = R(0);
  const int nn = T.mat_n[m];
  const R* dens = CEP<R>::dens(T);
  for (int k = 0; k < nn; ++k) {
    const R d = dens[m * T.max_nuc + k];
    R t, fi;
    CEP<R>::micro_tf(T, m, k, gi, fr, &t, &fi);
    st = st + d * t;
    sf = sf + d * fi;
  }
  *st_out = st;
  *sf_out = sf;
}

// Macroscopic total and fission cross sections at e.
template <class R>
__device__ __forceinline__ CEXS<R> ce_macro(const Tables& T, int m, R e) {
  CEXS<R> x;
  ce_locate<R>(T, e, &x.gi, &x.f);
  ce_sums<R>(T, m, x.gi, x.f, &x.st, &x.sf);
  return x;
}

// The lookups of the last energy: its interval and the sums of the last two
// materials at it.  A particle keeps its energy from one collision to the
// next, so the flights in between that stay in, or come back to, a
// material (ring crossings, reflections) reuse them; the values are the ones
// a new lookup computes.
template <class R>
struct CECache {
  R e;  // energy of gi and f, -1 when empty
  int gi;
  R f;
  int m0, m1, next;
  R st0, sf0, st1, sf1;
};

template <class R>
__device__ __forceinline__ void ce_cache_clear(CECache<R>& c) {
  c.e = R(-1);
  c.m0 = -1;
  c.m1 = -1;
  c.next = 0;
}

template <class R>
__device__ __forceinline__ CEXS<R> ce_macro_cached(const Tables& T, int m, R e, CECache<R>& c) {
  CEXS<R> x;
  if (!(c.e == e)) {
    ce_locate<R>(T, e, &c.gi, &c.f);
    c.e = e;
    c.m0 = -1;
    c.m1 = -1;
  }
  x.gi = c.gi;
  x.f = c.f;
  if (c.m0 == m) {
    x.st = c.st0;
    x.sf = c.sf0;
  } else if (c.m1 == m) {
    x.st = c.st1;
    x.sf = c.sf1;
  } else {
    ce_sums<R>(T, m, x.gi, x.f, &x.st, &x.sf);
    if (c.next == 0) {
      c.m0 = m;
      c.st0 = x.st;
      c.sf0 = x.sf;
    } else {
      c.m1 = m;
      c.st1 = x.st;
      c.sf1 = x.sf;
    }
    c.next ^= 1;
  }
  return x;
}

// Macroscopic scattering cross section at the interval and fraction of x.
template <class R>
__device__ __forceinline__ R ce_macro_s(const Tables& T, int m, const CEXS<R>& x) {
  R ss = R(0);
  const int nn = T.mat_n[m];
  const R* dens = CEP<R>::dens(T);
  for (int k = 0; k < nn; ++k) {
    const R d = dens[m * T.max_nuc + k];
    ss = ss + d * CEP<R>::micro_s(T, m, k, x.gi, x.f);
  }
  return ss;
}

// One attempt of the Watt sampler: a Maxwellian W of temperature a from
// three draws, W = -a (ln x1 + ln x2 cos^2(pi x3 / 2)), then
// E = W + a^2 b / 4 + (2 x4 - 1) sqrt(a^2 b W).
template <class R>
__device__ __forceinline__ R watt_attempt(R a, R b, R x1, R x2, R x3, R x4) {
  R c, s;
  CEP<R>::cossin_2pi(R(0.25) * x3, &c, &s);
  const R w = -a * (CEP<R>::log(x1) + CEP<R>::log(x2) * (c * c));
  const R q = a * a * b;
  return (w + R(0.25) * q) + (R(2) * x4 - R(1)) * CEP<R>::sqrt(q * w);
}

// Watt energy: attempts of four draws until one lies in (0, e_max].
template <class R, class S>
__device__ __forceinline__ R watt_sample(const Tables& T, S& s) {
  const R a = (R)T.watt_a, b = (R)T.watt_b, e_max = (R)T.e_max;
  for (int t = 0; t < 10000; ++t) {
    const R x1 = Prec<R>::xi(s.next());
    const R x2 = Prec<R>::xi(s.next());
    const R x3 = Prec<R>::xi(s.next());
    const R x4 = Prec<R>::xi(s.next());
    const R e = watt_attempt<R>(a, b, x1, x2, x3, x4);
    if (e > R(0) && e <= e_max) return e;
  }
  return e_max;
}

// Elastic scattering off a target of mass ratio awr at rest, isotropic in
// the centre-of-mass frame: outgoing energy and lab cosine.
template <class R>
__device__ __forceinline__ R elastic(R awr, R e, R xi_mu, R* mu_lab) {
  const R mu = R(2) * xi_mu - R(1);
  const R num = (awr * awr + R(2) * awr * mu) + R(1);
  const R ap1 = awr + R(1);
  *mu_lab = (R(1) + awr * mu) / CEP<R>::sqrt(num);
  return e * num / (ap1 * ap1);
}

// Turn (u, v, w) by the polar cosine mu about itself, azimuth 2 pi xi_phi;
// near the z axis (1 - w^2 at most rot_eps), x takes z's role.
template <class R>
__device__ __forceinline__ void rotate(R mu, R xi_phi, R* pu, R* pv, R* pw) {
  R c, s;
  CEP<R>::cossin_2pi(xi_phi, &c, &s);
  const R u = *pu, v = *pv, w = *pw;
  R sm = R(1) - mu * mu;
  sm = sm > R(0) ? CEP<R>::sqrt(sm) : R(0);
  const R a = R(1) - w * w;
  // new values in locals, stored once (stores through the pointers in two
  // orders put the particle in scratch memory)
  R nu, nv, nw;
  if (a > CEP<R>::rot_eps) {
    const R t = CEP<R>::sqrt(a);
    nu = mu * u + sm * (u * w * c - v * s) / t;
    nv = mu * v + sm * (v * w * c + u * s) / t;
    nw = mu * w - sm * t * c;
  } else {
    const R t = CEP<R>::sqrt(R(1) - u * u);
    nv = mu * v + sm * (v * u * c - w * s) / t;
    nw = mu * w + sm * (w * u * c + v * s) / t;
    nu = mu * u - sm * t * c;
  }
  *pu = nu;
  *pv = nv;
  *pw = nw;
}

// Source site: rejection in the lattice box (FP64) until the point is
// fissile, then a Watt energy from the same stream.
template <class R>
__device__ __forceinline__ bool sample_source_ce(const Tables& T, const Geo& L, uint64_t seed,
                                                 uint64_t prob, uint64_t id, uint32_t gen,
                                                 double* sx, double* sy, double* se) {
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
      *sx = x;
      *sy = y;
      *se = T.src_energy > 0.0 ? T.src_energy : (double)watt_sample<R>(T, s);
      return true;
    }
  }
  *sx = L.x0;
  *sy = L.y0;
  *se = T.e_max;
  return false;
}

template <class R, bool REC>
__device__ __forceinline__ void die_ce(const PartCE<R>& p, int fate, const Accum& A,
                                       const Records& Rc, const Tables& T) {
  A.nsite_id[p.id] = p.nsite;
  if (REC) {
    Rc.fate[p.id] = fate;
    Rc.g_final[p.id] = ce_interval<R>(CEP<R>::edges(T), T.n_ebins + 1, p.e);
    Rc.ctr_final[p.id] = p.ctr;
    Rc.x_final[p.id] = p.x;
    Rc.y_final[p.id] = p.y;
    Rc.e_final[p.id] = (double)p.e;
    Rc.t_final[p.id] = p.t;
  }
}

// Add a fixed-point term to the pair (lo, hi) of bin `bin` of a striped
// accumulator: one returning 64-bit atomic with carry, or (HALVES, the tail
// kernel) two non-returning atomics on the low and high 32-bit halves.
template <bool HALVES>
__device__ __forceinline__ void tally_add(unsigned long long* pairs, unsigned long long* halves,
                                          size_t stripe_off, int bin, uint64_t q) {
  if (HALVES) {
    if (q) {
      atomicAdd(halves + stripe_off + 2 * bin, (unsigned long long)(q & 0xFFFFFFFFull));
      atomicAdd(halves + stripe_off + 2 * bin + 1, (unsigned long long)(q >> 32));
    }
  } else {
    acc_add(pairs + stripe_off + 2 * bin, q);
  }
}

// One flight at the particle's energy (see the multigroup segment for the
// geometry).  *q_tl receives the fixed-point track-length k term.
template <class R, bool REC, bool HALVES, bool TLDS = false>
__device__ __forceinline__ int segment_ce(const Tables& T, const Geo& L, PartCE<R>& p, Stream& rs,
                                          const Accum& A, const Records& Rc, bool* refl_out,
                                          uint64_t* q_tl, CECache<R>& cache) {
  const int c = p.j * L.nx + p.i;
  const int un = L.pin_map[c];
  const int nr = L.n_rings[un];
  const int m = L.mats[un * L.mr1 + p.r];
  const CEXS<R> X = ce_macro_cached<R>(T, m, p.e, cache);
  const R st = X.st;
  const R nusf = (R)T.nu * X.sf;

  const R xi = Prec<R>::xi(rs.next());
  const R d_col = Prec<R>::dcol(xi, st);

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
  // that comes first (census); it flies at the speed of its energy
  bool census = false;
  double ve = 0.0;
  if (T.time) {
    ve = neutron_speed((double)p.e);
    const double d_cen = (T.t_max - p.t) * ve;
    if (d_cen < d) {
      d = d_cen;
      census = true;
      collide = false;
    }
  }
  p.x = p.x + d * u;
  p.y = p.y + d * v;

  // flux per (cell, region, energy bin[, time bin]); time-dependent: the
  // length flown and the time spent (density) in each time bin it spans
  const int b = ce_interval<R>(CEP<R>::edges(T), T.n_ebins + 1, p.e);
  const int bin = L.bin_base + ((c * L.mr1 + p.r) * T.n_ebins + b) * T.nt;
  const size_t stripe_off = (size_t)(blockIdx.x % (unsigned)T.tally_stripes) * (size_t)(2 * T.n_bins);
  if (T.time) {
    double t1 = census ? T.t_max : p.t + d / ve;
    if (t1 > T.t_max) t1 = T.t_max;
    int lo_b = 0, hi_b = T.nt;
    while (hi_b - lo_b > 1) {
      const int mid = lo_b + (hi_b - lo_b) / 2;
      if (T.t_edges[mid] <= p.t)
        lo_b = mid;
      else
        hi_b = mid;
    }
    for (int q = lo_b; q < T.nt; ++q) {
      const double e0 = T.t_edges[q], e1 = T.t_edges[q + 1];
      const double lo = e0 > p.t ? e0 : p.t;
      const double hi = e1 < t1 ? e1 : t1;
      if (hi > lo) {
        tally_add<HALVES>(A.tally, A.tally_t, stripe_off, bin + q, quantize((hi - lo) * ve, T.q_flux));
        tally_add<HALVES>(A.dens, A.dens_t, stripe_off, bin + q, quantize(hi - lo, T.q_dens));
      }
      if (e1 >= t1) break;
    }
    p.t = t1;
  } else if constexpr (TLDS) {
    // the block's LDS flux words (halves), added to device memory once per block
    const uint64_t q = quantize(d, T.q_flux);
    if (q) {
      unsigned long long* w = lds_tally(T);
      atomicAdd(w + 2 * bin, (unsigned long long)(q & 0xFFFFFFFFull));
      atomicAdd(w + 2 * bin + 1, (unsigned long long)(q >> 32));
    }
  } else {
    tally_add<HALVES>(A.tally, A.tally_t, stripe_off, bin, quantize(d, T.q_flux));
  }
  *q_tl = quantize(d * (double)nusf, T.q_ktl);
  int k_ev = 0;
  if (REC) {
    k_ev = Rc.n_seg[p.id];
    Rc.n_seg[p.id] += 1;
    Rc.tl_sum[p.id] += d;
  }
  *refl_out = false;
  if (census) {
    if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, (double)p.e, c, p.r, b, 4);
    return EV_CENSUS;
  }
  if (collide) {
    if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, (double)p.e, c, p.r, b, 1);
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
      if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, (double)p.e, c, p.r, b, 3);
      return EV_LEAK;
    }
    if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, (double)p.e, c, p.r, b, 2);
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
    p.r = L.n_rings[L.pin_map[p.j * L.nx + p.i]];
  } else {
    if (REC) log_flight(Rc, p.id, k_ev, p.x, p.y, d, (double)p.e, c, p.r, b, 2);
    p.r += t_out == d_bnd ? 1 : -1;
  }
  return EV_CROSS;
}

// Collision, first part: cross sections at the collision energy, the
// collision-estimator term and the number of fission sites.
template <class R>
struct ColCE {
  int m;
  CEXS<R> x;
  R nusf;
};

// The collision point's material and lookup: from the flight's cache (the
// tail kernel) or as stored with the particle by the flight kernel.
template <class R>
__device__ __forceinline__ ColCE<R> col_ce(const Tables& T, const Geo& L, const PartCE<R>& p,
                                           CECache<R>& cache) {
  ColCE<R> c;
  const int un = L.pin_map[p.j * L.nx + p.i];
  c.m = L.mats[un * L.mr1 + p.r];
  c.x = ce_macro_cached<R>(T, c.m, p.e, cache);
  c.nusf = (R)T.nu * c.x.sf;
  return c;
}

template <class R>
__device__ __forceinline__ ColCE<R> col_ce_stored(const Tables& T, const Geo& L,
                                                  const PartCE<R>& p, const Bank& b, uint32_t k) {
  ColCE<R> c;
  const int un = L.pin_map[p.j * L.nx + p.i];
  c.m = L.mats[un * L.mr1 + p.r];
  c.x.gi = b.xgi[k];
  c.x.f = static_cast<const R*>(b.xf)[k];
  c.x.st = static_cast<const R*>(b.xst)[k];
  c.x.sf = static_cast<const R*>(b.xsf)[k];
  c.nusf = (R)T.nu * c.x.sf;
  return c;
}

template <class R, class S>
__device__ __forceinline__ uint32_t fission_count_ce(const Tables& T, const ColCE<R>& c,
                                                     S& rs, double k_used) {
  if (T.fixed_source || !(c.nusf > R(0))) return 0u;
  const R xf = Prec<R>::xi(rs.next());
  const R f = floor(c.nusf / (c.x.st * (R)k_used) + xf);
  return f < R(65536) ? (uint32_t)(int)f : 65536u;
}

// Collision, second part: the nf sites reserved at slot (Watt energies),
// the nuclide, then elastic scatter or absorption.  Returns FATE_ALIVE after
// a scatter above the cutoff, FATE_CUTOFF or FATE_ABSORBED.
template <class R, class S>
__device__ __forceinline__ int collide_rest_ce(const Tables& T, PartCE<R>& p, S& rs,
                                               const ColCE<R>& c, uint32_t nf, uint32_t slot,
                                               const Accum& A, uint64_t* q_kabs) {
  for (uint32_t s = 0; s < nf; ++s) {
    const R es = watt_sample<R>(T, rs);
    const uint32_t k = slot + s;
    if (k < A.fis_cap) {
      A.fis.x[k] = p.x;
      A.fis.y[k] = p.y;
      A.fis.g[k] = 0;
      A.fis.e[k] = (double)es;
      A.fis.parent[k] = p.id;
      A.fis.seq[k] = p.nsite + s;
    } else {
      atomicOr(A.status, ST_OVERFLOW);
    }
  }
  if (p.nsite + nf > 0xFFFFu) atomicOr(A.status, ST_OVERFLOW);
  p.nsite += nf;
  // nuclide: first k with xi Sigma_t below the running sum of N_k sigma_t,k
  const R xn = Prec<R>::xi(rs.next());
  const R target = xn * c.x.st;
  const int nn = T.mat_n[c.m];
  const R* dens = CEP<R>::dens(T);
  R cum = R(0);
  int pick = -1, last_nz = -1;
  R mt = R(0), last_t = R(0);
  for (int k = 0; k < nn; ++k) {
    R t, fi;
    CEP<R>::micro_tf(T, c.m, k, c.x.gi, c.x.f, &t, &fi);
    const R term = dens[c.m * T.max_nuc + k] * t;
    cum = cum + term;
    if (term > R(0)) {
      last_nz = k;
      last_t = t;
    }
    if (target < cum) {  // the first such k; the later ones do not matter
      pick = k;
      mt = t;
      break;
    }
  }
  if (pick < 0) {
    pick = last_nz;
    mt = last_t;
  }
  // the scattering cross section of the chosen nuclide only
  const R ms = pick >= 0 ? CEP<R>::micro_s(T, c.m, pick, c.x.gi, c.x.f) : R(0);
  const int nuc = T.mat_nuc[c.m * T.max_nuc + (pick < 0 ? 0 : pick)];
  const R xr = Prec<R>::xi(rs.next());
  if (xr * mt < ms) {
    const R xm = Prec<R>::xi(rs.next());
    R mu;
    p.e = elastic<R>(CEP<R>::awr(T)[nuc], p.e, xm, &mu);
    *q_kabs = 0;
    if (p.e < (R)T.e_cut) return FATE_CUTOFF;
    const R xp = Prec<R>::xi(rs.next());
    rotate<R>(mu, xp, &p.u, &p.v, &p.w);
    return FATE_ALIVE;
  }
  *q_kabs = c.nusf > R(0)
                ? quantize((double)(c.nusf / (c.x.st - ce_macro_s<R>(T, c.m, c.x))), T.q_kabs)
                : 0;
  return FATE_ABSORBED;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <class R>
__global__ void k_ce_source(Tables T, uint32_t gen, uint32_t n, double* sx, double* sy,
                            double* se, uint32_t* status) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  if (!sample_source_ce<R>(T, T.geo, T.seed, T.prob, id, gen, &sx[id], &sy[id], &se[id]))
    atomicOr(status, ST_SOURCE);
}

template <class R>
__global__ void k_ce_birth(Tables T, uint32_t gen, uint32_t n, const double* sx, const double* sy,
                           const double* se, Bank out, uint32_t* cnt_live, uint32_t* cnt_col,
                           const uint32_t* prev_status, uint32_t* status) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  const bool skip = (prev_status && *prev_status != 0u) || (*status & ST_SOURCE);
  if (id == 0) {
    cnt_live[0] = skip ? 0u : n;
    cnt_live[1] = 0;
    cnt_col[0] = 0;
    if (skip) atomicOr(status, ST_SKIPPED);
  }
  if (skip || id >= n) return;
  PartCE<R> p;
  p.x = sx[id];
  p.y = sy[id];
  p.e = (R)se[id];
  Stream rs(T.seed, TAG_TRANSPORT, id, gen, T.prob, 0);
  const R xm = Prec<R>::xi(rs.next());
  const R xp = Prec<R>::xi(rs.next());
  p.w = R(2) * xm - R(1);
  const R s2 = R(1) - p.w * p.w;
  const R sq = CEP<R>::sqrt(s2 > R(0) ? s2 : R(0));
  R cs, sn;
  CEP<R>::cossin_2pi(xp, &cs, &sn);
  p.u = sq * cs;
  p.v = sq * sn;
  locate(T.geo, p.x, p.y, &p.i, &p.j, &p.r);
  p.nsite = 0;
  p.ctr = rs.draw;
  p.id = id;
  p.nseg = 0;
  p.t = 0.0;
  store_ce<R>(out, id, p);
}

// TL: the block's flux tally is staged in LDS (16 B per bin, dynamic LDS at
// T.lds_tally_off; no time grid) and each nonzero bin is added to the
// block's stripe of device memory once, instead of one returning device
// atomic per flight on the few hot bins of a small problem.
template <class R, bool REC, bool TL>
__global__ void __launch_bounds__(1024) k_ce_advance(Tables T, uint32_t gen, uint32_t flights,
                                                     Bank in, const uint32_t* __restrict__ n_in_p,
                                                     Bank live, uint32_t* n_live, Bank col,
                                                     uint32_t* n_col, Accum A, Records Rc,
                                                     uint32_t* clr_live, uint32_t* clr_col) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *clr_live = 0;
    *clr_col = 0;
  }
  const uint32_t n_in = *n_in_p;
  if (TL) {
    if (blockIdx.x * blockDim.x >= n_in) return;  // the whole block
    lds_tally_clear(T);
  }
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  int ev = EV_NONE;
  uint32_t c_seg = 0, c_cross = 0, c_refl = 0;
  unsigned long long tl_lo = 0, tl_hi = 0;
  PartCE<R> p;
  CEXS<R> X{};
  if (k < n_in) {
    p = load_ce<R>(in, k);
    Stream rs(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    CECache<R> cache;
    ce_cache_clear(cache);
    for (uint32_t f = 0; f < flights; ++f) {
      if ((int64_t)p.nseg >= T.max_events) {
        ev = EV_KILL;
        break;
      }
      bool refl = false;
      uint64_t q = 0;
      ev = segment_ce<R, REC, false, TL>(T, T.geo, p, rs, A, Rc, &refl, &q, cache);
      tl_lo += q & 0xFFFFFFFFull;
      tl_hi += q >> 32;
      p.nseg += 1;
      c_seg += 1;
      c_cross += (ev == EV_CROSS || ev == EV_LEAK) ? 1u : 0u;
      c_refl += refl ? 1u : 0u;
      if (ev != EV_CROSS) break;
    }
    p.ctr = rs.draw;
    if (ev == EV_KILL) die_ce<R, REC>(p, FATE_KILLED, A, Rc, T);
    if (ev == EV_LEAK) die_ce<R, REC>(p, FATE_LEAKED, A, Rc, T);
    if (ev == EV_CENSUS) die_ce<R, REC>(p, FATE_CENSUS, A, Rc, T);
    // the collision point's lookup (a hit in the cache) goes with the particle
    if (ev == EV_COLLIDE) {
      const Geo& L = T.geo;
      X = ce_macro_cached<R>(T, L.mats[L.pin_map[p.j * L.nx + p.i] * L.mr1 + p.r], p.e, cache);
    }
  }
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  uint32_t pl, pc;
  block_append2(ev == EV_CROSS, ev == EV_COLLIDE, n_live, n_col, lds, &pl, &pc);
  if (ev == EV_CROSS) store_ce<R>(live, pl, p);
  if (ev == EV_COLLIDE) {
    store_ce<R>(col, pc, p);
    col.xgi[pc] = X.gi;
    static_cast<R*>(col.xf)[pc] = X.f;
    static_cast<R*>(col.xst)[pc] = X.st;
    static_cast<R*>(col.xsf)[pc] = X.sf;
  }
  wave_count(A.cnt + CNT_SEG * STRIPES, c_seg);
  wave_count(A.cnt + CNT_CROSS * STRIPES, c_cross);
  wave_count(A.cnt + CNT_REFL * STRIPES, c_refl);
  wave_flag(A.cnt + CNT_LEAK * STRIPES, ev == EV_LEAK);
  wave_flag(A.cnt + CNT_KILLED * STRIPES, ev == EV_KILL);
  wave_flag(A.cnt + CNT_CENSUS * STRIPES, ev == EV_CENSUS);
  wave_flag(A.cnt + CNT_ADV_ITEMS * STRIPES, k < n_in);
  wave_count(A.cnt + CNT_ADV_SEGS * STRIPES, c_seg);
  wave_acc_halves(A.k + K_TL * STRIPES * 2, tl_lo, tl_hi);
  if (TL) lds_tally_flush(T, A);
}

template <class R, bool REC>
__global__ void __launch_bounds__(1024) k_ce_collide(Tables T, uint32_t gen, Bank in,
                                                     const uint32_t* __restrict__ n_in_p,
                                                     Bank live, uint32_t* n_live, Accum A,
                                                     Records Rc) {
  const uint32_t n_in = *n_in_p;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = k < n_in;
  const double k_used = *A.k_used;
  PartCE<R> p;
  ColCE<R> c;
  uint32_t nf = 0;
  uint64_t q_kcol = 0;
  LockStream rs(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
  if (valid) {
    p = load_ce<R>(in, k);
    // both Philox blocks of the collision's first draws, evaluated by every
    // lane at once
    rs = LockStream(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    rs.top_up();
    rs.fill_next();
    c = col_ce_stored<R>(T, T.geo, p, in, k);
    const double kc = (double)(c.nusf / c.x.st);
    q_kcol = quantize(kc, T.q_kcol);
    if (REC) {
      Rc.n_col[p.id] += 1;
      Rc.kcol_sum[p.id] += kc;
    }
    nf = fission_count_ce<R>(T, c, rs, k_used);
  }
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  const uint32_t slot = block_reserve(nf, A.n_fis, lds);
  int fate = FATE_ALIVE;
  uint64_t q_kabs = 0;
  if (valid) {
    fate = collide_rest_ce<R>(T, p, rs, c, nf, slot, A, &q_kabs);
    p.ctr = rs.draw;
    if (fate != FATE_ALIVE) die_ce<R, REC>(p, fate, A, Rc, T);
  }
  const bool alive = valid && fate == FATE_ALIVE;
  const uint32_t pl = block_reserve(alive ? 1u : 0u, n_live, lds);
  if (alive) store_ce<R>(live, pl, p);
  wave_flag(A.cnt + CNT_COL * STRIPES, valid);
  wave_flag(A.cnt + CNT_COL_ITEMS * STRIPES, valid);
  wave_flag(A.cnt + CNT_SCAT * STRIPES, valid && fate != FATE_ABSORBED);
  wave_flag(A.cnt + CNT_ABS * STRIPES, valid && fate == FATE_ABSORBED);
  wave_flag(A.cnt + CNT_CUTOFF * STRIPES, valid && fate == FATE_CUTOFF);
  wave_count(A.cnt + CNT_SITES * STRIPES, nf);
  wave_acc(A.k + K_COL * STRIPES * 2, q_kcol);
  wave_acc(A.k + K_ABS * STRIPES * 2, q_kabs);
}

template <class R, bool REC, bool TL>
__global__ void __launch_bounds__(256) k_ce_tail(Tables T, uint32_t gen, Bank in,
                                                 const uint32_t* __restrict__ n_in_p, Accum A,
                                                 Records Rc) {
  const uint32_t n_in = *n_in_p;
  if (TL) lds_tally_clear(T);
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long c_seg = 0, c_col = 0, c_cross = 0, c_refl = 0, c_leak = 0, c_abs = 0,
                     c_kill = 0, c_sites = 0, c_scat = 0, c_cut = 0, c_cen = 0;
  unsigned long long kcol[2] = {0, 0}, kabs[2] = {0, 0}, ktl[2] = {0, 0};
  // one pass of the loop is one flight of every live lane of the wave; the
  // fission sites of a pass are reserved with one atomic per wave
  const double k_used = *A.k_used;
  bool live = k < n_in;
  PartCE<R> p;
  Stream rs(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
  CECache<R> cache;
  ce_cache_clear(cache);
  int64_t nseg = 0;
  if (live) {
    p = load_ce<R>(in, k);
    rs = Stream(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    nseg = p.nseg;
  }
  while (__ballot(live) != 0ull) {
    bool col = false;
    ColCE<R> c{};
    uint32_t nf = 0;
    if (live) {
      if (nseg >= T.max_events) {
        p.ctr = rs.draw;
        die_ce<R, REC>(p, FATE_KILLED, A, Rc, T);
        ++c_kill;
        live = false;
      } else {
        bool refl = false;
        uint64_t q = 0;
        const int ev = segment_ce<R, REC, true, TL>(T, T.geo, p, rs, A, Rc, &refl, &q, cache);
        ktl[0] += q & 0xFFFFFFFFull;
        ktl[1] += q >> 32;
        ++nseg;
        ++c_seg;
        if (ev == EV_LEAK) {
          ++c_cross;
          ++c_leak;
          p.ctr = rs.draw;
          die_ce<R, REC>(p, FATE_LEAKED, A, Rc, T);
          live = false;
        } else if (ev == EV_CENSUS) {
          ++c_cen;
          p.ctr = rs.draw;
          die_ce<R, REC>(p, FATE_CENSUS, A, Rc, T);
          live = false;
        } else if (ev == EV_CROSS) {
          ++c_cross;
          c_refl += refl ? 1 : 0;
        } else {
          ++c_col;
          c = col_ce<R>(T, T.geo, p, cache);
          const double kc = (double)(c.nusf / c.x.st);
          const uint64_t qk = quantize(kc, T.q_kcol);
          kcol[0] += qk & 0xFFFFFFFFull;
          kcol[1] += qk >> 32;
          if (REC) {
            Rc.n_col[p.id] += 1;
            Rc.kcol_sum[p.id] += kc;
          }
          nf = fission_count_ce<R>(T, c, rs, k_used);
          col = true;
        }
      }
    }
    const uint32_t slot = __ballot(nf != 0) ? wave_reserve(nf, A.n_fis) : 0u;
    if (col) {
      c_sites += nf;
      uint64_t qa = 0;
      const int fate = collide_rest_ce<R>(T, p, rs, c, nf, slot, A, &qa);
      if (fate == FATE_ALIVE) {
        ++c_scat;
      } else {
        p.ctr = rs.draw;
        if (fate == FATE_CUTOFF) {
          ++c_scat;
          ++c_cut;
        } else {
          kabs[0] += qa & 0xFFFFFFFFull;
          kabs[1] += qa >> 32;
          ++c_abs;
        }
        die_ce<R, REC>(p, fate, A, Rc, T);
        live = false;
      }
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
  wave_count(A.cnt + CNT_CUTOFF * STRIPES, c_cut);
  wave_count(A.cnt + CNT_CENSUS * STRIPES, c_cen);
  wave_acc_halves(A.k + K_COL * STRIPES * 2, kcol[0], kcol[1]);
  wave_acc_halves(A.k + K_ABS * STRIPES * 2, kabs[0], kabs[1]);
  wave_acc_halves(A.k + K_TL * STRIPES * 2, ktl[0], ktl[1]);
  if (TL) lds_tally_flush(T, A);
}

// Monolithic event of the continuous-energy path (see k_mono): one segment
// of every particle per launch, the collision or the crossing in the same
// kernel, survivors to the processed bank.
template <class R, bool REC, bool TL>
__global__ void __launch_bounds__(1024) k_ce_mono(Tables T, uint32_t gen, Bank in,
                                                  const uint32_t* __restrict__ n_in_p, Bank out,
                                                  uint32_t* n_out, Accum A, Records Rc,
                                                  uint32_t* clr_out) {
  if (TL) lds_tally_clear(T);
  if (blockIdx.x == 0 && threadIdx.x == 0) *clr_out = 0;
  const uint32_t n_in = *n_in_p;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = k < n_in;
  const double k_used = *A.k_used;
  int ev = EV_NONE;
  bool refl = false;
  PartCE<R> p;
  ColCE<R> c{};
  uint32_t nf = 0;
  uint64_t q_kcol = 0, q_tl = 0;
  Stream rs(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
  if (valid) {
    p = load_ce<R>(in, k);
    rs = Stream(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    if ((int64_t)p.nseg >= T.max_events) {
      ev = EV_KILL;
    } else {
      CECache<R> cache;
      ce_cache_clear(cache);
      ev = segment_ce<R, REC, false, TL>(T, T.geo, p, rs, A, Rc, &refl, &q_tl, cache);
      p.nseg += 1;
      if (ev == EV_COLLIDE) {
        c = col_ce<R>(T, T.geo, p, cache);
        const double kc = (double)(c.nusf / c.x.st);
        q_kcol = quantize(kc, T.q_kcol);
        if (REC) {
          Rc.n_col[p.id] += 1;
          Rc.kcol_sum[p.id] += kc;
        }
        nf = fission_count_ce<R>(T, c, rs, k_used);
      }
    }
  }
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  const uint32_t slot = block_reserve(nf, A.n_fis, lds);
  int fate = ev == EV_CROSS ? FATE_ALIVE : FATE_KILLED;
  uint64_t q_kabs = 0;
  if (ev == EV_COLLIDE) fate = collide_rest_ce<R>(T, p, rs, c, nf, slot, A, &q_kabs);
  if (ev == EV_LEAK) fate = FATE_LEAKED;
  if (ev == EV_CENSUS) fate = FATE_CENSUS;
  const bool alive = valid && fate == FATE_ALIVE;
  if (valid) {
    p.ctr = rs.draw;
    if (!alive) die_ce<R, REC>(p, fate, A, Rc, T);
  }
  const uint32_t po = block_reserve(alive ? 1u : 0u, n_out, lds);
  if (alive) store_ce<R>(out, po, p);
  const bool seg = valid && ev != EV_KILL;
  const bool col = ev == EV_COLLIDE;
  wave_flag(A.cnt + CNT_SEG * STRIPES, seg);
  wave_flag(A.cnt + CNT_CROSS * STRIPES, ev == EV_CROSS || ev == EV_LEAK);
  wave_flag(A.cnt + CNT_REFL * STRIPES, refl);
  wave_flag(A.cnt + CNT_LEAK * STRIPES, ev == EV_LEAK);
  wave_flag(A.cnt + CNT_KILLED * STRIPES, ev == EV_KILL);
  wave_flag(A.cnt + CNT_CENSUS * STRIPES, ev == EV_CENSUS);
  wave_flag(A.cnt + CNT_COL * STRIPES, col);
  wave_flag(A.cnt + CNT_SCAT * STRIPES, col && fate != FATE_ABSORBED);
  wave_flag(A.cnt + CNT_ABS * STRIPES, col && fate == FATE_ABSORBED);
  wave_flag(A.cnt + CNT_CUTOFF * STRIPES, col && fate == FATE_CUTOFF);
  wave_count(A.cnt + CNT_SITES * STRIPES, nf);
  wave_flag(A.cnt + CNT_ADV_ITEMS * STRIPES, valid);
  wave_flag(A.cnt + CNT_ADV_SEGS * STRIPES, seg);
  wave_flag(A.cnt + CNT_COL_ITEMS * STRIPES, col);
  wave_acc(A.k + K_COL * STRIPES * 2, q_kcol);
  wave_acc(A.k + K_ABS * STRIPES * 2, q_kabs);
  wave_acc(A.k + K_TL * STRIPES * 2, q_tl);
  if (TL) lds_tally_flush(T, A);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static unsigned nblk_ce(uint32_t n, int b) { return (unsigned)((n + (uint32_t)b - 1) / (uint32_t)b); }

hipError_t launch_ce_source(int prec, const Tables& T, uint32_t gen, uint32_t n, double* sx,
                            double* sy, double* se, uint32_t* status, hipStream_t s) {
  const dim3 g(std::max(1u, nblk_ce(n, 256))), b(256);
  if (prec == 0)
    hipLaunchKernelGGL(k_ce_source<double>, g, b, 0, s, T, gen, n, sx, sy, se, status);
  else
    hipLaunchKernelGGL(k_ce_source<float>, g, b, 0, s, T, gen, n, sx, sy, se, status);
  return hipGetLastError();
}

hipError_t launch_ce_birth(int prec, const Tables& T, uint32_t gen, uint32_t n, const double* sx,
                           const double* sy, const double* se, const Bank& out,
                           uint32_t* cnt_live, uint32_t* cnt_col, const uint32_t* prev_status,
                           uint32_t* status, hipStream_t s) {
  const dim3 g(std::max(1u, nblk_ce(n, 256))), b(256);
  if (prec == 0)
    hipLaunchKernelGGL(k_ce_birth<double>, g, b, 0, s, T, gen, n, sx, sy, se, out, cnt_live,
                       cnt_col, prev_status, status);
  else
    hipLaunchKernelGGL(k_ce_birth<float>, g, b, 0, s, T, gen, n, sx, sy, se, out, cnt_live,
                       cnt_col, prev_status, status);
  return hipGetLastError();
}

// the LDS-staged flux words of the flight, tail and monolithic kernels:
// small tallies, no time grid
constexpr size_t CE_LDS_TALLY_MAX = 32768;

// Dynamic LDS of the staged flux words for these tables, or 0 when they are
// not staged.
static size_t ce_lt_bytes(const Tables& T) {
  const size_t lb = 16 * (size_t)T.n_bins;
  return (!T.time && !T.probs && lb <= CE_LDS_TALLY_MAX) ? lb : 0;
}

template <class R, bool REC>
static void ce_advance_k(dim3 g, dim3 b, hipStream_t s, const Tables& T0, uint32_t gen,
                         uint32_t flights, const Bank& in, const uint32_t* n_in, const Bank& live,
                         uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                         const Records& Rc, uint32_t* clr_live, uint32_t* clr_col) {
  const size_t lb = ce_lt_bytes(T0);
  if (lb) {
    Tables T = T0;
    T.lds_tally_off = 0;
    T.lds_bin_lo = 0;
    T.lds_bin_n = (uint32_t)T.n_bins;
    hipLaunchKernelGGL((k_ce_advance<R, REC, true>), g, b, lb, s, T, gen, flights, in, n_in, live,
                       n_live, col, n_col, A, Rc, clr_live, clr_col);
  } else {
    hipLaunchKernelGGL((k_ce_advance<R, REC, false>), g, b, 0, s, T0, gen, flights, in, n_in,
                       live, n_live, col, n_col, A, Rc, clr_live, clr_col);
  }
}

hipError_t launch_ce_advance(int prec, bool rec, const Tables& T, uint32_t gen, uint32_t flights,
                             const Bank& in, const uint32_t* n_in, const Bank& live,
                             uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                             const Records& Rc, uint32_t* clr_live, uint32_t* clr_col,
                             uint32_t bound, int block, hipStream_t s) {
  const dim3 g(std::max(1u, nblk_ce(bound, block))), b(block);
  if (prec == 0) {
    if (rec)
      ce_advance_k<double, true>(g, b, s, T, gen, flights, in, n_in, live, n_live, col, n_col, A,
                                 Rc, clr_live, clr_col);
    else
      ce_advance_k<double, false>(g, b, s, T, gen, flights, in, n_in, live, n_live, col, n_col,
                                  A, Rc, clr_live, clr_col);
  } else {
    if (rec)
      ce_advance_k<float, true>(g, b, s, T, gen, flights, in, n_in, live, n_live, col, n_col, A,
                                Rc, clr_live, clr_col);
    else
      ce_advance_k<float, false>(g, b, s, T, gen, flights, in, n_in, live, n_live, col, n_col, A,
                                 Rc, clr_live, clr_col);
  }
  return hipGetLastError();
}

hipError_t launch_ce_collide(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                             const uint32_t* n_in, const Bank& live, uint32_t* n_live,
                             const Accum& A, const Records& Rc, uint32_t bound, int block,
                             hipStream_t s) {
  const dim3 g(std::max(1u, nblk_ce(bound, block))), b(block);
  if (prec == 0) {
    if (rec)
      hipLaunchKernelGGL((k_ce_collide<double, true>), g, b, 0, s, T, gen, in, n_in, live,
                         n_live, A, Rc);
    else
      hipLaunchKernelGGL((k_ce_collide<double, false>), g, b, 0, s, T, gen, in, n_in, live,
                         n_live, A, Rc);
  } else {
    if (rec)
      hipLaunchKernelGGL((k_ce_collide<float, true>), g, b, 0, s, T, gen, in, n_in, live, n_live,
                         A, Rc);
    else
      hipLaunchKernelGGL((k_ce_collide<float, false>), g, b, 0, s, T, gen, in, n_in, live,
                         n_live, A, Rc);
  }
  return hipGetLastError();
}

hipError_t launch_ce_mono(int prec, bool rec, const Tables& T0, uint32_t gen, const Bank& in,
                          const uint32_t* n_in, const Bank& out, uint32_t* n_out, const Accum& A,
                          const Records& Rc, uint32_t* clr_out, uint32_t bound, int block,
                          hipStream_t s) {
  const dim3 g(std::max(1u, nblk_ce(bound, block))), b(block);
  const size_t lb = ce_lt_bytes(T0);
  Tables T = T0;
  T.lds_tally_off = 0;
  T.lds_bin_lo = 0;
  T.lds_bin_n = (uint32_t)T.n_bins;
#define MCX_CE_MONO(R_, REC_)                                                                   \
  if (lb)                                                                                     \
    hipLaunchKernelGGL((k_ce_mono<R_, REC_, true>), g, b, lb, s, T, gen, in, n_in, out, n_out, A, \
                       Rc, clr_out);                                                          \
  else                                                                                        \
    hipLaunchKernelGGL((k_ce_mono<R_, REC_, false>), g, b, 0, s, T, gen, in, n_in, out, n_out, A, \
                       Rc, clr_out);
  if (prec == 0) {
    if (rec) {
      MCX_CE_MONO(double, true)
    } else {
      MCX_CE_MONO(double, false)
    }
  } else {
    if (rec) {
      MCX_CE_MONO(float, true)
    } else {
      MCX_CE_MONO(float, false)
    }
  }
#undef MCX_CE_MONO
  return hipGetLastError();
}

hipError_t launch_ce_tail(int prec, bool rec, const Tables& T0, uint32_t gen, const Bank& in,
                          const uint32_t* n_in, const Accum& A, const Records& Rc, uint32_t bound,
                          hipStream_t s) {
  const dim3 g(std::max(1u, nblk_ce(bound, 64))), b(64);
  const size_t lb = ce_lt_bytes(T0);
  Tables T = T0;
  T.lds_tally_off = 0;
  T.lds_bin_lo = 0;
  T.lds_bin_n = (uint32_t)T.n_bins;
#define MCX_CE_TAIL(R_, REC_)                                                               \
  if (lb)                                                                                 \
    hipLaunchKernelGGL((k_ce_tail<R_, REC_, true>), g, b, lb, s, T, gen, in, n_in, A, Rc);  \
  else                                                                                    \
    hipLaunchKernelGGL((k_ce_tail<R_, REC_, false>), g, b, 0, s, T, gen, in, n_in, A, Rc);
  if (prec == 0) {
    if (rec) {
      MCX_CE_TAIL(double, true)
    } else {
      MCX_CE_TAIL(double, false)
    }
  } else {
    if (rec) {
      MCX_CE_TAIL(float, true)
    } else {
      MCX_CE_TAIL(float, false)
    }
  }
#undef MCX_CE_TAIL
  return hipGetLastError();
}

}  // namespace mcx
