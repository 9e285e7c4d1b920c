/*
 * oracle.c - plain FP64 history-based Monte Carlo k-eigenvalue transport.
 *
 * TEST INFRASTRUCTURE: the reference the HIP event-based path is checked
 * against.  Loaded only by the tests, the smoke check and the benchmark's
 * CPU-baseline leg.  Nothing here is shared with the HIP path.
 *
 * The paper (Sec. 1) names the capabilities: multigroup energy physics,
 * constructive solid geometry with surface tracking, k-eigenvalue power
 * iteration and replicable random numbers; Sec. 2 describes the
 * to-be-processed / processed particle banks and the fission bank; Sec. 5
 * fixes FP64 arithmetic.  It gives no transport equations, so each history
 * here is textbook analog Monte Carlo, one particle at a time, in the order:
 *
 *   birth -> { cross-section lookup, distance to collision, distance to
 *   boundary, move + track-length tally, collide | cross } until death
 *
 * and each generation ends with a canonical fission bank, the k estimators,
 * the Shannon entropy of the bank and systematic combing back to N sites.
 *
 * Build: gcc -O2 -std=gnu11 -ffp-contract=off -fno-fast-math (no FMA
 * contraction; every product and sum is rounded on its own), -lquadmath.
 *
 * The two transcendental functions of the path, ln(xi) for the flight
 * distance and cos/sin(2 pi xi) for the azimuth, are taken correctly rounded
 * (the binary64 value nearest the exact result), so that the result of every
 * operation of a history has a single definition independent of any libm.
 *
 * Parity unpinned: the k estimates and tallies of the heterogeneous problems
 * (the pin cell, the 17x17 lattice, the continuous-energy pin cell) have no
 * closed form; they are pinned only through the closed-form limits the tests
 * reduce them to (infinite media, one-material cells, slabs, symmetric
 * lattices), through invariants, and through agreement with the GPU path.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <quadmath.h>
#include <stdatomic.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  Round: multiply words 0 and 2 by the two     */
/* round multipliers, swap and xor the high halves with the other words    */
/* and the key; the key is bumped by the two Weyl constants between rounds. */
/* ------------------------------------------------------------------------ */

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* 64-bit word -> uniform in the open interval (0, 1): the top 52 bits plus
   one half, times 2^-52.  Every value is exact in binary64 and lies in
   [2^-53, 1 - 2^-53]. */
double orc_uniform(uint64_t word) { return ((double)(word >> 12) + 0.5) * 0x1p-52; }

/* A stream is keyed by (seed, tag) and counts draws; draw d reads word d % 4
   of the block at counter (d / 4, particle id, generation, problem). */
typedef struct {
  uint64_t key[2];
  uint64_t id, gen, prob;
  uint32_t draw;
  int64_t blk_idx;
  uint64_t blk[4];
} stream_t;

static void stream_init(stream_t* s, uint64_t seed, uint64_t tag, uint64_t id, uint64_t gen,
                        uint64_t prob) {
  s->key[0] = seed;
  s->key[1] = tag;
  s->id = id;
  s->gen = gen;
  s->prob = prob;
  s->draw = 0;
  s->blk_idx = -1;
}

static double next_uniform(stream_t* s) {
  int64_t b = (int64_t)(s->draw >> 2);
  if (b != s->blk_idx) {
    uint64_t ctr[4] = {(uint64_t)b, s->id, s->gen, s->prob};
    orc_philox4x64_10(ctr, s->key, s->blk);
    s->blk_idx = b;
  }
  uint64_t w = s->blk[s->draw & 3u];
  s->draw += 1u;
  return orc_uniform(w);
}

double orc_stream_uniform(uint64_t seed, uint64_t tag, uint64_t id, uint64_t gen,
                          uint64_t prob, uint32_t draw) {
  stream_t s;
  stream_init(&s, seed, tag, id, gen, prob);
  s.draw = draw;
  return next_uniform(&s);
}

/* ------------------------------------------------------------------------ */
/* geometry                                                                 */
/* ------------------------------------------------------------------------ */

/* Distance along the flight direction to the plane ahead of a particle in
   the slab lo <= x <= hi: the upper plane when moving up, the lower when
   moving down, infinity for a direction parallel to both; a negative
   distance (position a rounding error past the plane) counts as zero. */
double orc_dist_plane(double x, double lo, double hi, double u) {
  double t;
  if (u > 0.0) {
    t = (hi - x) / u;
  } else if (u < 0.0) {
    t = (lo - x) / u;
  } else {
    return INFINITY;
  }
  return t < 0.0 ? 0.0 : t;
}

/* Distance to a z-aligned cylinder of radius R centred at the local origin,
   for a particle at (dx, dy) with direction (u, v, w): the smallest positive
   root of a t^2 + 2 k t + c = 0, a = u^2 + v^2, k = dx u + dy v,
   c = dx^2 + dy^2 - R^2.  The side the particle is on is known logically
   (surface tracking), so c is clamped to that side, and each root is taken
   in the cancellation-free form. */
double orc_dist_cylinder(double dx, double dy, double u, double v, double radius, int inside) {
  double a = u * u + v * v;
  if (a == 0.0) return INFINITY;
  double k = dx * u + dy * v;
  double c = dx * dx + dy * dy - radius * radius;
  if (inside) {
    if (c > 0.0) c = 0.0;
  } else {
    if (c < 0.0) c = 0.0;
  }
  double disc = k * k - a * c;
  if (inside) {
    if (k >= 0.0) {
      double q = -(k + sqrt(disc));
      return q == 0.0 ? 0.0 : c / q;
    }
    return (-k + sqrt(disc)) / a;
  }
  if (k >= 0.0 || disc < 0.0) return INFINITY;
  return c / (-k + sqrt(disc));
}

/* ------------------------------------------------------------------------ */
/* correctly rounded transcendental functions                               */
/* ------------------------------------------------------------------------ */

/* ln(x), correctly rounded.  The 64-bit-significand (x87 extended) logarithm
   is accurate to about 2^-63 relative, so rounding it to binary64 gives the
   nearest double unless it falls within 2^-8 of a binary64 ulp of a rounding
   boundary; there the 113-bit quad-precision logarithm decides. */
double orc_cr_log(double x) {
  long double yl = logl((long double)x);
  double y = (double)yl;
  double nb = (long double)y < yl ? nextafter(y, INFINITY) : nextafter(y, -INFINITY);
  long double mid = ((long double)y + (long double)nb) * 0.5L;
  long double ulp = fabsl((long double)nb - (long double)y);
  if (fabsl(yl - mid) < ulp * 0x1p-8L) return (double)logq((__float128)x);
  return y;
}

/* cos(2 pi t) and sin(2 pi t) for the exact real 2 pi t, 0 <= t < 1,
   correctly rounded.  The angle pi x, x = 2t, is folded exactly (every
   subtraction below is exact by Sterbenz's lemma) into pi y with
   0 <= y <= 1/4, where the quad-precision sine and cosine have a relative
   error near 2^-112, and the result is rounded once to binary64. */
void orc_cr_cossin_2pi(double t, double* c, double* s) {
  double x = 2.0 * t;
  int neg_s = 0, neg_c = 0, swap = 0;
  if (x >= 1.0) { /* sin(pi (x + 1)) = -sin(pi x), cos likewise */
    x = x - 1.0;
    neg_s = !neg_s;
    neg_c = !neg_c;
  }
  if (x > 0.5) { /* sin(pi (1 - x)) = sin(pi x), cos(pi (1 - x)) = -cos(pi x) */
    x = 1.0 - x;
    neg_c = !neg_c;
  }
  if (x > 0.25) { /* sin(pi x) = cos(pi (1/2 - x)) and the reverse */
    x = 0.5 - x;
    swap = 1;
  }
  __float128 a = M_PIq * (__float128)x;
  double sv = (double)sinq(a);
  double cv = (double)cosq(a);
  if (swap) {
    double tmp = sv;
    sv = cv;
    cv = tmp;
  }
  *s = neg_s ? -sv : sv;
  *c = neg_c ? -cv : cv;
}

/* Isotropic direction: polar cosine w = 2 xi_mu - 1 about z, azimuth
   2 pi xi_phi. */
void orc_isotropic(double xi_mu, double xi_phi, double out[3]) {
  double w = 2.0 * xi_mu - 1.0;
  double s2 = 1.0 - w * w;
  double s = sqrt(s2 > 0.0 ? s2 : 0.0);
  double c, sn;
  orc_cr_cossin_2pi(xi_phi, &c, &sn);
  out[0] = s * c;
  out[1] = s * sn;
  out[2] = w;
}

/* Discrete sampling: cumulate the weights in index order; the sample is the
   first index j with xi * total < cum_j; if rounding leaves none, the last
   index with a nonzero weight. */
int orc_sample_cdf(double xi, const double* weights, int n) {
  double total = 0.0;
  for (int j = 0; j < n; ++j) total += weights[j];
  double target = xi * total;
  double cum = 0.0;
  for (int j = 0; j < n; ++j) {
    cum += weights[j];
    if (target < cum) return j;
  }
  for (int j = n - 1; j >= 0; --j)
    if (weights[j] > 0.0) return j;
  return n - 1;
}

/* Systematic combing of M banked sites down (or up) to N: site i of the new
   source is bank entry floor((i + xi0) M / N), capped at M - 1. */
void orc_comb(int64_t n, int64_t m, double xi0, int64_t* idx) {
  for (int64_t i = 0; i < n; ++i) {
    double t = ((double)i + xi0) * (double)m / (double)n;
    int64_t k = (int64_t)floor(t);
    if (k > m - 1) k = m - 1;
    idx[i] = k;
  }
}

/* Shannon entropy (base 2) of the bank over the mesh bins. */
double orc_entropy(const int64_t* counts, int64_t n_bins, int64_t m) {
  double h = 0.0;
  if (m <= 0) return 0.0;
  for (int64_t b = 0; b < n_bins; ++b) {
    if (counts[b] > 0) {
      double p = (double)counts[b] / (double)m;
      h -= p * log2(p);
    }
  }
  return h;
}

/* Neumaier's compensated summation. */
typedef struct {
  double s, c;
} nsum_t;

static void nadd(nsum_t* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static double nval(const nsum_t* a) { return a->s + a->c; }

double orc_neumaier(const double* v, int64_t n) {
  nsum_t a = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) nadd(&a, v[i]);
  return nval(&a);
}

/* ------------------------------------------------------------------------ */
/* continuous energy (Sec. 1 capability; Sec. 4 continuous-energy pin cell)   */
/* ------------------------------------------------------------------------ */

/* The interval of an increasing grid that holds e: the largest i with
   grid[i] <= e, limited to [0, n - 2], so energies beyond either end use the
   end intervals.  Found by bisection; the index is unique, so any search
   that returns it is equivalent. */
int orc_ce_interval(const double* grid, int n, double e) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = lo + (hi - lo) / 2;
    if (grid[mid] <= e)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

/* Linear interpolation in energy within interval i: the fraction
   (e - E_i) / (E_{i+1} - E_i) clipped to [0, 1], then v_i + f (v_{i+1} - v_i). */
static double ce_frac(const double* grid, int i, double e) {
  double f = (e - grid[i]) / (grid[i + 1] - grid[i]);
  if (f < 0.0) f = 0.0;
  if (f > 1.0) f = 1.0;
  return f;
}

static double ce_lerp(const double* row, int i, double f) { return row[i] + f * (row[i + 1] - row[i]); }

/* Macroscopic total, scattering and fission cross sections of material m at
   energy e: sums of density times interpolated microscopic values, taken in
   the material's nuclide order. */
void orc_ce_macro(const orc_ce* ce, int m, double e, double out[3]) {
  int i = orc_ce_interval(ce->e_grid, ce->n_pts, e);
  double f = ce_frac(ce->e_grid, i, e);
  double st = 0.0, ss = 0.0, sf = 0.0;
  for (int k = 0; k < ce->mat_n[m]; ++k) {
    int n = ce->mat_nuc[m * ce->max_nuc + k];
    double dens = ce->mat_dens[m * ce->max_nuc + k];
    int64_t row = (int64_t)n * ce->n_pts;
    st = st + dens * ce_lerp(ce->sig_t + row, i, f);
    ss = ss + dens * ce_lerp(ce->sig_s + row, i, f);
    sf = sf + dens * ce_lerp(ce->sig_f + row, i, f);
  }
  out[0] = st;
  out[1] = ss;
  out[2] = sf;
}

/* One attempt of the Watt spectrum sampler: a Maxwellian variate of
   temperature a by the three-uniform rule W = -a (ln x1 + ln x2 cos^2(pi x3 / 2)),
   then E = W + a^2 b / 4 + (2 x4 - 1) sqrt(a^2 b W).  cos(pi x3 / 2) is
   cos(2 pi (x3 / 4)), with x3 / 4 exact. */
double orc_watt_attempt(double a, double b, double xi1, double xi2, double xi3, double xi4) {
  double c, s;
  orc_cr_cossin_2pi(0.25 * xi3, &c, &s);
  double w = -a * (orc_cr_log(xi1) + orc_cr_log(xi2) * (c * c));
  double q = a * a * b;
  return (w + 0.25 * q) + (2.0 * xi4 - 1.0) * sqrt(q * w);
}

/* Elastic scattering off a target of mass ratio A at rest, isotropic in the
   centre-of-mass frame: mu_cm = 2 xi - 1, outgoing energy
   E (A^2 + 2 A mu_cm + 1) / (A + 1)^2, lab cosine
   (1 + A mu_cm) / sqrt(A^2 + 2 A mu_cm + 1). */
double orc_elastic(double awr, double e, double xi_mu, double* mu_lab) {
  double mu = 2.0 * xi_mu - 1.0;
  double num = (awr * awr + 2.0 * awr * mu) + 1.0;
  double ap1 = awr + 1.0;
  *mu_lab = (1.0 + awr * mu) / sqrt(num);
  return e * num / (ap1 * ap1);
}

/* Turn the unit direction dir by the polar cosine mu about itself, azimuth
   2 pi xi_phi (the textbook rotation; when the direction lies within 1e-10
   of the z axis, the same formula with x taking z's role). */
void orc_rotate(double mu, double xi_phi, double dir[3]) {
  double c, s;
  orc_cr_cossin_2pi(xi_phi, &c, &s);
  double u = dir[0], v = dir[1], w = dir[2];
  double sm = 1.0 - mu * mu;
  sm = sm > 0.0 ? sqrt(sm) : 0.0;
  double a = 1.0 - w * w;
  if (a > 1e-10) {
    double t = sqrt(a);
    dir[0] = mu * u + sm * (u * w * c - v * s) / t;
    dir[1] = mu * v + sm * (v * w * c + u * s) / t;
    dir[2] = mu * w - sm * t * c;
  } else {
    double t = sqrt(1.0 - u * u);
    dir[1] = mu * v + sm * (v * u * c - w * s) / t;
    dir[2] = mu * w + sm * (w * u * c + v * s) / t;
    dir[0] = mu * u - sm * t * c;
  }
}

/* ------------------------------------------------------------------------ */
/* the run                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  double* x;
  double* y;
  int32_t* g;
  double* e;
  int64_t n, cap;
} sites_t;

static int sites_push(sites_t* s, double x, double y, int32_t g, double e) {
  if (s->n == s->cap) {
    int64_t nc = s->cap ? 2 * s->cap : 1024;
    double* nx = realloc(s->x, (size_t)nc * sizeof(double));
    if (!nx) return -1;
    s->x = nx;
    double* ny = realloc(s->y, (size_t)nc * sizeof(double));
    if (!ny) return -1;
    s->y = ny;
    int32_t* ng = realloc(s->g, (size_t)nc * sizeof(int32_t));
    if (!ng) return -1;
    s->g = ng;
    double* ne = realloc(s->e, (size_t)nc * sizeof(double));
    if (!ne) return -1;
    s->e = ne;
    s->cap = nc;
  }
  s->x[s->n] = x;
  s->y[s->n] = y;
  s->g[s->n] = g;
  s->e[s->n] = e;
  s->n += 1;
  return 0;
}

static void sites_free(sites_t* s) {
  free(s->x);
  free(s->y);
  free(s->g);
  free(s->e);
  memset(s, 0, sizeof(*s));
}

/* Accumulators of one fixed chunk of histories.  Chunks are summed in chunk
   order, so results do not depend on the number of threads. */
typedef struct {
  nsum_t k[3];
  nsum_t* flux;
  nsum_t* prod;
  int64_t counts[ORC_NCOUNT];
  sites_t sites;
  int err;
} chunk_t;

typedef struct {
  const orc_problem* p;
  int64_t n_bins;
  int32_t mr1;                 /* max_rings + 1 */
  int32_t* fissile;            /* [n_mat] */
  double* sig_s_tot;           /* [n_mat][n_grp], summed in index order */
  /* current generation */
  int gen;
  double k_used;
  const double* src_x;
  const double* src_y;
  const int32_t* src_g;
  const double* src_e;         /* continuous energy: source energies */
  const double* src_dir;       /* [N][3] or NULL */
  chunk_t* chunks;
  int64_t n_chunks, chunk_size;
  atomic_long next_chunk;
  orc_record* records;         /* this generation's records or NULL */
  orc_event* events;           /* this generation's event log or NULL */
  int32_t event_cap;
} ctx_t;

static void log_flight(const ctx_t* C, int64_t id, int32_t k, double x, double y, double d,
                       double e, int cell, int region, int group, int type) {
  if (!C->events || k >= C->event_cap) return;
  orc_event* ev = &C->events[id * C->event_cap + k];
  ev->x = x;
  ev->y = y;
  ev->d = d;
  ev->e = e;
  ev->cell = cell;
  ev->region = region;
  ev->group = group;
  ev->type = type;
}

static void locate(const orc_problem* p, double x, double y, int* ci, int* cj, int* cr) {
  int i = (int)floor((x - p->x0) / p->pitch);
  int j = (int)floor((y - p->y0) / p->pitch);
  if (i < 0) i = 0;
  if (i > p->nx - 1) i = p->nx - 1;
  if (j < 0) j = 0;
  if (j > p->ny - 1) j = p->ny - 1;
  int un = p->pin_map[j * p->nx + i];
  double dx = x - (p->x0 + ((double)i + 0.5) * p->pitch);
  double dy = y - (p->y0 + ((double)j + 0.5) * p->pitch);
  double rr = dx * dx + dy * dy;
  int nr = p->n_rings[un];
  int r = nr;
  for (int k = 0; k < nr; ++k) {
    double rad = p->radii[un * p->max_rings + k];
    if (rr < rad * rad) {
      r = k;
      break;
    }
  }
  *ci = i;
  *cj = j;
  *cr = r;
}

static int material_at(const ctx_t* C, int i, int j, int r) {
  const orc_problem* p = C->p;
  int un = p->pin_map[j * p->nx + i];
  return p->mats[un * C->mr1 + r];
}

/* Source site of particle id in batch gen: rejection in the lattice's
   bounding box until the point lies in a fissile material, then a group
   from that material's fission spectrum. */
/* A Watt-spectrum energy: attempts of four draws each until one lies in
   (0, e_max]. */
static double watt_sample(const orc_ce* ce, stream_t* s) {
  for (int t = 0; t < 10000; ++t) {
    double x1 = next_uniform(s);
    double x2 = next_uniform(s);
    double x3 = next_uniform(s);
    double x4 = next_uniform(s);
    double e = orc_watt_attempt(ce->watt_a, ce->watt_b, x1, x2, x3, x4);
    if (e > 0.0 && e <= ce->e_max) return e;
  }
  return ce->e_max;
}

double orc_speed(double e) { return 2.99792458e10 * sqrt(2.0 * e / 939.56542052e6); }

static int sample_source(const ctx_t* C, int64_t id, int gen, double* sx, double* sy,
                         int32_t* sg, double* se) {
  const orc_problem* p = C->p;
  stream_t s;
  stream_init(&s, p->seed, ORC_TAG_SRC, (uint64_t)id, (uint64_t)gen, p->problem_id);
  double width = (double)p->nx * p->pitch;
  double height = (double)p->ny * p->pitch;
  for (int t = 0; t < 10000; ++t) {
    double xa = next_uniform(&s);
    double ya = next_uniform(&s);
    double x = p->x0 + xa * width;
    double y = p->y0 + ya * height;
    int i, j, r;
    locate(p, x, y, &i, &j, &r);
    int m = material_at(C, i, j, r);
    if (C->fissile[m]) {
      *sx = x;
      *sy = y;
      if (p->ce) {
        *sg = 0;
        *se = p->ce->src_energy > 0.0 ? p->ce->src_energy : watt_sample(p->ce, &s);
      } else {
        double xi = next_uniform(&s);
        *sg = orc_sample_cdf(xi, p->chi + (int64_t)m * p->n_grp, p->n_grp);
        *se = 0.0;
      }
      return 0;
    }
  }
  return -1;
}

static void run_history(ctx_t* C, int64_t id, int64_t slot, chunk_t* ch) {
  const orc_problem* p = C->p;
  const int G = p->n_grp;
  stream_t rs;
  stream_init(&rs, p->seed, ORC_TAG_TRANSPORT, (uint64_t)id, (uint64_t)C->gen, p->problem_id);

  double x = C->src_x[slot], y = C->src_y[slot];
  int g = C->src_g[slot];
  int i, j, r;
  locate(p, x, y, &i, &j, &r);
  double dir[3];
  if (C->src_dir) {
    dir[0] = C->src_dir[3 * slot + 0];
    dir[1] = C->src_dir[3 * slot + 1];
    dir[2] = C->src_dir[3 * slot + 2];
  } else {
    double xm = next_uniform(&rs);
    double xp = next_uniform(&rs);
    orc_isotropic(xm, xp, dir);
  }
  double u = dir[0], v = dir[1], w = dir[2];
  (void)w; /* z-invariant geometry: w only fixes the in-plane speed sqrt(1-w^2) */
  const orc_time* tm = p->time;
  const int NT = tm ? tm->n_tbins : 1;
  const double t_max = tm ? tm->t_edges[NT] : 0.0;
  double t = 0.0;  /* time since the source pulse */

  int32_t n_seg = 0, n_col = 0, n_cross = 0, n_refl = 0, n_sites = 0;
  int fate = ORC_ALIVE;
  double tl_sum = 0.0, kcol_sum = 0.0;

  for (;;) {
    if (n_seg >= p->max_events) {
      fate = ORC_KILLED;
      break;
    }
    int c = j * p->nx + i;
    int un = p->pin_map[c];
    int nr = p->n_rings[un];
    int m = p->mats[un * C->mr1 + r];
    double st = p->sig_t[m * G + g];
    double nusf = p->nu_sig_f[m * G + g];

    /* distance to collision: exponential with mean 1 / sig_t */
    double xi = next_uniform(&rs);
    double d_col = -orc_cr_log(xi) / st;

    /* distance to boundary: the lattice cell's planes ahead and the rings
       bounding the current region */
    double xlo = p->x0 + (double)i * p->pitch, xhi = p->x0 + (double)(i + 1) * p->pitch;
    double ylo = p->y0 + (double)j * p->pitch, yhi = p->y0 + (double)(j + 1) * p->pitch;
    double tx = orc_dist_plane(x, xlo, xhi, u);
    double ty = orc_dist_plane(y, ylo, yhi, v);
    double cx = p->x0 + ((double)i + 0.5) * p->pitch;
    double cy = p->y0 + ((double)j + 0.5) * p->pitch;
    double dx = x - cx, dy = y - cy;
    double t_out = INFINITY, t_in = INFINITY;
    if (r < nr) t_out = orc_dist_cylinder(dx, dy, u, v, p->radii[un * p->max_rings + r], 1);
    if (r > 0) t_in = orc_dist_cylinder(dx, dy, u, v, p->radii[un * p->max_rings + r - 1], 0);
    double d_bnd = tx;
    if (ty < d_bnd) d_bnd = ty;
    if (t_out < d_bnd) d_bnd = t_out;
    if (t_in < d_bnd) d_bnd = t_in;

    n_seg += 1;
    int collide = d_col < d_bnd;
    double d = collide ? d_col : d_bnd;
    /* time-dependent: the flight stops at the end of the time grid if that
       comes first (census) */
    int census = 0;
    double vg = 0.0;
    if (tm) {
      vg = tm->speed[g];
      double d_cen = (t_max - t) * vg;
      if (d_cen < d) {
        d = d_cen;
        census = 1;
        collide = 0;
      }
    }
    x = x + d * u;
    y = y + d * v;

    /* track-length tallies: flux and nu-fission production per bin (per
       time bin by the time the flight spends in it) */
    int64_t bin = ((int64_t)c * C->mr1 + r) * G + g;
    if (tm) {
      double t1 = census ? t_max : t + d / vg;
      if (t1 > t_max) t1 = t_max;
      for (int b = orc_ce_interval(tm->t_edges, NT + 1, t); b < NT; ++b) {
        double lo = tm->t_edges[b] > t ? tm->t_edges[b] : t;
        double hi = tm->t_edges[b + 1] < t1 ? tm->t_edges[b + 1] : t1;
        if (hi > lo) {
          double ell = (hi - lo) * vg;
          nadd(&ch->flux[bin * NT + b], ell);
          nadd(&ch->prod[bin * NT + b], ell * nusf);
        }
        if (tm->t_edges[b + 1] >= t1) break;
      }
      t = t1;
    } else {
      nadd(&ch->flux[bin], d);
      nadd(&ch->prod[bin], d * nusf);
    }
    nadd(&ch->k[1], d * nusf);
    tl_sum += d;
    const int r_flight = r;
    if (census) {
      log_flight(C, id, n_seg - 1, x, y, d, 0.0, c, r_flight, g, 4);
      fate = ORC_CENSUS;
      break;
    }

    if (collide) {
      log_flight(C, id, n_seg - 1, x, y, d, 0.0, c, r_flight, g, 1);
      n_col += 1;
      double kc = nusf / st;
      kcol_sum += kc;
      nadd(&ch->k[0], kc);
      /* fission: bank floor(nu_sig_f / (sig_t k) + xi) sites at the
         collision point, each with a group from the fission spectrum */
      if (!p->fixed_source && nusf > 0.0) {
        double xf = next_uniform(&rs);
        int nf = (int)floor(nusf / (st * C->k_used) + xf);
        for (int s = 0; s < nf; ++s) {
          double xs = next_uniform(&rs);
          int gs = orc_sample_cdf(xs, p->chi + (int64_t)m * G, G);
          if (sites_push(&ch->sites, x, y, gs, 0.0)) ch->err = ORC_ENOMEM;
          n_sites += 1;
        }
      }
      /* scatter with probability sig_s / sig_t, else absorption */
      double xr = next_uniform(&rs);
      double sst = C->sig_s_tot[m * G + g];
      if (xr * st < sst) {
        double xg = next_uniform(&rs);
        g = orc_sample_cdf(xg, p->sig_s + ((int64_t)m * G + g) * G, G);
        double xm = next_uniform(&rs);
        double xp = next_uniform(&rs);
        orc_isotropic(xm, xp, dir);
        u = dir[0];
        v = dir[1];
        w = dir[2];
        ch->counts[ORC_C_SCAT] += 1;
      } else {
        nadd(&ch->k[2], nusf > 0.0 ? nusf / (st - sst) : 0.0);
        fate = ORC_ABSORBED;
        break;
      }
    } else {
      n_cross += 1;
      int hit_x = tx == d_bnd;
      int hit_y = ty == d_bnd;
      if (hit_x || hit_y) {
        /* lattice boundary: neighbour cell, or an outer side of the lattice */
        int out_x = hit_x && (u > 0.0 ? i == p->nx - 1 : i == 0);
        int out_y = hit_y && (v > 0.0 ? j == p->ny - 1 : j == 0);
        int side_x = u > 0.0 ? 1 : 0;
        int side_y = v > 0.0 ? 3 : 2;
        if ((out_x && p->bc[side_x] == ORC_VACUUM) || (out_y && p->bc[side_y] == ORC_VACUUM)) {
          log_flight(C, id, n_seg - 1, x, y, d, 0.0, c, r_flight, g, 3);
          fate = ORC_LEAKED;
          break;
        }
        log_flight(C, id, n_seg - 1, x, y, d, 0.0, c, r_flight, g, 2);
        int refl = 0;
        if (hit_x) {
          if (out_x) {
            u = -u;
            refl = 1;
          } else {
            i += u > 0.0 ? 1 : -1;
          }
        }
        if (hit_y) {
          if (out_y) {
            v = -v;
            refl = 1;
          } else {
            j += v > 0.0 ? 1 : -1;
          }
        }
        if (refl) n_refl += 1;
        /* a lattice face lies outside every ring */
        r = p->n_rings[p->pin_map[j * p->nx + i]];
      } else if (t_out == d_bnd) {
        log_flight(C, id, n_seg - 1, x, y, d, 0.0, c, r_flight, g, 2);
        r += 1;
      } else {
        log_flight(C, id, n_seg - 1, x, y, d, 0.0, c, r_flight, g, 2);
        r -= 1;
      }
    }
  }

  ch->counts[ORC_C_SEG] += n_seg;
  ch->counts[ORC_C_COL] += n_col;
  ch->counts[ORC_C_CROSS] += n_cross;
  ch->counts[ORC_C_REFL] += n_refl;
  ch->counts[ORC_C_SITES] += n_sites;
  if (fate == ORC_LEAKED) ch->counts[ORC_C_LEAK] += 1;
  if (fate == ORC_ABSORBED) ch->counts[ORC_C_ABS] += 1;
  if (fate == ORC_KILLED) ch->counts[ORC_C_KILLED] += 1;
  if (fate == ORC_CENSUS) ch->counts[ORC_C_CENSUS] += 1;
  if (C->records) {
    orc_record* rec = &C->records[slot];
    rec->t_final = t;
    rec->n_seg = n_seg;
    rec->n_col = n_col;
    rec->n_cross = n_cross;
    rec->n_refl = n_refl;
    rec->fate = fate;
    rec->n_sites = n_sites;
    rec->g_final = g;
    rec->ctr_final = rs.draw;
    rec->tl_sum = tl_sum;
    rec->kcol_sum = kcol_sum;
    rec->x_final = x;
    rec->y_final = y;
    rec->e_final = 0.0;
  }
}

/* One continuous-energy history.  The flight is the multigroup one with the
   macroscopic cross sections of the current energy; a collision banks
   fission sites with Watt energies, picks the nuclide by its share of the
   total cross section, then scatters elastically off it (target at rest) or
   absorbs.  Draw order per collision: fission (k-eigenvalue, fissile), four
   per Watt attempt per site, nuclide, scatter test, then for a scatter the
   centre-of-mass cosine and, above the cutoff, the azimuth. */
static void run_history_ce(ctx_t* C, int64_t id, int64_t slot, chunk_t* ch) {
  const orc_problem* p = C->p;
  const orc_ce* ce = p->ce;
  const int NB = ce->n_ebins;
  stream_t rs;
  stream_init(&rs, p->seed, ORC_TAG_TRANSPORT, (uint64_t)id, (uint64_t)C->gen, p->problem_id);

  double x = C->src_x[slot], y = C->src_y[slot], e = C->src_e[slot];
  int i, j, r;
  locate(p, x, y, &i, &j, &r);
  double dir[3];
  if (C->src_dir) {
    dir[0] = C->src_dir[3 * slot + 0];
    dir[1] = C->src_dir[3 * slot + 1];
    dir[2] = C->src_dir[3 * slot + 2];
  } else {
    double xm = next_uniform(&rs);
    double xp = next_uniform(&rs);
    orc_isotropic(xm, xp, dir);
  }

  int32_t n_seg = 0, n_col = 0, n_cross = 0, n_refl = 0, n_sites = 0;
  int fate = ORC_ALIVE;
  double tl_sum = 0.0, kcol_sum = 0.0;
  const orc_time* tm = p->time;
  const int NT = tm ? tm->n_tbins : 1;
  const double t_max = tm ? tm->t_edges[NT] : 0.0;
  double t = 0.0; /* time since the source pulse */

  for (;;) {
    if (n_seg >= p->max_events) {
      fate = ORC_KILLED;
      break;
    }
    int c = j * p->nx + i;
    int un = p->pin_map[c];
    int nr = p->n_rings[un];
    int m = p->mats[un * C->mr1 + r];
    double xs[3];
    orc_ce_macro(ce, m, e, xs);
    double st = xs[0];
    double nusf = ce->nu * xs[2];
    double u = dir[0], v = dir[1];

    double xi = next_uniform(&rs);
    double d_col = -orc_cr_log(xi) / st;

    double xlo = p->x0 + (double)i * p->pitch, xhi = p->x0 + (double)(i + 1) * p->pitch;
    double ylo = p->y0 + (double)j * p->pitch, yhi = p->y0 + (double)(j + 1) * p->pitch;
    double tx = orc_dist_plane(x, xlo, xhi, u);
    double ty = orc_dist_plane(y, ylo, yhi, v);
    double cx = p->x0 + ((double)i + 0.5) * p->pitch;
    double cy = p->y0 + ((double)j + 0.5) * p->pitch;
    double dx = x - cx, dy = y - cy;
    double t_out = INFINITY, t_in = INFINITY;
    if (r < nr) t_out = orc_dist_cylinder(dx, dy, u, v, p->radii[un * p->max_rings + r], 1);
    if (r > 0) t_in = orc_dist_cylinder(dx, dy, u, v, p->radii[un * p->max_rings + r - 1], 0);
    double d_bnd = tx;
    if (ty < d_bnd) d_bnd = ty;
    if (t_out < d_bnd) d_bnd = t_out;
    if (t_in < d_bnd) d_bnd = t_in;

    n_seg += 1;
    int collide = d_col < d_bnd;
    double d = collide ? d_col : d_bnd;
    /* time-dependent: the flight stops at the end of the time grid if that
       comes first (census); its speed is the neutron speed at e */
    int census = 0;
    double ve = 0.0;
    if (tm) {
      ve = orc_speed(e);
      double d_cen = (t_max - t) * ve;
      if (d_cen < d) {
        d = d_cen;
        census = 1;
        collide = 0;
      }
    }
    x = x + d * u;
    y = y + d * v;

    /* track-length flux per (cell, region, energy bin[, time bin]); the
       track-length k estimator sums d nu Sigma_f(E); time-dependent: the
       flux of each time bin is the length flown in it and the density the
       time spent in it */
    int b = orc_ce_interval(ce->e_edges, NB + 1, e);
    int64_t bin = ((int64_t)c * C->mr1 + r) * NB + b;
    if (tm) {
      double t1 = census ? t_max : t + d / ve;
      if (t1 > t_max) t1 = t_max;
      for (int q = orc_ce_interval(tm->t_edges, NT + 1, t); q < NT; ++q) {
        double lo = tm->t_edges[q] > t ? tm->t_edges[q] : t;
        double hi = tm->t_edges[q + 1] < t1 ? tm->t_edges[q + 1] : t1;
        if (hi > lo) {
          nadd(&ch->flux[bin * NT + q], (hi - lo) * ve);
          nadd(&ch->prod[bin * NT + q], hi - lo);
        }
        if (tm->t_edges[q + 1] >= t1) break;
      }
      t = t1;
    } else {
      nadd(&ch->flux[bin], d);
    }
    nadd(&ch->k[1], d * nusf);
    tl_sum += d;
    const int r_flight = r;
    if (census) {
      log_flight(C, id, n_seg - 1, x, y, d, e, c, r_flight, b, 4);
      fate = ORC_CENSUS;
      break;
    }

    if (collide) {
      log_flight(C, id, n_seg - 1, x, y, d, e, c, r_flight, b, 1);
      n_col += 1;
      double kc = nusf / st;
      kcol_sum += kc;
      nadd(&ch->k[0], kc);
      if (!p->fixed_source && nusf > 0.0) {
        double xf = next_uniform(&rs);
        int nf = (int)floor(nusf / (st * C->k_used) + xf);
        for (int q = 0; q < nf; ++q) {
          double es = watt_sample(ce, &rs);
          if (sites_push(&ch->sites, x, y, 0, es)) ch->err = ORC_ENOMEM;
          n_sites += 1;
        }
      }
      /* nuclide: first k with xi * Sigma_t below the running sum of
         N_k sigma_t,k (the same sums as the macroscopic total) */
      int gi = orc_ce_interval(ce->e_grid, ce->n_pts, e);
      double f = ce_frac(ce->e_grid, gi, e);
      double xn = next_uniform(&rs);
      double target = xn * st;
      double cum = 0.0;
      int pick = -1, last_nz = -1;
      for (int k = 0; k < ce->mat_n[m]; ++k) {
        int n = ce->mat_nuc[m * ce->max_nuc + k];
        double term = ce->mat_dens[m * ce->max_nuc + k] *
                      ce_lerp(ce->sig_t + (int64_t)n * ce->n_pts, gi, f);
        cum = cum + term;
        if (term > 0.0) last_nz = k;
        if (pick < 0 && target < cum) pick = k;
      }
      if (pick < 0) pick = last_nz;
      int nuc = ce->mat_nuc[m * ce->max_nuc + pick];
      double mt = ce_lerp(ce->sig_t + (int64_t)nuc * ce->n_pts, gi, f);
      double ms = ce_lerp(ce->sig_s + (int64_t)nuc * ce->n_pts, gi, f);
      double xr = next_uniform(&rs);
      if (xr * mt < ms) {
        ch->counts[ORC_C_SCAT] += 1;
        double xm = next_uniform(&rs);
        double mu;
        double e_out = orc_elastic(ce->awr[nuc], e, xm, &mu);
        e = e_out;
        if (e < ce->e_cut) {
          fate = ORC_CUTOFF;
          break;
        }
        double xp = next_uniform(&rs);
        orc_rotate(mu, xp, dir);
      } else {
        nadd(&ch->k[2], nusf > 0.0 ? nusf / (st - xs[1]) : 0.0);
        fate = ORC_ABSORBED;
        break;
      }
    } else {
      n_cross += 1;
      int hit_x = tx == d_bnd;
      int hit_y = ty == d_bnd;
      if (hit_x || hit_y) {
        int out_x = hit_x && (u > 0.0 ? i == p->nx - 1 : i == 0);
        int out_y = hit_y && (v > 0.0 ? j == p->ny - 1 : j == 0);
        int side_x = u > 0.0 ? 1 : 0;
        int side_y = v > 0.0 ? 3 : 2;
        if ((out_x && p->bc[side_x] == ORC_VACUUM) || (out_y && p->bc[side_y] == ORC_VACUUM)) {
          log_flight(C, id, n_seg - 1, x, y, d, e, c, r_flight, b, 3);
          fate = ORC_LEAKED;
          break;
        }
        log_flight(C, id, n_seg - 1, x, y, d, e, c, r_flight, b, 2);
        int refl = 0;
        if (hit_x) {
          if (out_x) {
            dir[0] = -u;
            refl = 1;
          } else {
            i += u > 0.0 ? 1 : -1;
          }
        }
        if (hit_y) {
          if (out_y) {
            dir[1] = -v;
            refl = 1;
          } else {
            j += v > 0.0 ? 1 : -1;
          }
        }
        if (refl) n_refl += 1;
        r = p->n_rings[p->pin_map[j * p->nx + i]];
      } else if (t_out == d_bnd) {
        log_flight(C, id, n_seg - 1, x, y, d, e, c, r_flight, b, 2);
        r += 1;
      } else {
        log_flight(C, id, n_seg - 1, x, y, d, e, c, r_flight, b, 2);
        r -= 1;
      }
    }
  }

  ch->counts[ORC_C_SEG] += n_seg;
  ch->counts[ORC_C_COL] += n_col;
  ch->counts[ORC_C_CROSS] += n_cross;
  ch->counts[ORC_C_REFL] += n_refl;
  ch->counts[ORC_C_SITES] += n_sites;
  if (fate == ORC_LEAKED) ch->counts[ORC_C_LEAK] += 1;
  if (fate == ORC_ABSORBED) ch->counts[ORC_C_ABS] += 1;
  if (fate == ORC_KILLED) ch->counts[ORC_C_KILLED] += 1;
  if (fate == ORC_CUTOFF) ch->counts[ORC_C_CUTOFF] += 1;
  if (fate == ORC_CENSUS) ch->counts[ORC_C_CENSUS] += 1;
  if (C->records) {
    orc_record* rec = &C->records[slot];
    rec->n_seg = n_seg;
    rec->n_col = n_col;
    rec->n_cross = n_cross;
    rec->n_refl = n_refl;
    rec->fate = fate;
    rec->n_sites = n_sites;
    rec->g_final = orc_ce_interval(ce->e_edges, NB + 1, e);
    rec->ctr_final = rs.draw;
    rec->tl_sum = tl_sum;
    rec->kcol_sum = kcol_sum;
    rec->x_final = x;
    rec->y_final = y;
    rec->e_final = e;
    rec->t_final = t;
  }
}

static void* worker(void* arg) {
  ctx_t* C = (ctx_t*)arg;
  const int64_t n = C->p->n_per_gen;
  for (;;) {
    int64_t k = atomic_fetch_add(&C->next_chunk, 1);
    if (k >= C->n_chunks) break;
    chunk_t* ch = &C->chunks[k];
    int64_t lo = k * C->chunk_size;
    int64_t hi = lo + C->chunk_size;
    if (hi > n) hi = n;
    if (C->p->ce)
      for (int64_t id = lo; id < hi; ++id) run_history_ce(C, id, id, ch);
    else
      for (int64_t id = lo; id < hi; ++id) run_history(C, id, id, ch);
  }
  return NULL;
}

static void chunk_reset(chunk_t* ch, int64_t n_bins) {
  memset(ch->k, 0, sizeof(ch->k));
  memset(ch->flux, 0, (size_t)n_bins * sizeof(nsum_t));
  memset(ch->prod, 0, (size_t)n_bins * sizeof(nsum_t));
  memset(ch->counts, 0, sizeof(ch->counts));
  ch->sites.n = 0;
  ch->err = 0;
}

int64_t orc_n_bins(const orc_problem* p) {
  return (int64_t)p->nx * p->ny * (p->max_rings + 1) * (p->ce ? p->ce->n_ebins : p->n_grp) *
         (p->time ? p->time->n_tbins : 1);
}

static int fail(orc_output* out, int code, const char* msg) {
  snprintf(out->errmsg, sizeof(out->errmsg), "%s", msg);
  return code;
}

static int validate(const orc_problem* p, orc_output* out) {
  if (p->nx < 1 || p->ny < 1 || !(p->pitch > 0.0)) return fail(out, ORC_EINVAL, "bad lattice");
  if (p->n_univ < 1 || p->max_rings < 1 || p->n_mat < 1 || (!p->ce && p->n_grp < 1))
    return fail(out, ORC_EINVAL, "bad sizes");
  if (p->n_per_gen < 1 || p->n_gen < 1 || p->n_inactive < 0 || p->n_inactive >= p->n_gen)
    return fail(out, ORC_EINVAL, "bad run sizes");
  for (int k = 0; k < p->nx * p->ny; ++k)
    if (p->pin_map[k] < 0 || p->pin_map[k] >= p->n_univ) return fail(out, ORC_EINVAL, "pin map");
  for (int u = 0; u < p->n_univ; ++u) {
    int nr = p->n_rings[u];
    if (nr < 0 || nr > p->max_rings) return fail(out, ORC_EINVAL, "ring count");
    for (int k = 0; k <= nr; ++k) {
      int m = p->mats[u * (p->max_rings + 1) + k];
      if (m < 0 || m >= p->n_mat) return fail(out, ORC_EINVAL, "ring material");
    }
    double prev = 0.0;
    for (int k = 0; k < nr; ++k) {
      double rad = p->radii[u * p->max_rings + k];
      if (!(rad > prev) || !(rad < 0.5 * p->pitch)) return fail(out, ORC_EINVAL, "ring radius");
      prev = rad;
    }
  }
  if (p->time) {
    const orc_time* tm = p->time;
    if (!p->fixed_source || tm->n_tbins < 1 || !(tm->t_edges[0] == 0.0))
      return fail(out, ORC_EINVAL, "time-dependent mode: fixed source, edges from 0");
    for (int k = 0; k < tm->n_tbins; ++k)
      if (!(tm->t_edges[k] < tm->t_edges[k + 1]) || !isfinite(tm->t_edges[k + 1]))
        return fail(out, ORC_EINVAL, "time edges must increase");
    for (int g = 0; g < (p->ce ? 0 : p->n_grp); ++g)
      if (!(tm->speed[g] > 0.0) || !isfinite(tm->speed[g]))
        return fail(out, ORC_EINVAL, "group speeds must be positive");
  }
  if (p->ce) {
    const orc_ce* ce = p->ce;
    if (ce->n_nuc < 1 || ce->n_pts < 2 || ce->max_nuc < 1 || ce->n_ebins < 1 || !(ce->nu >= 0.0) ||
        !(ce->watt_a > 0.0) || !(ce->watt_b >= 0.0) || !(ce->e_max > 0.0) || !(ce->e_cut >= 0.0) ||
        !(ce->src_energy >= 0.0) || !isfinite(ce->src_energy))
      return fail(out, ORC_EINVAL, "continuous-energy sizes");
    for (int k = 0; k + 1 < ce->n_pts; ++k)
      if (!(ce->e_grid[k] < ce->e_grid[k + 1])) return fail(out, ORC_EINVAL, "energy grid order");
    for (int k = 0; k < ce->n_ebins; ++k)
      if (!(ce->e_edges[k] < ce->e_edges[k + 1])) return fail(out, ORC_EINVAL, "tally edges order");
    for (int64_t k = 0; k < (int64_t)ce->n_nuc * ce->n_pts; ++k)
      if (!(ce->sig_s[k] >= 0.0) || !(ce->sig_f[k] >= 0.0) || !(ce->sig_t[k] >= ce->sig_s[k]))
        return fail(out, ORC_EINVAL, "pointwise cross sections");
    for (int n = 0; n < ce->n_nuc; ++n)
      if (!(ce->awr[n] > 0.0)) return fail(out, ORC_EINVAL, "target mass");
    for (int m = 0; m < p->n_mat; ++m) {
      if (ce->mat_n[m] < 1 || ce->mat_n[m] > ce->max_nuc) return fail(out, ORC_EINVAL, "material size");
      for (int k = 0; k < ce->mat_n[m]; ++k) {
        int n = ce->mat_nuc[m * ce->max_nuc + k];
        if (n < 0 || n >= ce->n_nuc || !(ce->mat_dens[m * ce->max_nuc + k] >= 0.0))
          return fail(out, ORC_EINVAL, "material nuclide");
      }
    }
    return ORC_OK;
  }
  for (int64_t k = 0; k < (int64_t)p->n_mat * p->n_grp; ++k) {
    if (!(p->sig_t[k] > 0.0) || !(p->nu_sig_f[k] >= 0.0) || !(p->chi[k] >= 0.0))
      return fail(out, ORC_EINVAL, "cross section sign");
  }
  for (int64_t k = 0; k < (int64_t)p->n_mat * p->n_grp * p->n_grp; ++k)
    if (!(p->sig_s[k] >= 0.0)) return fail(out, ORC_EINVAL, "scatter sign");
  return ORC_OK;
}

/* The run context of problem p: the fissile flag of each material and, for
   multigroup data, each group's total scattering cross section (at most
   sigma_t). */
static int ctx_begin(ctx_t* C, const orc_problem* p, orc_output* out) {
  const int G = p->n_grp;
  memset(C, 0, sizeof(*C));
  C->p = p;
  C->n_bins = orc_n_bins(p);
  C->mr1 = p->max_rings + 1;
  C->fissile = calloc((size_t)p->n_mat, sizeof(int32_t));
  C->sig_s_tot = calloc((size_t)p->n_mat * (p->ce ? 1 : G), sizeof(double));
  if (p->ce) {
    /* fissile: a nuclide with a nonzero density and some fission cross section */
    const orc_ce* ce = p->ce;
    for (int m = 0; m < p->n_mat; ++m)
      for (int k = 0; k < ce->mat_n[m]; ++k) {
        int n = ce->mat_nuc[m * ce->max_nuc + k];
        if (!(ce->mat_dens[m * ce->max_nuc + k] > 0.0) || !(ce->nu > 0.0)) continue;
        for (int q = 0; q < ce->n_pts; ++q)
          if (ce->sig_f[(int64_t)n * ce->n_pts + q] > 0.0) {
            C->fissile[m] = 1;
            break;
          }
      }
  }
  for (int m = 0; m < (p->ce ? 0 : p->n_mat); ++m) {
    for (int g = 0; g < G; ++g) {
      if (p->nu_sig_f[m * G + g] > 0.0) C->fissile[m] = 1;
      double s = 0.0;
      for (int h = 0; h < G; ++h) s += p->sig_s[((int64_t)m * G + g) * G + h];
      C->sig_s_tot[m * G + g] = s;
      if (s > p->sig_t[m * G + g]) {
        free(C->fissile);
        free(C->sig_s_tot);
        return fail(out, ORC_EINVAL, "sig_s exceeds sig_t");
      }
    }
  }
  return ORC_OK;
}

int orc_run(const orc_problem* p, orc_output* out) {
  out->errmsg[0] = 0;
  int rc = validate(p, out);
  if (rc) return rc;
  const int64_t N = p->n_per_gen;

  ctx_t C;
  rc = ctx_begin(&C, p, out);
  if (rc) return rc;
  /* fixed chunking: at most 256 chunks of at least 512 histories */
  C.chunk_size = 512;
  if ((N + C.chunk_size - 1) / C.chunk_size > 256) C.chunk_size = (N + 255) / 256;
  C.n_chunks = (N + C.chunk_size - 1) / C.chunk_size;
  C.chunks = calloc((size_t)C.n_chunks, sizeof(chunk_t));
  for (int64_t k = 0; k < C.n_chunks; ++k) {
    C.chunks[k].flux = calloc((size_t)C.n_bins, sizeof(nsum_t));
    C.chunks[k].prod = calloc((size_t)C.n_bins, sizeof(nsum_t));
  }

  double* src_x = malloc((size_t)N * sizeof(double));
  double* src_y = malloc((size_t)N * sizeof(double));
  int32_t* src_g = malloc((size_t)N * sizeof(int32_t));
  double* src_e = malloc((size_t)N * sizeof(double));
  double* src_dir = NULL;
  double* gflux = malloc((size_t)p->n_gen * C.n_bins * sizeof(double));
  double* gprod = malloc((size_t)p->n_gen * C.n_bins * sizeof(double));
  sites_t bank = {0};
  int64_t* ent_counts = calloc((size_t)p->ent_nx * p->ent_ny, sizeof(int64_t));
  int64_t* comb_idx = malloc((size_t)N * sizeof(int64_t));
  if (!src_x || !src_y || !src_g || !src_e || !gflux || !gprod || !ent_counts || !comb_idx) {
    rc = fail(out, ORC_ENOMEM, "out of host memory");
    goto done;
  }

  double k_used = 1.0;
  int n_threads = p->n_threads > 0 ? p->n_threads : 1;
  for (int gen = 0; gen < p->n_gen; ++gen) {
    /* source of this generation */
    if (gen == 0 || p->fixed_source) {
      free(src_dir);
      src_dir = NULL;
      if (gen == 0 && p->ext_state) {
        src_dir = malloc((size_t)N * 3 * sizeof(double));
        for (int64_t id = 0; id < N; ++id) {
          src_x[id] = p->ext_state[6 * id + 0];
          src_y[id] = p->ext_state[6 * id + 1];
          src_dir[3 * id + 0] = p->ext_state[6 * id + 2];
          src_dir[3 * id + 1] = p->ext_state[6 * id + 3];
          src_dir[3 * id + 2] = p->ext_state[6 * id + 4];
          src_g[id] = p->ce ? 0 : (int32_t)p->ext_state[6 * id + 5];
          src_e[id] = p->ce ? p->ext_state[6 * id + 5] : 0.0;
        }
      } else {
        for (int64_t id = 0; id < N; ++id) {
          if (sample_source(&C, id, gen, &src_x[id], &src_y[id], &src_g[id], &src_e[id])) {
            rc = fail(out, ORC_EINVAL, "source rejection sampling found no fissile point");
            goto done;
          }
        }
      }
    }

    if (out->source)
      for (int64_t id = 0; id < N; ++id) {
        double* o = out->source + ((int64_t)gen * N + id) * 3;
        o[0] = src_x[id];
        o[1] = src_y[id];
        o[2] = p->ce ? src_e[id] : (double)src_g[id];
      }

    C.gen = gen;
    C.k_used = k_used;
    C.src_x = src_x;
    C.src_y = src_y;
    C.src_g = src_g;
    C.src_e = src_e;
    C.src_dir = src_dir;
    C.records = out->records ? out->records + (int64_t)gen * N : NULL;
    C.events = out->events && out->event_cap > 0 ? out->events + (int64_t)gen * N * out->event_cap
                                                 : NULL;
    C.event_cap = out->event_cap;
    for (int64_t k = 0; k < C.n_chunks; ++k) chunk_reset(&C.chunks[k], C.n_bins);
    atomic_store(&C.next_chunk, 0);
    if (n_threads == 1) {
      worker(&C);
    } else {
      pthread_t th[256];
      int nt = n_threads > 256 ? 256 : n_threads;
      for (int t = 0; t < nt; ++t) pthread_create(&th[t], NULL, worker, &C);
      for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    }

    /* combine chunks in chunk order */
    nsum_t ks[3] = {{0, 0}, {0, 0}, {0, 0}};
    int64_t counts[ORC_NCOUNT] = {0};
    bank.n = 0;
    for (int64_t k = 0; k < C.n_chunks; ++k) {
      chunk_t* ch = &C.chunks[k];
      if (ch->err) {
        rc = fail(out, ch->err, "out of host memory in the fission bank");
        goto done;
      }
      for (int e = 0; e < 3; ++e) {
        nadd(&ks[e], ch->k[e].s);
        nadd(&ks[e], ch->k[e].c);
      }
      for (int e = 0; e < ORC_NCOUNT; ++e) counts[e] += ch->counts[e];
      for (int64_t s = 0; s < ch->sites.n; ++s)
        if (sites_push(&bank, ch->sites.x[s], ch->sites.y[s], ch->sites.g[s], ch->sites.e[s])) {
          rc = fail(out, ORC_ENOMEM, "out of host memory in the bank");
          goto done;
        }
    }
    for (int64_t b = 0; b < C.n_bins; ++b) {
      nsum_t fs = {0, 0}, ps = {0, 0};
      for (int64_t k = 0; k < C.n_chunks; ++k) {
        nadd(&fs, C.chunks[k].flux[b].s);
        nadd(&fs, C.chunks[k].flux[b].c);
        nadd(&ps, C.chunks[k].prod[b].s);
        nadd(&ps, C.chunks[k].prod[b].c);
      }
      gflux[(int64_t)gen * C.n_bins + b] = nval(&fs) / (double)N;
      gprod[(int64_t)gen * C.n_bins + b] = nval(&ps) / (double)N;
    }
    for (int e = 0; e < 3; ++e) out->gen_k[gen * 3 + e] = nval(&ks[e]) / (double)N;
    for (int e = 0; e < ORC_NCOUNT; ++e) out->gen_counts[(int64_t)gen * ORC_NCOUNT + e] = counts[e];

    /* the canonical bank is the chunk concatenation: histories in id order,
       each history's sites in the order they were banked */
    const int64_t M = bank.n;
    const int64_t n_ent = (int64_t)p->ent_nx * p->ent_ny;
    memset(ent_counts, 0, (size_t)n_ent * sizeof(int64_t));
    double width = (double)p->nx * p->pitch;
    double height = (double)p->ny * p->pitch;
    for (int64_t s = 0; s < M; ++s) {
      int bx = (int)floor((bank.x[s] - p->x0) / width * (double)p->ent_nx);
      int by = (int)floor((bank.y[s] - p->y0) / height * (double)p->ent_ny);
      if (bx < 0) bx = 0;
      if (bx > p->ent_nx - 1) bx = p->ent_nx - 1;
      if (by < 0) by = 0;
      if (by > p->ent_ny - 1) by = p->ent_ny - 1;
      ent_counts[(int64_t)by * p->ent_nx + bx] += 1;
    }
    out->gen_entropy[gen] = orc_entropy(ent_counts, n_ent, M);

    if (!p->fixed_source) {
      if (M == 0) {
        rc = fail(out, ORC_EEXTINCT, "fission bank is empty");
        goto done;
      }
      stream_t rs;
      stream_init(&rs, p->seed, ORC_TAG_RESAMPLE, 0, (uint64_t)gen, p->problem_id);
      double xi0 = next_uniform(&rs);
      orc_comb(N, M, xi0, comb_idx);
      for (int64_t id = 0; id < N; ++id) {
        src_x[id] = bank.x[comb_idx[id]];
        src_y[id] = bank.y[comb_idx[id]];
        src_g[id] = bank.g[comb_idx[id]];
        src_e[id] = bank.e[comb_idx[id]];
      }
      free(src_dir);
      src_dir = NULL;
      k_used = out->gen_k[gen * 3 + 0];
    }
  }

  /* active-generation mean and standard deviation of the mean */
  {
    const int A = p->n_gen - p->n_inactive;
    for (int e = 0; e < 3; ++e) {
      double s = 0.0;
      for (int g = p->n_inactive; g < p->n_gen; ++g) s += out->gen_k[g * 3 + e];
      double mean = s / (double)A;
      double v = 0.0;
      for (int g = p->n_inactive; g < p->n_gen; ++g) {
        double d = out->gen_k[g * 3 + e] - mean;
        v += d * d;
      }
      out->k_mean[e] = mean;
      out->k_sigma[e] = A > 1 ? sqrt(v / ((double)A * (double)(A - 1))) : 0.0;
    }
    for (int t = 0; t < 2; ++t) {
      const double* gv = t == 0 ? gflux : gprod;
      double* mo = t == 0 ? out->flux_mean : out->prod_mean;
      double* so = t == 0 ? out->flux_sigma : out->prod_sigma;
      if (!mo) continue;
      for (int64_t b = 0; b < C.n_bins; ++b) {
        double s = 0.0;
        for (int g = p->n_inactive; g < p->n_gen; ++g) s += gv[(int64_t)g * C.n_bins + b];
        double mean = s / (double)A;
        double v = 0.0;
        for (int g = p->n_inactive; g < p->n_gen; ++g) {
          double d = gv[(int64_t)g * C.n_bins + b] - mean;
          v += d * d;
        }
        mo[b] = mean;
        if (so) so[b] = A > 1 ? sqrt(v / ((double)A * (double)(A - 1))) : 0.0;
      }
    }
    if (out->gen_flux) memcpy(out->gen_flux, gflux, (size_t)p->n_gen * C.n_bins * sizeof(double));
    if (out->gen_prod) memcpy(out->gen_prod, gprod, (size_t)p->n_gen * C.n_bins * sizeof(double));
    out->bank_len = bank.n;
    if (out->bank) {
      int64_t nb = bank.n < out->bank_cap ? bank.n : out->bank_cap;
      for (int64_t s = 0; s < nb; ++s) {
        out->bank[3 * s + 0] = bank.x[s];
        out->bank[3 * s + 1] = bank.y[s];
        out->bank[3 * s + 2] = p->ce ? bank.e[s] : (double)bank.g[s];
      }
    }
  }

done:
  for (int64_t k = 0; k < C.n_chunks; ++k) {
    free(C.chunks[k].flux);
    free(C.chunks[k].prod);
    sites_free(&C.chunks[k].sites);
  }
  free(C.chunks);
  free(C.fissile);
  free(C.sig_s_tot);
  free(src_x);
  free(src_y);
  free(src_g);
  free(src_e);
  free(src_dir);
  free(gflux);
  free(gprod);
  free(ent_counts);
  free(comb_idx);
  sites_free(&bank);
  return rc;
}

/* Histories ids[0..n_ids) of the first generation only, each with the
   source sample, transport and record orc_run gives it there (k_used = 1):
   a first-generation history depends on nothing but the problem, the seed
   and its id, so a sample of a run too large to compute whole can be checked
   history by history.  out->records receives one record per listed id, in
   list order; no other output is written. */
int orc_histories(const orc_problem* p, const int64_t* ids, int64_t n_ids, orc_output* out) {
  out->errmsg[0] = 0;
  int rc = validate(p, out);
  if (rc) return rc;
  if (n_ids < 0 || (n_ids > 0 && (!ids || !out->records)))
    return fail(out, ORC_EINVAL, "history list");
  for (int64_t k = 0; k < n_ids; ++k)
    if (ids[k] < 0 || ids[k] >= p->n_per_gen) return fail(out, ORC_EINVAL, "history id");
  ctx_t C;
  rc = ctx_begin(&C, p, out);
  if (rc) return rc;
  chunk_t ch;
  memset(&ch, 0, sizeof(ch));
  ch.flux = calloc((size_t)C.n_bins, sizeof(nsum_t));
  ch.prod = calloc((size_t)C.n_bins, sizeof(nsum_t));
  const size_t n = n_ids > 0 ? (size_t)n_ids : 1;
  double* sx = malloc(n * sizeof(double));
  double* sy = malloc(n * sizeof(double));
  int32_t* sg = malloc(n * sizeof(int32_t));
  double* se = malloc(n * sizeof(double));
  double* sd = p->ext_state ? malloc(n * 3 * sizeof(double)) : NULL;
  if (!ch.flux || !ch.prod || !sx || !sy || !sg || !se || (p->ext_state && !sd)) {
    rc = fail(out, ORC_ENOMEM, "out of host memory");
    goto done;
  }
  for (int64_t k = 0; k < n_ids; ++k) {
    const int64_t id = ids[k];
    if (p->ext_state) {
      sx[k] = p->ext_state[6 * id + 0];
      sy[k] = p->ext_state[6 * id + 1];
      sd[3 * k + 0] = p->ext_state[6 * id + 2];
      sd[3 * k + 1] = p->ext_state[6 * id + 3];
      sd[3 * k + 2] = p->ext_state[6 * id + 4];
      sg[k] = p->ce ? 0 : (int32_t)p->ext_state[6 * id + 5];
      se[k] = p->ce ? p->ext_state[6 * id + 5] : 0.0;
    } else if (sample_source(&C, id, 0, &sx[k], &sy[k], &sg[k], &se[k])) {
      rc = fail(out, ORC_EINVAL, "source rejection sampling found no fissile point");
      goto done;
    }
  }
  C.gen = 0;
  C.k_used = 1.0;
  C.src_x = sx;
  C.src_y = sy;
  C.src_g = sg;
  C.src_e = se;
  C.src_dir = sd;
  C.records = out->records;
  C.events = NULL;
  for (int64_t k = 0; k < n_ids; ++k) {
    if (p->ce)
      run_history_ce(&C, ids[k], k, &ch);
    else
      run_history(&C, ids[k], k, &ch);
    if (ch.err) {
      rc = fail(out, ch.err, "out of host memory in the fission bank");
      goto done;
    }
  }
done:
  free(sx);
  free(sy);
  free(sg);
  free(se);
  free(sd);
  free(ch.flux);
  free(ch.prod);
  sites_free(&ch.sites);
  free(C.fissile);
  free(C.sig_s_tot);
  return rc;
}
