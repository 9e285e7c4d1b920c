// mcx_device.hpp - particle state, problem tables and the per-particle
// transport operations shared by the event kernels and the tail kernel.
//
// Geometry (paper Sec. 1: constructive solid geometry with surface
// tracking): a rectangular lattice (nx x ny, square pitch, per-side vacuum or
// reflective boundary) of pin universes made of concentric z-cylinders.  A
// particle carries its lattice cell (i, j) and ring region r; positions are
// only located once, at birth, and every later move is a logical transition
// across the surface that bounds the flight.
//
// Physics (Sec. 1: multigroup energy; Sec. 2: collision and fission-bank
// events): analog capture / isotropic scatter with a scattering-matrix group
// transfer, and expected-value fission banking floor(nu_sig_f / (sig_t k) + xi)
// at every collision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcx_math.hpp"

namespace mcx {

enum : int { BC_VACUUM = 0, BC_REFLECT = 1 };
enum : int { FATE_ALIVE = 0, FATE_ABSORBED = 1, FATE_LEAKED = 2, FATE_KILLED = 3 };
enum : int {
  CNT_SEG = 0,
  CNT_COL = 1,
  CNT_CROSS = 2,
  CNT_REFL = 3,
  CNT_LEAK = 4,
  CNT_ABS = 5,
  CNT_KILLED = 6,
  CNT_SITES = 7,
  CNT_SCAT = 8,
  N_CNT = 9,
  CNT_ADV_ITEMS = 9,   // lanes processed by advance kernels
  CNT_COL_ITEMS = 10,  // lanes processed by collide kernels
  N_CNT_ALL = 11
};
enum : int { K_COL = 0, K_TL = 1, K_ABS = 2 };
constexpr int STRIPES = 64;  // copies of each global accumulator (atomic contention)

// cell word: j (12 bits) | i (12 bits) | ring region (8 bits)
MCX_HD uint32_t pack_cell(int i, int j, int r) {
  return ((uint32_t)j << 20) | ((uint32_t)i << 8) | (uint32_t)r;
}
MCX_HD int cell_i(uint32_t c) { return (int)((c >> 8) & 0xFFFu); }
MCX_HD int cell_j(uint32_t c) { return (int)(c >> 20); }
MCX_HD int cell_r(uint32_t c) { return (int)(c & 0xFFu); }

// Read-only problem description (device pointers into the workspace).
struct Tables {
  int nx, ny, n_univ, max_rings, mr1;
  double pitch, x0, y0, width, height;
  int bc[4];  // xmin, xmax, ymin, ymax
  const int* pin_map;
  const int* n_rings;
  const double* radii;
  const int* mats;
  int n_mat, G;
  const double* sig_t;    // [m][g]
  const double* nusf;     // [m][g]
  const double* sst;      // [m][g] total scatter, summed in group order
  const double* cum_s;    // [m][g][g'] running sums of the scatter row
  const int* last_s;      // [m][g] last nonzero out-group
  const double* cum_chi;  // [m][g]
  const int* last_chi;    // [m]
  const int* fissile;     // [m]
  uint64_t seed, prob;
  int fixed_source;
  int ent_nx, ent_ny;
  int n_bins;          // bins per tally: nx * ny * mr1 * G
  int tally_stripes;   // copies of the tally accumulators
  double q_flux, q_prod, q_kcol, q_kabs;  // fixed-point scales 2^s
  int64_t max_events;
};

// Particle bank in structure-of-arrays form.
struct Bank {
  double* x;
  double* y;
  double* u;
  double* v;
  uint32_t* cell;
  uint32_t* gs;   // group (16 bits) | sites banked so far (16 bits)
  uint32_t* ctr;  // transport-stream draws consumed
  uint32_t* id;   // source index of the history
};

// Fission sites as banked (unordered) and in canonical (parent, seq) order.
struct Sites {
  double* x;
  double* y;
  int32_t* g;
  uint32_t* parent;
  uint32_t* seq;
};

// Per-history debug records, indexed by history id.
struct Records {
  int32_t* n_seg;
  int32_t* n_col;
  int32_t* n_cross;
  int32_t* n_refl;
  int32_t* fate;
  int32_t* g_final;
  uint32_t* ctr_final;
  double* tl_sum;
  double* kcol_sum;
  double* x_final;
  double* y_final;
};

// Per-generation accumulators (zeroed at the start of every generation).
struct Accum {
  unsigned long long* tally;  // [stripe][2 tallies][bin][2 halves]
  unsigned long long* k;      // [3][STRIPES][2 halves]
  unsigned long long* cnt;    // [N_CNT_ALL][STRIPES]
  uint32_t* n_fis;            // fission sites appended
  uint32_t* nsite_id;         // [N] sites banked per history
  uint32_t* status;           // error bits
  const double* k_used;       // previous generation's collision estimate
  Sites fis;
  uint32_t fis_cap;
};

enum : uint32_t { ST_OVERFLOW = 1u, ST_SITE_SEQ = 2u, ST_SCAN = 4u, ST_SOURCE = 8u };

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------

// Distance to the plane ahead in the slab lo <= x <= hi; infinity when the
// flight is parallel to it; a negative value (rounding past the plane) is 0.
MCX_HD double dist_plane(double x, double lo, double hi, double u) {
  double t;
  if (u > 0.0) {
    t = (hi - x) / u;
  } else if (u < 0.0) {
    t = (lo - x) / u;
  } else {
    return __builtin_inf();
  }
  return t < 0.0 ? 0.0 : t;
}

// Distance to the z-cylinder of radius R about the cell centre; the side of
// the particle is known logically and clamps the sign of c = |d|^2 - R^2.
MCX_HD double dist_cylinder(double dx, double dy, double u, double v, double R, bool inside) {
  const double a = u * u + v * v;
  if (a == 0.0) return __builtin_inf();
  const double k = dx * u + dy * v;
  double c = dx * dx + dy * dy - R * R;
  if (inside) {
    if (c > 0.0) c = 0.0;
  } else {
    if (c < 0.0) c = 0.0;
  }
  const double disc = k * k - a * c;
  if (inside) {
    if (k >= 0.0) {
      const double q = -(k + sqrt(disc));
      return q == 0.0 ? 0.0 : c / q;
    }
    return (-k + sqrt(disc)) / a;
  }
  if (k >= 0.0 || disc < 0.0) return __builtin_inf();
  return c / (-k + sqrt(disc));
}

MCX_HD void locate(const Tables& T, double x, double y, int* pi, int* pj, int* pr) {
  int i = (int)floor((x - T.x0) / T.pitch);
  int j = (int)floor((y - T.y0) / T.pitch);
  i = i < 0 ? 0 : (i > T.nx - 1 ? T.nx - 1 : i);
  j = j < 0 ? 0 : (j > T.ny - 1 ? T.ny - 1 : j);
  const int un = T.pin_map[j * T.nx + i];
  const double dx = x - (T.x0 + ((double)i + 0.5) * T.pitch);
  const double dy = y - (T.y0 + ((double)j + 0.5) * T.pitch);
  const double rr = dx * dx + dy * dy;
  const int nr = T.n_rings[un];
  int r = nr;
  for (int k = 0; k < nr; ++k) {
    const double rad = T.radii[un * T.max_rings + k];
    if (rr < rad * rad) {
      r = k;
      break;
    }
  }
  *pi = i;
  *pj = j;
  *pr = r;
}

// ---------------------------------------------------------------------------
// sampling
// ---------------------------------------------------------------------------

// First index j with xi * total < cum[j] (cum = running sums in index order,
// total = cum[n-1]); if rounding leaves none, the last nonzero entry.
MCX_HD int sample_cum(double xi, const double* cum, int n, int last_nz) {
  const double target = xi * cum[n - 1];
  for (int j = 0; j < n; ++j)
    if (target < cum[j]) return j;
  return last_nz;
}

// Isotropic direction from two draws; only (u, v) matter in z-invariant
// geometry (w = 2 xi_mu - 1 sets the in-plane speed sqrt(1 - w^2)).
MCX_HD void isotropic_uv(double xi_mu, double xi_phi, double* u, double* v) {
  const double w = 2.0 * xi_mu - 1.0;
  const double s2 = 1.0 - w * w;
  const double s = sqrt(s2 > 0.0 ? s2 : 0.0);
  double c, sn;
  cr_cossin_2pi(xi_phi, sc_tab(), &c, &sn);
  *u = s * c;
  *v = s * sn;
}

// ---------------------------------------------------------------------------
// exact fixed-point accumulation: a nonnegative term t becomes the integer
// q = round(t * 2^s) < 2^62, added as two 32-bit halves into 64-bit counters,
// so that sums are exact and independent of the order of the atomics.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t quantize(double t, double scale) {
  return (uint64_t)__double2ull_rn(t * scale);
}

__device__ __forceinline__ void acc_add(unsigned long long* pair, uint64_t q) {
  if (q == 0) return;
  atomicAdd(pair + 0, (unsigned long long)(q & 0xFFFFFFFFull));
  const uint64_t hi = q >> 32;
  if (hi) atomicAdd(pair + 1, (unsigned long long)hi);
}

// ---------------------------------------------------------------------------
// wavefront helpers (every lane of the wave must call them)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Reserve one slot per lane with pred set: one atomic per wave.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* counter) {
  const unsigned long long mask = __ballot(pred);
  const uint32_t lane = lane_id();
  const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
  const uint32_t total = (uint32_t)__popcll(mask);
  uint32_t base = 0;
  if (total) {
    const int leader = __ffsll((long long)mask) - 1;
    if ((int)lane == leader) base = atomicAdd(counter, total);
    base = __shfl(base, leader);
  }
  return base + rank;
}

// Reserve n slots per lane (exclusive wave prefix sum): one atomic per wave.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t n, uint32_t* counter) {
  const uint32_t lane = lane_id();
  uint32_t incl = n;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off);
    if ((int)lane >= off) incl += t;
  }
  const uint32_t total = __shfl(incl, 63);
  uint32_t base = 0;
  if (total) {
    if (lane == 0) base = atomicAdd(counter, total);
    base = __shfl(base, 0);
  }
  return base + incl - n;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Wave-reduced add of a 64-bit count into one of STRIPES copies.
__device__ __forceinline__ void wave_count(unsigned long long* base, unsigned long long v) {
  v = wave_sum(v);
  if (lane_id() == 0 && v) atomicAdd(base + (blockIdx.x % STRIPES), v);
}

// Wave-reduced add of fixed-point terms (q < 2^62 per lane) into a striped
// (lo, hi) accumulator pair.
__device__ __forceinline__ void wave_acc(unsigned long long* k_base, uint64_t q) {
  const unsigned long long lo = wave_sum((unsigned long long)(q & 0xFFFFFFFFull));
  const unsigned long long hi = wave_sum((unsigned long long)(q >> 32));
  if (lane_id() == 0) {
    unsigned long long* p = k_base + 2 * (blockIdx.x % STRIPES);
    if (lo) atomicAdd(p + 0, lo);
    if (hi) atomicAdd(p + 1, hi);
  }
}

}  // namespace mcx
