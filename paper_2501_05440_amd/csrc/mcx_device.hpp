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
enum : int {
  FATE_ALIVE = 0,
  FATE_ABSORBED = 1,
  FATE_LEAKED = 2,
  FATE_KILLED = 3,
  FATE_CUTOFF = 4,
  FATE_CENSUS = 5
};
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
  CNT_CUTOFF = 9,      // histories ended below the energy cutoff (continuous energy)
  CNT_CENSUS = 10,     // histories that reached the end of the time grid
  N_CNT = 11,          // counters reported per generation
  CNT_ADV_ITEMS = 11,  // lanes processed by advance kernels
  CNT_COL_ITEMS = 12,  // lanes processed by collide kernels
  CNT_ADV_SEGS = 13,   // flights made inside advance kernels
  N_CNT_ALL = 14
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

// Lattice of one problem: nx x ny cells of pitch `pitch` from (x0, y0),
// per-side boundaries, pin universes (ring counts, radii, ring materials as
// global material indices), and the offset of the problem's tally bins.
struct Geo {
  int nx, ny, max_rings, mr1;
  double pitch, x0, y0, width, height;
  int bc[4];  // xmin, xmax, ymin, ymax
  const int* pin_map;
  const int* n_rings;
  const double* radii;
  const int* mats;
  int bin_base;
};

// One problem of a batch: its lattice, random-number key and counter word,
// and its range of histories in the batch.
struct ProbDesc {
  Geo geo;
  uint64_t seed, prob;
  uint64_t hist_base;
  uint32_t n_hist;
  int n_bins;
};

// Read-only problem description (device pointers into the workspace).
struct Tables {
  Geo geo;  // the lattice of a single-problem run
  int n_univ;
  int n_mat, G;
  const double* sig_t;    // [m][g]
  const double* nusf;     // [m][g]
  const double* sst;      // [m][g] total scatter, summed in group order
  const double* cum_s;    // [m][g][g'] running sums of the scatter row
  const int* last_s;      // [m][g] last nonzero out-group
  const double* cum_chi;  // [m][g]
  const int* last_chi;    // [m]
  const int* fissile;     // [m]
  // binary32 copies for the FP32-mixed mode (running sums summed in binary32)
  const float* sig_t_f;
  const float* nusf_f;
  const float* sst_f;
  const float* cum_s_f;
  const float* cum_chi_f;
  uint64_t seed, prob;
  int fixed_source;
  int ent_nx, ent_ny;
  int n_bins;          // bins per tally (all problems of a batch)
  const ProbDesc* probs;  // batch problems (persistent engine), or null
  int n_probs;
  uint64_t n_hist_total;
  int tally_stripes;   // copies of the tally accumulators
  uint32_t lds_tally_off;  // byte offset of a block's staged flux words in dynamic LDS
  // the staged words hold tally bins [lds_bin_lo, lds_bin_lo + lds_bin_n);
  // other bins go to device memory directly
  uint32_t lds_bin_lo, lds_bin_n;
  double q_flux, q_kcol, q_kabs;  // fixed-point scales 2^s
  int64_t max_events;
  // continuous energy (ce != 0; then G counts the flux tally's energy bins)
  int ce;
  int n_pts, max_nuc, n_ebins;
  const double* e_grid;    // [n_pts] increasing, eV
  const double* ce_tf;     // [n_mat][n_pts][max_nuc][2]: sig_t, sig_f (barns) of the
                           // material's nuclides in material order
  const double* ce_s;      // [n_mat][n_pts][max_nuc]: sig_s
  const double* awr;       // [n_nuc]
  const int* mat_n;        // [n_mat]
  const int* mat_nuc;      // [n_mat][max_nuc]
  const double* mat_dens;  // [n_mat][max_nuc]
  const double* e_edges;   // [n_ebins + 1]
  // binary32 copies for the FP32-mixed mode
  const float* e_grid_f;
  const float* ce_tf_f;    // [n_mat][n_pts][max_nuc][2]
  const float* ce_s_f;     // [n_mat][n_pts][max_nuc]
  const float* awr_f;
  const float* mat_dens_f;
  const float* e_edges_f;
  // interval search start points: bucket b of the bit patterns of E above
  // the first grid point holds the intervals hash[b] .. hash[b + 1]
  const int* e_hash;       // [n_hash + 1]
  const int* e_hash_f;     // [n_hash_f + 1]
  int n_hash, n_hash_f, hash_shift, hash_shift_f;
  uint64_t hash_base;
  uint32_t hash_base_f;
  double nu, watt_a, watt_b, e_max, e_cut;
  double q_ktl;            // fixed-point scale of the track-length k terms
  double q_dens;           // fixed-point scale of the density terms (continuous-energy
                           // time-dependent mode)
  double src_energy;       // > 0: continuous-energy source energy, eV (else Watt)
  // time-dependent fixed source (time != 0): nt time bins per tally bin,
  // group speeds, census at t_max
  int time;
  int nt;
  const double* t_edges;   // [nt + 1]
  const double* speed;     // [G] cm/s
  double t_max;
  // double-double tables of ln and sin/cos(2 pi t), bound on the device at
  // kernel entry (constant memory, or a copy in LDS)
  const double* lt;
  const double* sct;
};

// Particle bank in structure-of-arrays form.
struct Bank {
  double* x;
  double* y;
  void* u;  // direction cosines in the working precision (double or float)
  void* v;
  uint32_t* cell;
  uint32_t* gs;   // group (16 bits) | sites banked so far (16 bits)
  uint32_t* ctr;  // transport-stream draws consumed
  uint32_t* id;   // source index of the history
  uint32_t* nseg; // flights made so far (event guard)
  double* t;      // time-dependent mode: time since the source pulse
  void* w;        // continuous energy: z direction cosine (working precision)
  void* e;        // continuous energy: energy, eV (working precision)
  // continuous energy, collision bank only: the lookup of the collision
  // point made by the flight that ended there (grid interval, fraction,
  // macroscopic total and fission cross sections, working precision)
  int32_t* xgi;
  void* xf;
  void* xst;
  void* xsf;
};

// Fission sites as banked (unordered) and in canonical (parent, seq) order.
struct Sites {
  double* x;
  double* y;
  int32_t* g;
  uint32_t* parent;
  uint32_t* seq;
  double* e;  // continuous energy: site energies
};

// Fission sites filed by bucket of parent histories (generation end), one
// record per site: key = parent within its bucket (low 10 bits) | seq << 10.
struct StSite {
  double x, y;
  uint32_t key;
  int32_t g;
};
struct StSiteCE {
  double x, y, e;
  uint32_t key;
  int32_t pad;
};
struct Staging {
  StSite* mg;
  StSiteCE* ce;  // continuous energy (then mg is null)
};

// One logged flight: position after it, its length and energy, the cell,
// region and group (or energy bin) it flew in, and how it ended
// (1 collision, 2 surface crossing, 3 leak, 4 census).
struct EvEntry {
  double x, y, d, e;
  int cell, region, group, type;
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
  double* e_final;
  double* t_final;
  EvEntry* ev;  // [history][ev_cap] flights, or null
  int ev_cap;
};

// Record flight k of history id (debug event log).
MCX_HD void log_flight(const Records& Rc, uint32_t id, int k, double x, double y, double d,
                       double e, int cell, int region, int group, int type) {
  if (Rc.ev && k < Rc.ev_cap) {
    EvEntry& v = Rc.ev[(size_t)id * (size_t)Rc.ev_cap + (size_t)k];
    v.x = x;
    v.y = y;
    v.d = d;
    v.e = e;
    v.cell = cell;
    v.region = region;
    v.group = group;
    v.type = type;
  }
}

// Per-generation accumulators (zeroed at the start of every generation).
struct Accum {
  unsigned long long* tally;  // flux: [stripe][bin] (lo, hi) 128-bit pairs
  unsigned long long* tally_t;  // flux from the tail kernels: [stripe][bin] (sum of low, high 32-bit halves)
  // continuous-energy time-dependent mode: neutron density (time spent per
  // bin), laid out as tally and tally_t; null otherwise
  unsigned long long* dens;
  unsigned long long* dens_t;
  unsigned long long* k;      // [3][STRIPES][2 halves]
  unsigned long long* cnt;    // [N_CNT_ALL][STRIPES]
  uint32_t* n_fis;            // fission sites appended
  uint32_t* nsite_id;         // [N] sites banked per history
  uint32_t* status;           // error bits of this generation
  const double* k_used;       // previous generation's collision estimate
  Sites fis;
  uint32_t fis_cap;
};

// Per-generation status bits.  A generation that starts after a failed one
// runs empty and is marked ST_SKIPPED.
enum : uint32_t {
  ST_OVERFLOW = 1u,
  ST_SITE_SEQ = 2u,
  ST_SCAN = 4u,
  ST_SOURCE = 8u,
  ST_EXTINCT = 16u,
  ST_SKIPPED = 32u,
  ST_TALLY = 64u,  // 2^32 or more flights: a tail-kernel flux word may have wrapped
  ST_ASYNC = 128u  // the asynchronous engine gave up a wait past its bound
};

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

MCX_HD void locate(const Geo& L, double x, double y, int* pi, int* pj, int* pr) {
  int i = (int)floor((x - L.x0) / L.pitch);
  int j = (int)floor((y - L.y0) / L.pitch);
  i = i < 0 ? 0 : (i > L.nx - 1 ? L.nx - 1 : i);
  j = j < 0 ? 0 : (j > L.ny - 1 ? L.ny - 1 : j);
  const int un = L.pin_map[j * L.nx + i];
  const double dx = x - (L.x0 + ((double)i + 0.5) * L.pitch);
  const double dy = y - (L.y0 + ((double)j + 0.5) * L.pitch);
  const double rr = dx * dx + dy * dy;
  const int nr = L.n_rings[un];
  int r = nr;
  for (int k = 0; k < nr; ++k) {
    const double rad = L.radii[un * L.max_rings + k];
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
template <class R>
MCX_HD int sample_cum(R xi, const R* cum, int n, int last_nz) {
  const R target = xi * cum[n - 1];
  for (int j = 0; j < n; ++j)
    if (target < cum[j]) return j;
  return last_nz;
}

// Isotropic direction from two draws; only (u, v) matter in z-invariant
// geometry (w = 2 xi_mu - 1 sets the in-plane speed sqrt(1 - w^2)).  The _cs
// form takes cos and sin of the azimuth 2 pi xi_phi already evaluated.
MCX_HD void isotropic_uv_cs(double xi_mu, double c, double sn, double* u, double* v) {
  const double w = 2.0 * xi_mu - 1.0;
  const double s2 = 1.0 - w * w;
  const double s = sqrt(s2 > 0.0 ? s2 : 0.0);
  *u = s * c;
  *v = s * sn;
}

MCX_HD void isotropic_uv(double xi_mu, double xi_phi, double* u, double* v,
                         const double* sct = sc_tab()) {
  double c, sn;
  cr_cossin_2pi(xi_phi, sct, &c, &sn);
  isotropic_uv_cs(xi_mu, c, sn, u, v);
}

// ---------------------------------------------------------------------------
// exact fixed-point accumulation: a nonnegative term t becomes the integer
// q = round(t * 2^s) < 2^61; an accumulator is a pair of 64-bit words
// (lo, hi) holding hi * 2^64 + lo.  Adding q is one returning atomic on lo
// plus, when that add wraps around, one increment of hi, so every sum is
// exact and independent of the order of the atomics.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t quantize(double t, double scale) {
  return (uint64_t)__double2ull_rn(t * scale);
}

__device__ __forceinline__ void acc_add(unsigned long long* pair, uint64_t q) {
  if (q == 0) return;
  const unsigned long long old = atomicAdd(pair, (unsigned long long)q);
  if (old + q < old) atomicAdd(pair + 1, 1ull);
}

// Add the 128-bit value w1 * 2^64 + w0.
__device__ __forceinline__ void acc_add128(unsigned long long* pair, unsigned long long w0,
                                           unsigned long long w1) {
  if (w0) {
    const unsigned long long old = atomicAdd(pair, w0);
    if (old + w0 < old) w1 += 1ull;
  }
  if (w1) atomicAdd(pair + 1, w1);
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

// Block-level reservation: every thread of the block calls it with its own
// count; one atomic per block on the counter; the slots of a block are
// contiguous, in thread order.  lds: MAX_WAVES + 2 words, reusable after the
// call returns.
constexpr int MAX_WAVES = 16;

__device__ __forceinline__ uint32_t block_reserve(uint32_t n, uint32_t* counter, uint32_t* lds) {
  const uint32_t lane = lane_id();
  const uint32_t wid = threadIdx.x >> 6;
  const uint32_t nw = (blockDim.x + 63) >> 6;
  uint32_t incl = n;
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
    lds[MAX_WAVES] = run ? atomicAdd(counter, run) : 0u;
  }
  __syncthreads();
  const uint32_t slot = lds[MAX_WAVES] + lds[wid] + incl - n;
  __syncthreads();
  return slot;
}

// Two predicates (one slot each) reserved with one barrier pair and at most
// two atomics per block.
__device__ __forceinline__ void block_append2(bool pa, bool pb, uint32_t* ca, uint32_t* cb,
                                              uint32_t* lds, uint32_t* sa, uint32_t* sb) {
  const uint32_t lane = lane_id();
  const uint32_t wid = threadIdx.x >> 6;
  const uint32_t nw = (blockDim.x + 63) >> 6;
  const unsigned long long ma = __ballot(pa), mb = __ballot(pb);
  const unsigned long long lt = (1ull << lane) - 1ull;
  uint32_t* la = lds;
  uint32_t* lb = lds + MAX_WAVES + 1;
  if (lane == 0) {
    la[wid] = (uint32_t)__popcll(ma);
    lb[wid] = (uint32_t)__popcll(mb);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ra = 0, rb = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      const uint32_t ta = la[w], tb = lb[w];
      la[w] = ra;
      lb[w] = rb;
      ra += ta;
      rb += tb;
    }
    la[MAX_WAVES] = ra ? atomicAdd(ca, ra) : 0u;
    lb[MAX_WAVES] = rb ? atomicAdd(cb, rb) : 0u;
  }
  __syncthreads();
  *sa = la[MAX_WAVES] + la[wid] + (uint32_t)__popcll(ma & lt);
  *sb = lb[MAX_WAVES] + lb[wid] + (uint32_t)__popcll(mb & lt);
  __syncthreads();
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

// Wave-reduced add of per-lane fixed-point sums given as 32-bit halves
// (value = lo + hi * 2^32, each half below 2^56) into a striped pair.
__device__ __forceinline__ void wave_acc_halves(unsigned long long* k_base, unsigned long long lo,
                                                unsigned long long hi) {
  lo = wave_sum(lo);
  hi = wave_sum(hi);
  if (lane_id() == 0 && (lo | hi) != 0ull) {
    // lo + hi * 2^32 as a 128-bit (w1, w0)
    const unsigned long long hl = hi << 32, hh = hi >> 32;
    const unsigned long long w0 = lo + hl;
    const unsigned long long w1 = hh + (w0 < lo ? 1ull : 0ull);
    acc_add128(k_base + 2 * (blockIdx.x % STRIPES), w0, w1);
  }
}

// Wave-reduced add of one fixed-point term (q < 2^61) per lane.
__device__ __forceinline__ void wave_acc(unsigned long long* k_base, uint64_t q) {
  wave_acc_halves(k_base, q & 0xFFFFFFFFull, q >> 32);
}

}  // namespace mcx
