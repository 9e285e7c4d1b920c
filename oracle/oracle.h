/*
 * oracle.h - plain FP64 history-based Monte Carlo k-eigenvalue transport.
 *
 * TEST INFRASTRUCTURE.  This library is the reference that the HIP path is
 * checked against.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load it; the product path never does.  It shares no code,
 * header, table or helper with the HIP path.
 *
 * What it computes follows the paper's statement of the method (Sec. 1:
 * multigroup physics, CSG surface tracking, k-eigenvalue power iteration,
 * replicable counter-based random numbers; Sec. 2: event-based transport with
 * a bank of fission sites; Sec. 5: FP64 throughout).  The paper gives no
 * sampling laws or estimator formulas, so every step is textbook analog Monte
 * Carlo; the exact readings (distance formulas, tie rules, draw order,
 * estimators, combing) are listed in the design notes and restated at each
 * function in oracle.c.
 */
#ifndef MCX_ORACLE_H
#define MCX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ENOMEM = -3,
  ORC_EEXTINCT = -7,
};

enum { ORC_VACUUM = 0, ORC_REFLECT = 1 };
enum { ORC_TAG_SRC = 1, ORC_TAG_TRANSPORT = 2, ORC_TAG_RESAMPLE = 3 };
enum { ORC_ALIVE = 0, ORC_ABSORBED = 1, ORC_LEAKED = 2, ORC_KILLED = 3, ORC_CUTOFF = 4,
       ORC_CENSUS = 5 };

/* per-generation counters (gen_counts[g * ORC_NCOUNT + k]) */
enum {
  ORC_C_SEG = 0,     /* flight segments = collisions + crossings */
  ORC_C_COL = 1,     /* collisions */
  ORC_C_CROSS = 2,   /* surface-crossing events (leaks and reflections included) */
  ORC_C_REFL = 3,    /* crossing events with at least one reflection */
  ORC_C_LEAK = 4,    /* histories ended by leakage */
  ORC_C_ABS = 5,     /* histories ended by absorption */
  ORC_C_KILLED = 6,  /* histories ended by the event guard */
  ORC_C_SITES = 7,   /* fission sites banked (M) */
  ORC_C_SCAT = 8,    /* scatters */
  ORC_C_CUTOFF = 9,  /* histories ended below the energy cutoff (continuous energy) */
  ORC_C_CENSUS = 10, /* histories that reached the end of the time grid (time-dependent) */
  ORC_NCOUNT = 11
};

/* Time-dependent fixed source (Sec. 1: MC/DC's time-dependent mode; Sec. 4
   runs a continuous-energy pin cell in it): every history starts at t = 0,
   a flight of length d lasts d / v (v the group speed, or for continuous
   energy the speed of a neutron of the flight's energy, c sqrt(2 E / m c^2)),
   the flux is tallied per time bin by the length flown in it, and a history
   still flying at the last edge stops there (census).  For continuous energy
   the second tally is the neutron density: the time spent per bin. */
typedef struct {
  int32_t n_tbins;
  const double* t_edges;         /* [n_tbins + 1] increasing, t_edges[0] = 0, s */
  const double* speed;           /* [n_grp] group speeds, cm/s (multigroup only) */
} orc_time;

/* Neutron speed (cm/s) at kinetic energy e (eV), non-relativistic:
   c sqrt(2 e / m_n c^2) with c = 2.99792458e10 cm/s and
   m_n c^2 = 939.56542052e6 eV (CODATA 2018). */
double orc_speed(double e);

/* Continuous-energy data (Sec. 1 lists continuous-energy physics among the
   method's capabilities; Sec. 4 runs a continuous-energy pin cell).
   Pointwise microscopic cross sections on one shared energy grid,
   interpolated linearly in energy; elastic scattering off a target at rest;
   a Watt fission spectrum; constant nu. */
typedef struct {
  int32_t n_nuc, n_pts;
  const double* e_grid;          /* [n_pts] strictly increasing, eV */
  const double* sig_t;           /* [n_nuc][n_pts] total, barns */
  const double* sig_s;           /* [n_nuc][n_pts] elastic scattering */
  const double* sig_f;           /* [n_nuc][n_pts] fission */
  const double* awr;             /* [n_nuc] target mass in neutron masses */
  double nu;                     /* neutrons per fission */
  int32_t max_nuc;               /* row length of the material tables */
  const int32_t* mat_n;          /* [n_mat] nuclides in each material */
  const int32_t* mat_nuc;        /* [n_mat][max_nuc] nuclide indices */
  const double* mat_dens;        /* [n_mat][max_nuc] atoms per barn-cm */
  double watt_a, watt_b;         /* Watt spectrum parameters, eV and 1/eV */
  double e_max;                  /* Watt energies above e_max are drawn again */
  double e_cut;                  /* a scatter below e_cut ends the history (cutoff) */
  int32_t n_ebins;               /* energy bins of the flux tally */
  const double* e_edges;         /* [n_ebins + 1] increasing bin edges, eV */
  double src_energy;             /* > 0: every source particle starts at this energy
                                    (eV, no draws); 0: Watt spectrum */
} orc_ce;

typedef struct {
  /* geometry: nx x ny lattice, square pitch, lower-left corner (x0, y0) */
  int32_t nx, ny;
  double pitch, x0, y0;
  int32_t bc[4];                 /* xmin, xmax, ymin, ymax */
  int32_t n_univ, max_rings;
  const int32_t* n_rings;        /* [n_univ] */
  const double* radii;           /* [n_univ][max_rings] */
  const int32_t* mats;           /* [n_univ][max_rings + 1] */
  const int32_t* pin_map;        /* [ny][nx] */
  /* multigroup cross sections */
  int32_t n_mat, n_grp;
  const double* sig_t;           /* [n_mat][n_grp] */
  const double* sig_s;           /* [n_mat][n_grp][n_grp], row = outgoing spectrum */
  const double* nu_sig_f;        /* [n_mat][n_grp] */
  const double* chi;             /* [n_mat][n_grp] */
  /* run */
  uint64_t seed;
  int64_t n_per_gen;
  int32_t n_gen, n_inactive;
  int32_t fixed_source;          /* 1: fission is capture, fresh source each batch */
  uint64_t problem_id;
  int32_t ent_nx, ent_ny;
  int64_t max_events;
  int32_t n_threads;
  /* optional start states [n_per_gen][6] = x, y, u, v, w, g (energy in eV
     for continuous energy) (fixed source, first batch only); NULL samples
     the source */
  const double* ext_state;
  /* continuous-energy physics instead of the multigroup tables above
     (n_mat still counts the materials; n_grp, sig_t, sig_s, nu_sig_f and
     chi are unused); NULL = multigroup */
  const orc_ce* ce;
  /* time-dependent fixed source (multigroup, fixed_source = 1), or NULL */
  const orc_time* time;
} orc_problem;

typedef struct {
  int32_t n_seg, n_col, n_cross, n_refl;
  int32_t fate, n_sites, g_final;
  uint32_t ctr_final;            /* transport-stream draws consumed */
  double tl_sum;                 /* total track length */
  double kcol_sum;               /* sum of nu_sig_f / sig_t over collisions */
  double x_final, y_final;
  double e_final;                /* final energy (continuous energy), else 0 */
  double t_final;                /* final time (time-dependent), else 0 */
} orc_record;

/* One flight of a history (event log): where it ended, its length, and the
   state it flew in. */
typedef struct {
  double x, y;                   /* position after the flight */
  double d;                      /* flight length */
  double e;                      /* energy (continuous energy), else 0 */
  int32_t cell, region, group;   /* lattice cell j * nx + i, ring region, group or energy bin */
  int32_t type;                  /* 1 collision, 2 surface crossing, 3 leak, 4 census */
} orc_event;

typedef struct {
  double* gen_k;                 /* [n_gen][3]: k_col, k_tl, k_abs (required) */
  double* gen_entropy;           /* [n_gen] (required) */
  int64_t* gen_counts;           /* [n_gen][ORC_NCOUNT] (required) */
  double k_mean[3], k_sigma[3];  /* over active generations */
  double* flux_mean;             /* [n_bins] or NULL */
  double* flux_sigma;
  double* prod_mean;
  double* prod_sigma;
  double* gen_flux;              /* [n_gen][n_bins] or NULL */
  double* gen_prod;
  orc_record* records;           /* [n_gen][n_per_gen] or NULL */
  double* bank;                  /* last canonical bank [bank_cap][3] = x, y, g or NULL */
  int64_t bank_cap;
  int64_t bank_len;              /* out */
  orc_event* events;             /* [n_gen][n_per_gen][event_cap] flights, or NULL */
  int32_t event_cap;             /* flights logged per history (later ones are not) */
  double* source;                /* [n_gen][n_per_gen][3] = x, y, g (energy in eV for
                                    continuous energy) of every generation's source
                                    sites, or NULL */
  char errmsg[256];
} orc_output;

/* Tally bins: ((cell * (max_rings + 1)) + region) * n_grp + group,
   cell = j * nx + i (continuous energy: n_ebins energy bins in place of the
   groups; the production tally is then not kept and reads zero;
   time-dependent: that index times n_tbins plus the time bin). */
int64_t orc_n_bins(const orc_problem* p);

int orc_run(const orc_problem* p, orc_output* out);

/* Histories ids[0..n_ids) of the first generation only, with the records
   orc_run would give them (out->records: n_ids records in list order; no
   other output).  For checking a sample of a run too large to compute
   whole. */
int orc_histories(const orc_problem* p, const int64_t* ids, int64_t n_ids, orc_output* out);

/* building blocks, exported for the pins */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double orc_uniform(uint64_t word);
double orc_stream_uniform(uint64_t seed, uint64_t tag, uint64_t id, uint64_t gen,
                          uint64_t prob, uint32_t draw);
double orc_dist_plane(double x, double lo, double hi, double u);
double orc_dist_cylinder(double dx, double dy, double u, double v, double radius,
                         int inside);
double orc_cr_log(double x);
void orc_cr_cossin_2pi(double t, double* c, double* s);
void orc_isotropic(double xi_mu, double xi_phi, double out[3]);
int orc_sample_cdf(double xi, const double* weights, int n);
void orc_comb(int64_t n, int64_t m, double xi0, int64_t* idx);
double orc_entropy(const int64_t* counts, int64_t n_bins, int64_t m);
double orc_neumaier(const double* v, int64_t n);
int orc_ce_interval(const double* grid, int n, double e);
void orc_ce_macro(const orc_ce* ce, int m, double e, double out[3]);
double orc_watt_attempt(double a, double b, double xi1, double xi2, double xi3, double xi4);
double orc_elastic(double awr, double e, double xi_mu, double* mu_lab);
void orc_rotate(double mu, double xi_phi, double dir[3]);

#ifdef __cplusplus
}
#endif
#endif
