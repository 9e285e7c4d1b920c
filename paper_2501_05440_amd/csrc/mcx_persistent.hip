// mcx_persistent.hip - persistent engine: block-local event queues with refill.
//
// One launch processes every history of a run (a k-eigenvalue generation of
// one problem, or a batch of independent fixed-source problems).  Each
// workgroup keeps up to S particles in LDS slots and loops:
//
//   refill   when fewer than tau slots are live, reserve a chunk of history
//            indices from one global counter and give birth to them in the
//            free slots (source sampling for fixed-source problems, the
//            combed bank for k-eigenvalue generations);
//   advance  the dense list of live slots, one flight each (the same
//            segment() as the event kernels);
//   collide  the dense list of slots whose flight ended in a collision.
//
// The lists are rebuilt by block scans in slot order, so every phase runs
// its lanes on the same event (the paper's event-based decomposition, Sec. 2)
// without kernel launches or global queues between events, and the particle
// state never leaves LDS.  Every history performs exactly the operations of
// the event kernels in the same order, so per-history results are identical
// and the exact sums make every estimator independent of the schedule.
//
// Per-history results are written once, at death, to per-history outputs;
// k_hist_reduce turns them into per-problem estimators and counters.
#include "mcx_kernels_common.hpp"

namespace mcx {

// slot states; a collision in fissile material is SL_COLF when the collide
// list is sorted (fissile collisions first, so the fission-site loop runs in
// the same waves), else SL_COL
enum : uint8_t { SL_FREE = 0, SL_LIVE = 1, SL_COL = 2, SL_COLF = 3 };

template <class R, int S>
struct SlotMem {
  double x[S], y[S];
  R u[S], v[S];
  uint32_t cell[S], gs[S], ctr[S], hid[S];
  unsigned long long kc_lo[S], kc_hi[S];
  uint32_t nseg[S], ncol[S], ncross[S], nrefl[S], nscat[S];
  uint16_t prob[S];
  uint8_t state[S];
  uint16_t list[S];
  uint32_t scan[MAX_WAVES + 2];
  uint32_t n_list, n_free, got;
  uint32_t base;
  uint32_t exhausted;
  uint32_t win_move, win_next;  // the tally window moves to bin win_next
};

// Flux words staged per block: a window of at most P_WIN_BINS tally bins
// (16 B each) after the slots in LDS.  Histories enter a block in global
// order, so a block works on a few consecutive problems of a batch at a
// time; the window starts at the first bin of the problem of the chunk a
// refill takes, and moves (after adding its words to device memory) when
// that problem's bins leave it.  Flights of a bin outside it add to device
// memory directly.
constexpr uint32_t P_WIN_BINS = 256;

template <class R, int S>
__device__ __forceinline__ Part<R> slot_load(const SlotMem<R, S>& M, int s, const ProbDesc* P) {
  Part<R> p;
  p.x = M.x[s];
  p.y = M.y[s];
  p.u = M.u[s];
  p.v = M.v[s];
  const uint32_t c = M.cell[s];
  p.i = cell_i(c);
  p.j = cell_j(c);
  p.r = cell_r(c);
  p.g = (int)(M.gs[s] & 0xFFFFu);
  p.nsite = M.gs[s] >> 16;
  p.ctr = M.ctr[s];
  // the random-number id of a history is its index within its problem
  p.id = (uint32_t)(M.hid[s] - (P ? P[M.prob[s]].hist_base : 0ull));
  p.nseg = M.nseg[s];
  return p;
}

template <class R, int S>
__device__ __forceinline__ void slot_store(SlotMem<R, S>& M, int s, const Part<R>& p) {
  M.x[s] = p.x;
  M.y[s] = p.y;
  M.u[s] = p.u;
  M.v[s] = p.v;
  M.cell[s] = pack_cell(p.i, p.j, p.r);
  M.gs[s] = (uint32_t)p.g | (p.nsite << 16);
  M.ctr[s] = p.ctr;
}

// List (in slot order) of the slots whose state is in the bit set `want`
// (bit k = state k), written from M.list[base]; each thread owns S / PB
// consecutive slots.  Returns the count.
template <class R, int PB, int S>
__device__ __forceinline__ uint32_t build_list_set(SlotMem<R, S>& M, uint32_t want,
                                                   uint32_t base) {
  constexpr int K = S / PB;
  const int s0 = threadIdx.x * K;
  uint32_t n = 0;
#pragma unroll
  for (int e = 0; e < K; ++e) n += (want >> M.state[s0 + e]) & 1u;
  uint32_t total;
  uint32_t off = base + block_excl_scan(n, M.scan, &total);
#pragma unroll
  for (int e = 0; e < K; ++e)
    if ((want >> M.state[s0 + e]) & 1u) M.list[off++] = (uint16_t)(s0 + e);
  if (threadIdx.x == 0) M.n_list = base + total;
  __syncthreads();
  return total;
}

template <class R, int PB, int S>
__device__ __forceinline__ uint32_t build_list(SlotMem<R, S>& M, uint8_t want) {
  return build_list_set<R, PB, S>(M, 1u << want, 0);
}


template <class R, int S>
__device__ __forceinline__ void slot_death(SlotMem<R, S>& M, int s, const Part<R>& p, int fate,
                                           uint64_t q_kabs, const Accum& A, const HistOut& H) {
  const uint64_t h = M.hid[s];
  A.nsite_id[h] = p.nsite;
  H.kabs[h] = q_kabs;
  H.kcol[2 * h + 0] = M.kc_lo[s];
  H.kcol[2 * h + 1] = M.kc_hi[s];
  uint32_t* c = H.cnt + (size_t)h * HO_N;
  c[HO_SEG] = M.nseg[s];
  c[HO_COL] = M.ncol[s];
  c[HO_CROSS] = M.ncross[s];
  c[HO_REFL] = M.nrefl[s];
  c[HO_SCAT] = M.nscat[s];
  c[HO_SITES] = p.nsite;
  c[HO_FATE] = (uint32_t)fate;
  M.state[s] = SL_FREE;
}

template <class R, int PB, int S>
__global__ void __launch_bounds__(PB) k_persistent(Tables T0, uint32_t gen, Accum A, HistOut H,
                                                   uint32_t* work, uint32_t tau,
                                                   const double* sx, const double* sy,
                                                   const int32_t* sg,
                                                   const uint32_t* prev_status, int sort) {
  Tables T = kernel_tables<R, false>(T0);
  extern __shared__ unsigned char lds_raw[];
  SlotMem<R, S>& M = *reinterpret_cast<SlotMem<R, S>*>(lds_raw);
  const ProbDesc* P = T.probs;
  const uint64_t total = T.n_hist_total;
  const double k_used = *A.k_used;
  const Records Rc{};

  // after a failed generation (or a source that could not be sampled
  // before this launch) the generation runs empty, as in the event engine;
  // every block takes the same decision from words no block of this launch
  // writes
  if ((prev_status && *prev_status != 0u) || (sx && (*A.status & ST_SOURCE))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(A.status, ST_SKIPPED);
    return;
  }

  for (int s = threadIdx.x; s < S; s += PB) M.state[s] = SL_FREE;
  if (threadIdx.x == 0) M.exhausted = 0;
  lds_tally_clear(T);  // (a barrier)

  for (;;) {
    // ---------------- refill ----------------
    const uint32_t n_live = build_list<R, PB, S>(M, SL_LIVE);
    if (threadIdx.x == 0) {
      M.got = 0;
      if (!M.exhausted && n_live < tau) {
        const uint32_t want = (uint32_t)S - n_live;
        const uint32_t b = atomicAdd(work, want);
        if ((uint64_t)b >= total) {
          M.exhausted = 1;
        } else {
          M.base = b;
          M.got = (uint32_t)min((uint64_t)want, total - b);
          if ((uint64_t)b + want >= total) M.exhausted = 1;
        }
      }
      // the tally window follows the problem of the new chunk
      M.win_move = 0;
      if (M.got && P) {
        const int pi0 = problem_of(P, T.n_probs, (uint64_t)M.base);
        const uint32_t lo0 = (uint32_t)P[pi0].geo.bin_base;
        const uint32_t nb0 = (uint32_t)P[pi0].n_bins;
        if (lo0 < T.lds_bin_lo || lo0 + min(nb0, T.lds_bin_n) > T.lds_bin_lo + T.lds_bin_n) {
          M.win_move = 1;
          M.win_next = lo0;
        }
      }
    }
    __syncthreads();
    if (M.win_move) {
      lds_tally_flush(T, A, true);
      T.lds_bin_lo = M.win_next;
    }
    const uint32_t got = M.got;
    if (got) {
      build_list<R, PB, S>(M, SL_FREE);  // got <= number of free slots
      for (uint32_t t = threadIdx.x; t < got; t += PB) {
        const int s = M.list[t];
        const uint64_t h = (uint64_t)M.base + t;
        const int pi = P ? problem_of(P, T.n_probs, h) : 0;
        const Geo L = P ? P[pi].geo : T.geo;  // a copy keeps T out of scratch
        const uint64_t seed = P ? P[pi].seed : T.seed;
        const uint64_t prob = P ? P[pi].prob : T.prob;
        const uint64_t lid = h - (P ? P[pi].hist_base : 0ull);
        Part<R> p;
        if (sx) {
          p.x = sx[h];
          p.y = sy[h];
          p.g = sg[h];
        } else {
          int32_t g0;
          if (!sample_source(T, L, seed, prob, lid, gen, &p.x, &p.y, &g0))
            atomicOr(A.status, ST_SOURCE);
          p.g = g0;
        }
        Stream rs(seed, TAG_TRANSPORT, lid, gen, prob, 0);
        const R xm = Prec<R>::xi(rs.next());
        const R xp = Prec<R>::xi(rs.next());
        Prec<R>::iso(xm, xp, &p.u, &p.v);
        locate(L, p.x, p.y, &p.i, &p.j, &p.r);
        p.nsite = 0;
        p.ctr = rs.draw;
        slot_store(M, s, p);
        M.hid[s] = (uint32_t)h;
        M.prob[s] = (uint16_t)pi;
        M.kc_lo[s] = 0;
        M.kc_hi[s] = 0;
        M.nseg[s] = M.ncol[s] = M.ncross[s] = M.nrefl[s] = M.nscat[s] = 0;
        M.state[s] = SL_LIVE;
      }
      __syncthreads();
    }
    const uint32_t n_adv = got ? build_list<R, PB, S>(M, SL_LIVE) : n_live;
    if (n_adv == 0) {
      if (M.exhausted) break;
      continue;
    }

    // ---------------- advance ----------------
    // (M.list holds the live slots: either rebuilt above or from the refill check)
    for (uint32_t t = threadIdx.x; t < n_adv; t += PB) {
      const int s = M.list[t];
      Part<R> p = slot_load(M, s, P);
      const int pi = P ? M.prob[s] : 0;
      const Geo L = P ? P[pi].geo : T.geo;  // a copy keeps T out of scratch
      if ((int64_t)M.nseg[s] >= T.max_events) {
        slot_death(M, s, p, FATE_KILLED, 0, A, H);
        continue;
      }
      Stream rs(P ? P[pi].seed : T.seed, TAG_TRANSPORT, p.id, gen, P ? P[pi].prob : T.prob,
                p.ctr);
      bool refl = false;
      const int ev = segment<R, false, false, Stream, true>(T, L, p, rs, A, Rc, &refl);
      p.ctr = rs.draw;
      M.nseg[s] += 1;
      if (ev == EV_CROSS || ev == EV_LEAK) M.ncross[s] += 1;
      if (refl) M.nrefl[s] += 1;
      slot_store(M, s, p);
      if (ev == EV_LEAK || ev == EV_CENSUS) {
        slot_death(M, s, p, ev == EV_LEAK ? FATE_LEAKED : FATE_CENSUS, 0, A, H);
      } else if (ev == EV_COLLIDE) {
        uint8_t st = SL_COL;
        if (sort) {
          const int m = L.mats[L.pin_map[p.j * L.nx + p.i] * L.mr1 + p.r];
          if (T.fissile[m]) st = SL_COLF;
        }
        M.state[s] = st;
      } else {
        M.state[s] = SL_LIVE;
      }
    }
    __syncthreads();

    // ---------------- collide ----------------
    uint32_t n_col;
    if (sort) {
      const uint32_t nf = build_list_set<R, PB, S>(M, 1u << SL_COLF, 0);
      n_col = nf + build_list_set<R, PB, S>(M, 1u << SL_COL, nf);
    } else {
      n_col = build_list_set<R, PB, S>(M, (1u << SL_COL) | (1u << SL_COLF), 0);
    }
    for (uint32_t t0 = 0; t0 < n_col; t0 += PB) {
      const uint32_t t = t0 + threadIdx.x;
      const bool valid = t < n_col;
      const int s = valid ? M.list[t] : 0;
      Part<R> p;
      ColXS<R> x{0, R(1), R(0)};
      uint32_t nf = 0;
      int pi = 0;
      Stream rs(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
      if (valid) {
        p = slot_load(M, s, P);
        pi = P ? M.prob[s] : 0;
        const Geo L = P ? P[pi].geo : T.geo;  // a copy keeps T out of scratch
        rs = Stream(P ? P[pi].seed : T.seed, TAG_TRANSPORT, p.id, gen, P ? P[pi].prob : T.prob,
                    p.ctr);
        x = col_xs(T, L, p);
        const uint64_t q = quantize((double)(x.nusf / x.st), T.q_kcol);
        M.kc_lo[s] += q & 0xFFFFFFFFull;
        M.kc_hi[s] += q >> 32;
        M.ncol[s] += 1;
        nf = fission_count(T, x, rs, k_used);
      }
      const uint32_t slot = block_reserve(nf, A.n_fis, M.scan);
      if (valid) {
        uint64_t qa = 0;
        const bool alive = collide_rest<R, false>(T, p, rs, x, nf, slot, A, &qa);
        p.ctr = rs.draw;
        slot_store(M, s, p);
        if (alive) {
          M.nscat[s] += 1;
          M.state[s] = SL_LIVE;
        } else {
          slot_death(M, s, p, FATE_ABSORBED, qa, A, H);
        }
      }
    }
    __syncthreads();
  }
  lds_tally_flush(T, A);
}

// Per-problem reduction of the per-history outputs: exact counter sums and
// 128-bit estimator sums.  Grid: blocks x problems; each block reduces a
// strided share of its problem's histories and adds it atomically (exact
// integer sums, so the order does not matter).  Single-problem runs add into
// the generation accumulators, batches into per-problem totals.
__global__ void __launch_bounds__(256) k_hist_reduce(Tables T, HistOut H, Accum A,
                                                     unsigned long long* prob_cnt,
                                                     unsigned long long* prob_k) {
  __shared__ unsigned long long red[256];
  const int pi = blockIdx.y;
  const uint64_t base = T.probs ? T.probs[pi].hist_base : 0ull;
  const uint64_t n = T.probs ? T.probs[pi].n_hist : T.n_hist_total;
  unsigned long long v[N_CNT + 4];
  for (int e = 0; e < N_CNT + 4; ++e) v[e] = 0;
  for (uint64_t h = base + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < base + n;
       h += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t* q = H.cnt + (size_t)h * HO_N;
    v[CNT_SEG] += q[HO_SEG];
    v[CNT_COL] += q[HO_COL];
    v[CNT_CROSS] += q[HO_CROSS];
    v[CNT_REFL] += q[HO_REFL];
    v[CNT_SCAT] += q[HO_SCAT];
    v[CNT_SITES] += q[HO_SITES];
    v[CNT_LEAK] += q[HO_FATE] == FATE_LEAKED;
    v[CNT_ABS] += q[HO_FATE] == FATE_ABSORBED;
    v[CNT_KILLED] += q[HO_FATE] == FATE_KILLED;
    v[CNT_CUTOFF] += q[HO_FATE] == FATE_CUTOFF;
    v[CNT_CENSUS] += q[HO_FATE] == FATE_CENSUS;
    v[N_CNT + 0] += H.kcol[2 * h + 0];
    v[N_CNT + 1] += H.kcol[2 * h + 1];
    v[N_CNT + 2] += H.kabs[h] & 0xFFFFFFFFull;
    v[N_CNT + 3] += H.kabs[h] >> 32;
  }
  for (int e = 0; e < N_CNT + 4; ++e) {
    red[threadIdx.x] = v[e];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    v[e] = red[0];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  // halves (lo + hi * 2^32) as 128-bit pairs
  unsigned long long kc0, kc1, ka0, ka1;
  kc0 = v[N_CNT] + (v[N_CNT + 1] << 32);
  kc1 = (v[N_CNT + 1] >> 32) + (kc0 < v[N_CNT] ? 1ull : 0ull);
  ka0 = v[N_CNT + 2] + (v[N_CNT + 3] << 32);
  ka1 = (v[N_CNT + 3] >> 32) + (ka0 < v[N_CNT + 2] ? 1ull : 0ull);
  if (T.probs) {
    for (int e = 0; e < N_CNT; ++e)
      if (v[e]) atomicAdd(prob_cnt + (size_t)pi * N_CNT + e, v[e]);
    acc_add128(prob_k + (size_t)pi * 4 + 0, kc0, kc1);
    acc_add128(prob_k + (size_t)pi * 4 + 2, ka0, ka1);
  } else {
    const unsigned stripe = blockIdx.x % STRIPES;
    for (int e = 0; e < N_CNT; ++e)
      if (v[e]) atomicAdd(A.cnt + e * STRIPES + stripe, v[e]);
    acc_add128(A.k + K_COL * STRIPES * 2 + 2 * stripe, kc0, kc1);
    acc_add128(A.k + K_ABS * STRIPES * 2 + 2 * stripe, ka0, ka1);
  }
}

// Per-problem flux and production tallies and estimators of a batch (one
// block per problem): flux exact sums / n, production nu_sig_f * flux, k_tl
// the compensated sum of the production, k_col and k_abs from the reduced
// 128-bit sums.
__global__ void __launch_bounds__(256) k_batch_results(Tables T, Accum A,
                                                       const unsigned long long* prob_k,
                                                       double* flux_out, double* prod_out,
                                                       double* k_out) {
  __shared__ double ps[256], pc[256];
  const int pi = blockIdx.x;
  const ProbDesc& D = T.probs[pi];
  const Geo& L = D.geo;
  const int nb = D.n_bins;
  const int per_cell = L.mr1 * T.G;
  const double n = (double)D.n_hist;
  double s = 0.0, cmp = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int gb = L.bin_base + b;
    const double flux = flux_total(A.tally + 2 * (size_t)gb, T.tally_stripes,
                                   2 * (size_t)T.n_bins, A.tally_t + 2 * (size_t)gb) /
                        T.q_flux;
    const int cell = b / per_cell;
    const int r = (b / T.G) % L.mr1;
    const int g = b % T.G;
    const int m = L.mats[L.pin_map[cell] * L.mr1 + r];
    const double prod = T.nusf[m * T.G + g] * flux;
    flux_out[gb] = flux / n;
    prod_out[gb] = prod / n;
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
    const unsigned long long* q = prob_k + (size_t)pi * 4;
    k_out[(size_t)pi * 3 + 0] = u128_to_double(q[0], q[1]) / T.q_kcol / n;
    k_out[(size_t)pi * 3 + 1] = (a + ac) / n;
    k_out[(size_t)pi * 3 + 2] = u128_to_double(q[2], q[3]) / T.q_kabs / n;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <class R, int PB, int S>
static hipError_t launch_p(unsigned grid, const Tables& T, uint32_t gen, const Accum& A,
                           const HistOut& H, uint32_t* work, uint32_t tau, const double* sx,
                           const double* sy, const int32_t* sg, const uint32_t* prev_status,
                           int sort, hipStream_t s) {
  Tables Tw = T;
  Tw.lds_tally_off = (uint32_t)((sizeof(SlotMem<R, S>) + 15) & ~(size_t)15);
  Tw.lds_bin_lo = 0;
  Tw.lds_bin_n = std::min<uint32_t>((uint32_t)T.n_bins, P_WIN_BINS);
  const size_t lds = Tw.lds_tally_off + 16 * (size_t)Tw.lds_bin_n;
  hipLaunchKernelGGL((k_persistent<R, PB, S>), dim3(grid), dim3(PB), lds, s, Tw, gen, A, H, work,
                     tau, sx, sy, sg, prev_status, sort);
  return hipGetLastError();
}

hipError_t launch_persistent(int prec, const PersistentCfg& cfg, const Tables& T, uint32_t gen,
                             const Accum& A, unsigned long long* h_kcol,
                             unsigned long long* h_kabs, uint32_t* h_cnt, uint32_t* work,
                             const double* sx, const double* sy, const int32_t* sg,
                             const uint32_t* prev_status, hipStream_t s) {
  const HistOut H{h_kcol, h_kabs, h_cnt};
  const unsigned grid = (unsigned)std::max(1, cfg.grid);
  const int S = cfg.slots;
  const uint32_t tau = (uint32_t)std::max(1, (int)(cfg.tau * (double)S));
#define MCX_P(RT, PBV, SV)                                                                   \
  if (cfg.block == PBV && S == SV)                                                           \
    return launch_p<RT, PBV, SV>(grid, T, gen, A, H, work, tau, sx, sy, sg, prev_status, cfg.sort, s);
  if (prec == 0) {
    MCX_P(double, 128, 256)
    MCX_P(double, 128, 512)
    MCX_P(double, 256, 256)
    MCX_P(double, 256, 512)
  } else {
    MCX_P(float, 128, 256)
    MCX_P(float, 128, 512)
    MCX_P(float, 256, 256)
    MCX_P(float, 256, 512)
  }
#undef MCX_P
  return hipErrorInvalidValue;
}

size_t persistent_lds_bytes(int prec, int block, int slots) {
  (void)block;
  size_t b = 0;
  if (prec == 0) {
    if (slots == 256) b = sizeof(SlotMem<double, 256>);
    if (slots == 512) b = sizeof(SlotMem<double, 512>);
  } else {
    if (slots == 256) b = sizeof(SlotMem<float, 256>);
    if (slots == 512) b = sizeof(SlotMem<float, 512>);
  }
  return b ? ((b + 15) & ~(size_t)15) + 16 * (size_t)P_WIN_BINS : 0;
}

bool persistent_config_valid(int block, int slots) {
  return (block == 128 && (slots == 256 || slots == 512)) ||
         (block == 256 && (slots == 256 || slots == 512));
}

hipError_t launch_hist_reduce(const Tables& T, int n_probs, unsigned long long* h_kcol,
                              unsigned long long* h_kabs, uint32_t* h_cnt, const Accum& A,
                              unsigned long long* prob_cnt, unsigned long long* prob_k,
                              hipStream_t s) {
  const HistOut H{h_kcol, h_kabs, h_cnt};
  // single problems: enough blocks to stream the outputs; batches: a few per problem
  const unsigned bx = T.probs ? 8u : 512u;
  hipLaunchKernelGGL(k_hist_reduce, dim3(bx, std::max(1, n_probs)), dim3(256), 0, s, T, H, A,
                     prob_cnt, prob_k);
  return hipGetLastError();
}

hipError_t launch_batch_results(const Tables& T, int n_probs, const Accum& A,
                                const unsigned long long* prob_k, double* flux, double* prod,
                                double* k_out, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_results, dim3(n_probs), dim3(256), 0, s, T, A, prob_k, flux, prod,
                     k_out);
  return hipGetLastError();
}

}  // namespace mcx
