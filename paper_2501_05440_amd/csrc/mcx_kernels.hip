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
#include "mcx_kernels_common.hpp"

namespace mcx {

__global__ void k_source(Tables T, uint32_t gen, uint32_t n, double* sx, double* sy,
                         int32_t* sg, uint32_t* status) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  if (!sample_source(T, T.geo, T.seed, T.prob, id, gen, &sx[id], &sy[id], &sg[id]))
    atomicOr(status, ST_SOURCE);
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
  locate(T.geo, p.x, p.y, &p.i, &p.j, &p.r);
  p.nsite = 0;
  p.ctr = rs.draw;
  p.id = id;
  p.nseg = 0;
  p.t = 0.0;
  store_part(out, id, p);
}

// ---------------------------------------------------------------------------
// event kernels
// ---------------------------------------------------------------------------

// Advance every particle of the input bank: flights through the lattice
// until a collision, a leak, the event guard, or `flights` flights (1 is the
// one-event-per-launch form; more keeps a particle in the kernel across its
// surface crossings, with the same operations in the same order).
// Particles still flying go to the live bank of the next iteration,
// particles that collide go to the collision bank; leaks and guard kills end
// here.  Block 0 clears the counters the next iteration appends to.
template <class R, bool REC, bool LDS>
__global__ void __launch_bounds__(1024) k_advance(Tables T0, uint32_t gen, uint32_t flights, Bank in,
                                                  const uint32_t* __restrict__ n_in_p, Bank live,
                                                  uint32_t* n_live, Bank col, uint32_t* n_col,
                                                  Accum A, Records Rc, uint32_t* clr_live,
                                                  uint32_t* clr_col) {
  const uint32_t n_in = *n_in_p;
  // blocks past the live count (grids are sized from a bound) skip the copy
  const Tables T = kernel_tables<R, LDS>(T0, blockIdx.x * blockDim.x < n_in);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *clr_live = 0;
    *clr_col = 0;
  }
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  int ev = EV_NONE;
  uint32_t c_seg = 0, c_cross = 0, c_refl = 0;
  Part<R> p;
  if (k < n_in) {
    p = load_part<R>(in, k);
    LockStream rs(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    for (uint32_t f = 0; f < flights; ++f) {
      if ((int64_t)p.nseg >= T.max_events) {
        ev = EV_KILL;
        break;
      }
      bool refl = false;
      rs.top_up();
      ev = segment<R, REC, false, LockStream>(T, T.geo, p, rs, A, Rc, &refl);
      p.nseg += 1;
      c_seg += 1;
      c_cross += (ev == EV_CROSS || ev == EV_LEAK) ? 1u : 0u;
      c_refl += refl ? 1u : 0u;
      if (ev != EV_CROSS) break;
    }
    p.ctr = rs.draw;
    if (ev == EV_KILL) die<R, REC>(p, FATE_KILLED, A, Rc);
    if (ev == EV_LEAK) die<R, REC>(p, FATE_LEAKED, A, Rc);
    if (ev == EV_CENSUS) die<R, REC>(p, FATE_CENSUS, A, Rc);
  }
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  uint32_t pl, pc;
  block_append2(ev == EV_CROSS, ev == EV_COLLIDE, n_live, n_col, lds, &pl, &pc);
  if (ev == EV_CROSS) store_part(live, pl, p);
  if (ev == EV_COLLIDE) store_part(col, pc, p);
  wave_count(A.cnt + CNT_SEG * STRIPES, c_seg);
  wave_count(A.cnt + CNT_CROSS * STRIPES, c_cross);
  wave_count(A.cnt + CNT_REFL * STRIPES, c_refl);
  wave_flag(A.cnt + CNT_LEAK * STRIPES, ev == EV_LEAK);
  wave_flag(A.cnt + CNT_KILLED * STRIPES, ev == EV_KILL);
  wave_flag(A.cnt + CNT_CENSUS * STRIPES, ev == EV_CENSUS);
  wave_flag(A.cnt + CNT_ADV_ITEMS * STRIPES, k < n_in);
  wave_count(A.cnt + CNT_ADV_SEGS * STRIPES, c_seg);
}

// Advance with the flux tally staged in LDS.  Each flight of k_advance adds
// its exact fixed-point flux term to device memory with one atomic, and
// those atomics (one per flight, executed beyond the compute unit) are what
// bounds that kernel.  Here a block keeps its own flux words in LDS: per bin
// the sums of the low and high 32-bit halves of its terms, added with LDS
// atomics, and walks the input bank in chunks of blockDim particles
// (grid-stride), so one block serves many particles.  At the end it adds
// each nonzero bin to the bin's 128-bit device pair once (the exact sum
// lo + hi 2^32 of the block's terms).  Every other operation is k_advance's,
// per chunk: particles still flying go to the live bank, colliding ones to
// the collision bank (one atomic per block, queue and chunk).  The sums are
// exact, so results equal k_advance's for any grid.  Needs the table copies
// in LDS; the launcher sizes the dynamic LDS as tables + 16 B per bin.
template <class R, bool REC>
// 768 threads = 12 wavefronts, three per SIMD, so two blocks (two copies
// of the LDS flux words) give six wavefronts per SIMD; the register budget
// that needs is asked for explicitly (a few values spill).
__global__ void __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(6, 8))) k_advance_lt(Tables T0, uint32_t gen, uint32_t flights,
                                                     Bank in, const uint32_t* __restrict__ n_in_p,
                                                     Bank live, uint32_t* n_live, Bank col,
                                                     uint32_t* n_col, Accum A, Records Rc,
                                                     uint32_t* clr_live, uint32_t* clr_col) {
  const uint32_t n_in = *n_in_p;
  const bool any = blockIdx.x * blockDim.x < n_in;
  const Tables T = kernel_tables<R, true>(T0, any);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *clr_live = 0;
    *clr_col = 0;
  }
  if (!any) return;  // the whole block
  lds_tally_clear(T);

  uint32_t c_seg = 0, c_cross = 0, c_refl = 0, c_leak = 0, c_kill = 0, c_cen = 0, c_items = 0;
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  const uint32_t step = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n_in; base += step) {
    const uint32_t k = base + threadIdx.x;
    int ev = EV_NONE;
    Part<R> p;
    if (k < n_in) {
      c_items += 1;
      p = load_part<R>(in, k);
      LockStream rs(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
      for (uint32_t f = 0; f < flights; ++f) {
        if ((int64_t)p.nseg >= T.max_events) {
          ev = EV_KILL;
          break;
        }
        bool refl = false;
        rs.top_up();
        ev = segment<R, REC, false, LockStream, true>(T, T.geo, p, rs, A, Rc, &refl);
        p.nseg += 1;
        c_seg += 1;
        c_cross += (ev == EV_CROSS || ev == EV_LEAK) ? 1u : 0u;
        c_refl += refl ? 1u : 0u;
        if (ev != EV_CROSS) break;
      }
      p.ctr = rs.draw;
      if (ev == EV_KILL) {
        die<R, REC>(p, FATE_KILLED, A, Rc);
        c_kill += 1;
      }
      if (ev == EV_LEAK) {
        die<R, REC>(p, FATE_LEAKED, A, Rc);
        c_leak += 1;
      }
      if (ev == EV_CENSUS) {
        die<R, REC>(p, FATE_CENSUS, A, Rc);
        c_cen += 1;
      }
    }
    uint32_t pl, pc;
    block_append2(ev == EV_CROSS, ev == EV_COLLIDE, n_live, n_col, lds, &pl, &pc);
    if (ev == EV_CROSS) store_part(live, pl, p);
    if (ev == EV_COLLIDE) store_part(col, pc, p);
  }
  wave_count(A.cnt + CNT_SEG * STRIPES, c_seg);
  wave_count(A.cnt + CNT_CROSS * STRIPES, c_cross);
  wave_count(A.cnt + CNT_REFL * STRIPES, c_refl);
  wave_count(A.cnt + CNT_LEAK * STRIPES, c_leak);
  wave_count(A.cnt + CNT_KILLED * STRIPES, c_kill);
  wave_count(A.cnt + CNT_CENSUS * STRIPES, c_cen);
  wave_count(A.cnt + CNT_ADV_ITEMS * STRIPES, c_items);
  wave_count(A.cnt + CNT_ADV_SEGS * STRIPES, c_seg);
  lds_tally_flush(T, A);
}

// Advance with lanes refilled from the block's chunk of the input bank.
// Block b owns items [b C, (b + 1) C), C = rounds x blockDim.  A lane runs
// its particle's flights (up to `flights`, stopping at a collision, a leak,
// the census or the guard, exactly as k_advance does), then writes the
// particle back to its input slot, marks the slot's outcome in LDS and takes
// the next unstarted item of the chunk, so the wave's lanes stay busy until
// the chunk runs out instead of idling behind the wave's longest chain of
// crossings.  A wave takes new items only once at least REFILL_MIN of its
// lanes are free (or none is busy), so each refill's loads serve many lanes.
// At the end the block appends the chunk's survivors to the live and
// collision banks in slot order (one atomic per block and queue per pass).
constexpr uint32_t REFILL_MIN = 16;
constexpr uint32_t ADV_CHUNK_MAX = 4096;  // rounds x blockDim
enum : uint8_t { OUT_NONE = 0, OUT_LIVE = 1, OUT_COL = 2 };

template <class R, bool REC, bool LDS>
__global__ void __launch_bounds__(1024) k_advance_r(Tables T0, uint32_t gen, uint32_t flights,
                                                    uint32_t rounds, Bank in,
                                                    const uint32_t* __restrict__ n_in_p,
                                                    Bank live, uint32_t* n_live, Bank col,
                                                    uint32_t* n_col, Accum A, Records Rc,
                                                    uint32_t* clr_live, uint32_t* clr_col) {
  const uint32_t n_in = *n_in_p;
  const uint32_t C = rounds * blockDim.x;
  const uint32_t base = blockIdx.x * C;
  const Tables T = kernel_tables<R, LDS>(T0, base < n_in);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *clr_live = 0;
    *clr_col = 0;
  }
  const uint32_t n_chunk = base < n_in ? min(C, n_in - base) : 0u;
  __shared__ uint32_t next;
  __shared__ uint8_t outcome[ADV_CHUNK_MAX];
  if (threadIdx.x == 0) next = blockDim.x;
  __syncthreads();

  uint32_t c_seg = 0, c_cross = 0, c_refl = 0, c_leak = 0, c_kill = 0, c_cen = 0, c_items = 0;
  uint32_t my = threadIdx.x;
  bool have = my < n_chunk;
  Part<R> p;
  Stream rs(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
  uint32_t fl = 0;
  if (have) {
    p = load_part<R>(in, base + my);
    rs = Stream(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    c_items += 1;
  }
  const uint32_t lane = lane_id();
  const unsigned long long lt = (1ull << lane) - 1ull;
  while (__ballot(have) != 0ull || next < n_chunk) {
    if (have) {
      int ev;
      bool refl = false;
      if ((int64_t)p.nseg >= T.max_events) {
        ev = EV_KILL;
      } else {
        ev = segment<R, REC, false>(T, T.geo, p, rs, A, Rc, &refl);
        p.nseg += 1;
        c_seg += 1;
        fl += 1;
        c_cross += (ev == EV_CROSS || ev == EV_LEAK) ? 1u : 0u;
        c_refl += refl ? 1u : 0u;
      }
      if (ev != EV_CROSS || fl >= flights) {
        // the particle is done for this launch
        p.ctr = rs.draw;
        uint8_t o = OUT_NONE;
        if (ev == EV_KILL) {
          die<R, REC>(p, FATE_KILLED, A, Rc);
          c_kill += 1;
        } else if (ev == EV_LEAK) {
          die<R, REC>(p, FATE_LEAKED, A, Rc);
          c_leak += 1;
        } else if (ev == EV_CENSUS) {
          die<R, REC>(p, FATE_CENSUS, A, Rc);
          c_cen += 1;
        } else {
          store_part(in, base + my, p);
          o = ev == EV_COLLIDE ? OUT_COL : OUT_LIVE;
        }
        outcome[my] = o;
        have = false;
      }
    }
    // refill the free lanes from the chunk, one LDS atomic per wave
    const unsigned long long free_mask = __ballot(!have);
    const uint32_t n_free = (uint32_t)__popcll(free_mask);
    if (n_free >= REFILL_MIN || n_free == 64u) {
      uint32_t first = 0;
      const int leader = __ffsll((long long)free_mask) - 1;
      if ((int)lane == leader) first = atomicAdd(&next, n_free);
      first = __shfl(first, leader);
      if (first >= n_chunk) {
        if (n_free == 64u) break;  // nothing left for this wave
      } else if (!have) {
        const uint32_t item = first + (uint32_t)__popcll(free_mask & lt);
        if (item < n_chunk) {
          my = item;
          have = true;
          fl = 0;
          p = load_part<R>(in, base + my);
          rs = Stream(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
          c_items += 1;
        }
      }
    }
  }
  __syncthreads();
  // survivors of the chunk, in slot order, to the live and collision banks
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  for (uint32_t r0 = 0; r0 < C; r0 += blockDim.x) {
    const uint32_t li = r0 + threadIdx.x;
    const uint8_t o = li < n_chunk ? outcome[li] : OUT_NONE;
    uint32_t pl, pc;
    block_append2(o == OUT_LIVE, o == OUT_COL, n_live, n_col, lds, &pl, &pc);
    if (o != OUT_NONE) {
      const Part<R> q = load_part<R>(in, base + li);
      if (o == OUT_LIVE)
        store_part(live, pl, q);
      else
        store_part(col, pc, q);
    }
  }
  wave_count(A.cnt + CNT_SEG * STRIPES, c_seg);
  wave_count(A.cnt + CNT_CROSS * STRIPES, c_cross);
  wave_count(A.cnt + CNT_REFL * STRIPES, c_refl);
  wave_count(A.cnt + CNT_LEAK * STRIPES, c_leak);
  wave_count(A.cnt + CNT_KILLED * STRIPES, c_kill);
  wave_count(A.cnt + CNT_CENSUS * STRIPES, c_cen);
  wave_count(A.cnt + CNT_ADV_ITEMS * STRIPES, c_items);
  wave_count(A.cnt + CNT_ADV_SEGS * STRIPES, c_seg);
}

// Process the collision bank: collision estimator, fission-bank append
// (block-aggregated reservation), scatter to the live bank or absorb.
template <class R, bool REC, bool LDS>
__global__ void __launch_bounds__(1024) k_collide(Tables T0, uint32_t gen, Bank in,
                                                  const uint32_t* __restrict__ n_in_p, Bank live,
                                                  uint32_t* n_live, Accum A, Records Rc) {
  const uint32_t n_in = *n_in_p;
  const Tables T = kernel_tables<R, LDS>(T0, blockIdx.x * blockDim.x < n_in);
  const double k_used = *A.k_used;
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  // The grid walks the bank (as many blocks as are resident on the large
  // launches): each thread keeps its counts and its exact k sums and adds
  // them once, so a wavefront's counter atomics and the round trip of its
  // 128-bit sums are paid once per launch, not once per 64 collisions.
  uint32_t c_col = 0, c_scat = 0, c_abs = 0, c_sites = 0;
  unsigned long long kc_lo = 0, kc_hi = 0, ka_lo = 0, ka_hi = 0;
  const uint32_t step = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n_in; base += step) {
    const uint32_t k = base + threadIdx.x;
    const bool valid = k < n_in;
    Part<R> p;
    ColXS<R> x{0, R(1), R(0)};
    uint32_t nf = 0;
    // a collision takes about five draws: both blocks that hold them are
    // evaluated up front by every lane at once, not at whichever draw each
    // lane crosses a block boundary
    LockStream rs(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
    if (valid) {
      p = load_part<R>(in, k);
      rs = LockStream(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
      rs.top_up();
      rs.fill_next();
      x = col_xs(T, T.geo, p);
      const double kc = (double)(x.nusf / x.st);
      const uint64_t q = quantize(kc, T.q_kcol);
      kc_lo += q & 0xFFFFFFFFull;
      kc_hi += q >> 32;
      if (REC) {
        Rc.n_col[p.id] += 1;
        Rc.kcol_sum[p.id] += kc;
      }
      nf = fission_count(T, x, rs, k_used);
    }
    const uint32_t slot = block_reserve(nf, A.n_fis, lds);
    bool alive = false;
    uint64_t q_kabs = 0;
    if (valid) {
      alive = collide_rest<R, REC>(T, p, rs, x, nf, slot, A, &q_kabs);
      p.ctr = rs.draw;
      if (!alive) die<R, REC>(p, FATE_ABSORBED, A, Rc);
    }
    ka_lo += q_kabs & 0xFFFFFFFFull;
    ka_hi += q_kabs >> 32;
    const uint32_t pl = block_reserve(alive ? 1u : 0u, n_live, lds);
    if (alive) store_part(live, pl, p);
    c_col += valid ? 1u : 0u;
    c_scat += alive ? 1u : 0u;
    c_abs += (valid && !alive) ? 1u : 0u;
    c_sites += nf;
  }
  wave_count(A.cnt + CNT_COL * STRIPES, c_col);
  wave_count(A.cnt + CNT_COL_ITEMS * STRIPES, c_col);
  wave_count(A.cnt + CNT_SCAT * STRIPES, c_scat);
  wave_count(A.cnt + CNT_ABS * STRIPES, c_abs);
  wave_count(A.cnt + CNT_SITES * STRIPES, c_sites);
  wave_acc_halves(A.k + K_COL * STRIPES * 2, kc_lo, kc_hi);
  wave_acc_halves(A.k + K_ABS * STRIPES * 2, ka_lo, ka_hi);
}

// History-based finish of the last live particles: one lane runs its
// particle's remaining flights and collisions to the end (the same
// operations as the event kernels, in the same order).  One wave per block.
template <class R, bool REC, bool LDS>
__global__ void __launch_bounds__(64) k_tail(Tables T0, uint32_t gen, Bank in,
                                              const uint32_t* __restrict__ n_in_p, Accum A,
                                              Records Rc) {
  const uint32_t n_in = *n_in_p;
  const Tables T = kernel_tables<R, LDS>(T0, blockIdx.x * blockDim.x < n_in);
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long c_seg = 0, c_col = 0, c_cross = 0, c_refl = 0, c_leak = 0, c_abs = 0,
                     c_kill = 0, c_sites = 0, c_scat = 0, c_cen = 0;
  unsigned long long kcol[2] = {0, 0}, kabs[2] = {0, 0};
  // One pass of the loop is one flight of every live lane of the wave, so
  // the fission sites of the collisions of a pass are reserved together (one
  // atomic per wave, at a point all lanes reach): per-lane atomics on the one
  // bank counter would serialise.
  const double k_used = *A.k_used;
  bool live = k < n_in;
  Part<R> p;
  // FP64: draws through the wavefront's draw cache once few histories remain
  constexpr bool CACHE = std::is_same<R, double>::value;
  using S = typename std::conditional<CACHE, CachedStream, Stream>::type;
  S rs = Stream(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
  int64_t nseg = 0;
  if (live) {
    p = load_part<R>(in, k);
    rs = Stream(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    nseg = p.nseg;
  }
  // live lanes when the cache was set up (their ranks are the cache slots)
  unsigned long long slots = 0ull;
  // Let the particle's loads complete here, so that the loop head does not
  // wait on the memory counter, which in every later pass would also wait
  // for the previous flight's tally atomics.
  __builtin_amdgcn_s_waitcnt(0);
  while (__ballot(live) != 0ull) {
    if constexpr (CACHE) {
      if (slots == 0ull) {
        const unsigned long long lm = __ballot(live);
        if (__popcll(lm) <= TC_SLOTS) slots = lm;
      }
      if (slots != 0ull) {
        const bool need = live && (int)rs.clen - (int)(rs.draw - rs.cbase) < TC_LOW;
        const unsigned long long nm = __ballot(need);
        if (nm != 0ull) {
          // lane t evaluates draw t % TC_WORDS of the window of slot t / TC_WORDS
          const uint32_t t = lane_id();
          const int sl = (int)(t / TC_WORDS);
          unsigned long long m = slots;
          for (int i = 0; i < sl && m != 0ull; ++i) m &= m - 1ull;
          const int owner = m != 0ull ? __ffsll((long long)m) - 1 : -1;
          const int src = owner >= 0 ? owner : 0;
          const uint32_t d0 = __shfl(rs.draw, src);
          const uint32_t hid = __shfl(p.id, src);
          if (owner >= 0 && ((nm >> owner) & 1ull)) {
            const uint32_t w = d0 + t % TC_WORDS;
            const u64x4 b = philox4x64_10(w >> 2, hid, gen, T.prob, T.seed, TAG_TRANSPORT);
            const uint32_t q = w & 3u;
            const uint64_t word = q == 0 ? b.v[0] : q == 1 ? b.v[1] : q == 2 ? b.v[2] : b.v[3];
            DrawEntry e;
            e.u = u01(word);
            e.ln = cr_log(e.u, T.lt);
            cr_cossin_2pi(e.u, T.sct, &e.c, &e.s);
            tc_cache[t] = e;
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (need) {
            const int my = __popcll(slots & ((1ull << t) - 1ull));
            rs.ebase = (uint32_t)(my * TC_WORDS);
            rs.cbase = rs.draw;
            rs.clen = TC_WORDS;
          }
        }
      }
    }
    bool col = false;
    ColXS<R> x{0, R(1), R(0)};
    uint32_t nf = 0;
    if (live) {
      if (nseg >= T.max_events) {
        p.ctr = rs.draw;
        die<R, REC>(p, FATE_KILLED, A, Rc);
        ++c_kill;
        live = false;
      } else {
        bool refl = false;
        const int ev = segment<R, REC, true, S>(T, T.geo, p, rs, A, Rc, &refl);
        ++nseg;
        ++c_seg;
        if (ev == EV_LEAK) {
          ++c_cross;
          ++c_leak;
          p.ctr = rs.draw;
          die<R, REC>(p, FATE_LEAKED, A, Rc);
          live = false;
        } else if (ev == EV_CENSUS) {
          ++c_cen;
          p.ctr = rs.draw;
          die<R, REC>(p, FATE_CENSUS, A, Rc);
          live = false;
        } else if (ev == EV_CROSS) {
          ++c_cross;
          c_refl += refl ? 1 : 0;
        } else {
          ++c_col;
          x = col_xs(T, T.geo, p);
          const double kc = (double)(x.nusf / x.st);
          const uint64_t q = quantize(kc, T.q_kcol);
          kcol[0] += q & 0xFFFFFFFFull;
          kcol[1] += q >> 32;
          if (REC) {
            Rc.n_col[p.id] += 1;
            Rc.kcol_sum[p.id] += kc;
          }
          nf = fission_count(T, x, rs, k_used);
          col = true;
        }
      }
    }
    const uint32_t slot = __ballot(nf != 0) ? wave_reserve(nf, A.n_fis) : 0u;
    if (col) {
      c_sites += nf;
      uint64_t qa = 0;
      if (collide_rest<R, REC>(T, p, rs, x, nf, slot, A, &qa)) {
        ++c_scat;
      } else {
        kabs[0] += qa & 0xFFFFFFFFull;
        kabs[1] += qa >> 32;
        ++c_abs;
        p.ctr = rs.draw;
        die<R, REC>(p, FATE_ABSORBED, A, Rc);
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
  wave_count(A.cnt + CNT_CENSUS * STRIPES, c_cen);
  wave_acc_halves(A.k + K_COL * STRIPES * 2, kcol[0], kcol[1]);
  wave_acc_halves(A.k + K_ABS * STRIPES * 2, kabs[0], kabs[1]);
}

// Monolithic event (the paper's GPU scheme, Sec. 2): one launch does
// exactly one segment of every particle of the to-be-processed bank, all of
// its operations in one kernel: cross-section lookup, distance to
// collision, distance to boundary, move, tally, then the collision
// (fission-bank append, scatter or absorption) or the surface crossing.
// Survivors go to the processed bank, which the next launch reads (history
// length truncation with criterion 1); nothing is sorted and no event class
// gets a kernel of its own, so a wave runs both branches whenever its
// particles differ.  Block 0 clears the count the next launch appends to.
template <class R, bool REC, bool LDS>
__global__ void __launch_bounds__(1024) k_mono(Tables T0, uint32_t gen, Bank in,
                                               const uint32_t* __restrict__ n_in_p, Bank out,
                                               uint32_t* n_out, Accum A, Records Rc,
                                               uint32_t* clr_out) {
  const uint32_t n_in = *n_in_p;
  const Tables T = kernel_tables<R, LDS>(T0, blockIdx.x * blockDim.x < n_in);
  if (blockIdx.x == 0 && threadIdx.x == 0) *clr_out = 0;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = k < n_in;
  const double k_used = *A.k_used;
  int ev = EV_NONE;
  bool refl = false;
  Part<R> p;
  ColXS<R> x{0, R(1), R(0)};
  uint32_t nf = 0;
  uint64_t q_kcol = 0;
  Stream rs(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
  if (valid) {
    p = load_part<R>(in, k);
    rs = Stream(T.seed, TAG_TRANSPORT, p.id, gen, T.prob, p.ctr);
    if ((int64_t)p.nseg >= T.max_events) {
      ev = EV_KILL;
    } else {
      ev = segment<R, REC, false>(T, T.geo, p, rs, A, Rc, &refl);
      p.nseg += 1;
      if (ev == EV_COLLIDE) {
        x = col_xs(T, T.geo, p);
        const double kc = (double)(x.nusf / x.st);
        q_kcol = quantize(kc, T.q_kcol);
        if (REC) {
          Rc.n_col[p.id] += 1;
          Rc.kcol_sum[p.id] += kc;
        }
        nf = fission_count(T, x, rs, k_used);
      }
    }
  }
  __shared__ uint32_t lds[2 * (MAX_WAVES + 1)];
  const uint32_t slot = block_reserve(nf, A.n_fis, lds);
  bool alive = ev == EV_CROSS;
  uint64_t q_kabs = 0;
  if (ev == EV_COLLIDE) alive = collide_rest<R, REC>(T, p, rs, x, nf, slot, A, &q_kabs);
  if (valid) {
    p.ctr = rs.draw;
    if (ev == EV_KILL) die<R, REC>(p, FATE_KILLED, A, Rc);
    if (ev == EV_LEAK) die<R, REC>(p, FATE_LEAKED, A, Rc);
    if (ev == EV_CENSUS) die<R, REC>(p, FATE_CENSUS, A, Rc);
    if (ev == EV_COLLIDE && !alive) die<R, REC>(p, FATE_ABSORBED, A, Rc);
  }
  const uint32_t po = block_reserve(alive ? 1u : 0u, n_out, lds);
  if (alive) store_part(out, po, p);
  const bool seg = valid && ev != EV_KILL;
  wave_flag(A.cnt + CNT_SEG * STRIPES, seg);
  wave_flag(A.cnt + CNT_CROSS * STRIPES, ev == EV_CROSS || ev == EV_LEAK);
  wave_flag(A.cnt + CNT_REFL * STRIPES, refl);
  wave_flag(A.cnt + CNT_LEAK * STRIPES, ev == EV_LEAK);
  wave_flag(A.cnt + CNT_KILLED * STRIPES, ev == EV_KILL);
  wave_flag(A.cnt + CNT_CENSUS * STRIPES, ev == EV_CENSUS);
  wave_flag(A.cnt + CNT_COL * STRIPES, ev == EV_COLLIDE);
  wave_flag(A.cnt + CNT_SCAT * STRIPES, ev == EV_COLLIDE && alive);
  wave_flag(A.cnt + CNT_ABS * STRIPES, ev == EV_COLLIDE && !alive);
  wave_count(A.cnt + CNT_SITES * STRIPES, nf);
  wave_flag(A.cnt + CNT_ADV_ITEMS * STRIPES, valid);
  wave_flag(A.cnt + CNT_ADV_SEGS * STRIPES, seg);
  wave_flag(A.cnt + CNT_COL_ITEMS * STRIPES, ev == EV_COLLIDE);
  wave_acc(A.k + K_COL * STRIPES * 2, q_kcol);
  wave_acc(A.k + K_ABS * STRIPES * 2, q_kabs);
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
  // The chunk passes through LDS, so that the global loads and stores are
  // coalesced; thread t scans entries [16 t, 16 t + 16) of it (rows padded to
  // an odd stride, so that the row reads do not share banks).
  constexpr int PAD = SCAN_PER_THREAD + 1;
  __shared__ uint32_t buf[SCAN_THREADS * PAD];
  __shared__ uint32_t lds[SCAN_THREADS / 64 + 1];
  const size_t base = (size_t)blockIdx.x * SCAN_CHUNK;
  for (int e = 0; e < SCAN_PER_THREAD; ++e) {
    const uint32_t j = (uint32_t)e * SCAN_THREADS + threadIdx.x;
    const size_t k = base + j;
    buf[(j / SCAN_PER_THREAD) * PAD + j % SCAN_PER_THREAD] = k < n ? in[k] : 0u;
  }
  __syncthreads();
  uint32_t* mine = buf + threadIdx.x * PAD;
  uint32_t s = 0;
  for (int e = 0; e < SCAN_PER_THREAD; ++e) s += mine[e];
  uint32_t total;
  uint32_t run = block_excl_scan(s, lds, &total) + chunk_off[blockIdx.x];
  for (int e = 0; e < SCAN_PER_THREAD; ++e) {
    const uint32_t v = mine[e];
    mine[e] = run;
    run += v;
  }
  __syncthreads();
  for (int e = 0; e < SCAN_PER_THREAD; ++e) {
    const uint32_t j = (uint32_t)e * SCAN_THREADS + threadIdx.x;
    const size_t k = base + j;
    if (k < n) out[k] = buf[(j / SCAN_PER_THREAD) * PAD + j % SCAN_PER_THREAD];
  }
}

// Canonical bank, entropy and combing, in two passes over the banked sites.
// Site seq of history parent has canonical position offset[parent] + seq, so
// the sites of histories [h0, h0 + PB_SIZE) fill the positions [offset[h0],
// offset[h0 + PB_SIZE]).  Pass 1 (k_bucket) files every site, in banking
// order, into that range of the staging array for its parent's bucket (the
// bucket bases are a table of 4 bytes per PB_SIZE histories, which stays in
// cache, where a lookup of each parent's own offset would miss for nearly
// every site: banking order is far from parent order).  Pass 2 (k_place) loads a bucket's offsets and sites
// into LDS, each site at its place, writes the canonical entries in order,
// bins them on the entropy mesh, and writes the source entries of the next
// generation that combing takes from those positions.  A bucket with more
// sites than the LDS holds writes each site and its combed entries directly.
constexpr uint32_t PB_SHIFT = 10;
constexpr uint32_t PB_SIZE = 1u << PB_SHIFT;  // histories per bucket
constexpr uint32_t PLACE_CAP = 1536;          // sites of a bucket placed in LDS

template <bool CE>
__global__ void __launch_bounds__(256) k_bucket(Sites fis, const uint32_t* n_fis_p,
                                                const uint32_t* offs, const uint32_t* total_p,
                                                uint32_t n_hist, uint32_t cap, uint32_t* bk_fill,
                                                Staging st, uint32_t* status) {
  const uint32_t n = min(*n_fis_p, cap);
  const uint32_t total = *total_p;  // the sum of the per-history site counts
  const uint32_t lane = lane_id();
  const unsigned long long below = (1ull << lane) - 1ull;
  const uint32_t stride = gridDim.x * blockDim.x;
  // the loop runs on the index of the wavefront's first lane, so every lane
  // takes the same trips and the ballots below see the whole wavefront
  for (uint32_t s0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); s0 < n; s0 += stride) {
    const uint32_t s = s0 + lane;
    bool ok = s < n;
    uint32_t par = 0, q = 0;
    if (ok) {
      par = fis.parent[s];
      q = fis.seq[s];
      if (par >= n_hist) {
        atomicOr(status, ST_SCAN);
        ok = false;
      }
    }
    const uint32_t bk = par >> PB_SHIFT;
    // group the lanes by bucket (the lowest lane of a group leads it) ...
    uint32_t lead = lane, rank = 0, size = 0;
    unsigned long long todo = __ballot(ok);
    while (todo != 0ull) {
      const int first = __ffsll((long long)todo) - 1;
      const uint32_t lb = __shfl(bk, first);
      const unsigned long long same = __ballot(ok && bk == lb) & todo;
      if ((same >> lane) & 1ull) {
        lead = (uint32_t)first;
        rank = (uint32_t)__popcll(same & below);
        size = (uint32_t)__popcll(same);
      }
      todo &= ~same;
    }
    // ... then every leader reserves its group's slots at once: one round
    // trip per wavefront, however many buckets its sites fall into
    uint32_t base = 0, room = 0;
    if (ok && lead == lane) {
      const uint32_t h1 = (bk + 1u) << PB_SHIFT;
      const uint32_t b0 = offs[bk << PB_SHIFT];
      const uint32_t b1 = h1 < n_hist ? offs[h1] : total;
      const uint32_t got = atomicAdd(&bk_fill[bk], size);
      base = b0 + got;
      room = b1 >= b0 && b1 - b0 > got ? b1 - b0 - got : 0u;
    }
    base = __shfl(base, (int)lead);
    room = __shfl(room, (int)lead);
    if (ok) {
      if (rank >= room) {  // more sites than the bucket's histories count
        atomicOr(status, ST_SCAN);
      } else if (base + rank >= cap) {  // only after an overflow, which the host reports
        atomicOr(status, ST_OVERFLOW);
      } else {
        const uint32_t idx = base + rank;
        const uint32_t key = (par & (PB_SIZE - 1u)) | (q << PB_SHIFT);
        if (CE)
          st.ce[idx] = StSiteCE{fis.x[s], fis.y[s], fis.e[s], key, 0};
        else
          st.mg[idx] = StSite{fis.x[s], fis.y[s], key, fis.g[s]};
      }
    }
  }
}

// Combing: source site i of the next generation is canonical entry
// floor((i + xi0) M / N), capped at M - 1 (non-decreasing in i).
__device__ __forceinline__ uint32_t comb_pick(uint32_t i, double xi0, uint32_t m, uint32_t n) {
  const double t = ((double)i + xi0) * (double)m / (double)n;
  uint64_t k = (uint64_t)floor(t);
  if (k > m - 1) k = m - 1;
  return (uint32_t)k;
}

// The smallest i in [0, n] whose pick is at least target (n if none): an
// estimate from the inverse, then exact steps with comb_pick itself, so the
// source indices of neighbouring buckets meet without gap or overlap.
__device__ uint32_t comb_first(uint32_t target, double xi0, uint32_t m, uint32_t n) {
  if (target == 0u) return 0u;
  const double est = ceil((double)target * (double)n / (double)m - xi0);
  uint32_t i = est <= 0.0 ? 0u : (est >= (double)n ? n : (uint32_t)est);
  while (i > 0u && comb_pick(i - 1u, xi0, m, n) >= target) --i;
  while (i < n && comb_pick(i, xi0, m, n) < target) ++i;
  return i;
}

constexpr int PLACE_HIST = 4096;  // entropy meshes up to this many bins are binned in LDS
                                  // (dynamic LDS of 4 B per bin)

template <bool CE>
__global__ void __launch_bounds__(256) k_place(Tables T, const uint32_t* n_fis_p,
                                               const uint32_t* total_p, uint32_t cap,
                                               uint32_t n_hist, uint32_t n, const double* xi0_p,
                                               const uint32_t* offs, const uint32_t* bk_fill,
                                               Staging st, double* cx, double* cy, int32_t* cg,
                                               double* ce, double* sx, double* sy, int32_t* sg,
                                               double* se, uint32_t* hist, uint32_t* status) {
  __shared__ double lx[PLACE_CAP], ly[PLACE_CAP];
  __shared__ double le[CE ? PLACE_CAP : 1];
  __shared__ int32_t lg[PLACE_CAP];
  __shared__ uint32_t lo[PB_SIZE + 1];  // the bucket's history offsets, from its first
  __shared__ uint32_t seen[PLACE_CAP / 32];
  __shared__ uint32_t range[2];
  extern __shared__ uint32_t h[];  // nb words when nb <= PLACE_HIST
  const uint32_t m = min(*n_fis_p, cap);  // sites combing draws from
  const uint32_t total = *total_p;
  const double xi0 = *xi0_p;
  const int nb = T.ent_nx * T.ent_ny;
  const bool in_lds = nb <= PLACE_HIST;
  if (in_lds)
    for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  const uint32_t n_pb = (uint32_t)(((uint64_t)n_hist + PB_SIZE - 1u) >> PB_SHIFT);
  for (uint32_t b = blockIdx.x; b < n_pb; b += gridDim.x) {
    const uint32_t h0 = b << PB_SHIFT;
    const uint32_t nh = min(PB_SIZE, n_hist - h0);
    // the bucket's offsets (and the end of its range) in one round trip
    for (uint32_t t = threadIdx.x; t <= nh; t += blockDim.x)
      lo[t] = h0 + t < n_hist ? offs[h0 + t] : total;
    if (threadIdx.x == 0) range[0] = bk_fill[b];
    __syncthreads();
    const uint32_t base = lo[0], end = lo[nh], filled = range[0];
    __syncthreads();  // every thread has read range[0] and lo[0]
    if (end < base || filled != end - base) {  // sites missing or left over
      if (threadIdx.x == 0) atomicOr(status, ST_SCAN);
      continue;
    }
    const uint32_t cnt = end - base;
    if (cnt == 0u) continue;
    if (end > m) {  // past the bank: only after an overflow, which the host reports
      if (threadIdx.x == 0) atomicOr(status, ST_OVERFLOW);
      continue;
    }
    const bool fits = cnt <= PLACE_CAP;
    for (uint32_t t = threadIdx.x; t <= nh; t += blockDim.x) lo[t] -= base;
    if (fits && threadIdx.x < 2) range[threadIdx.x] = comb_first(base + threadIdx.x * cnt, xi0, m, n);
    if (threadIdx.x < PLACE_CAP / 32) seen[threadIdx.x] = 0u;
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < cnt; t += blockDim.x) {
      const size_t e = (size_t)base + t;
      double x, y, en = 0.0;
      uint32_t key;
      int32_t g = 0;
      if (CE) {
        const StSiteCE r = st.ce[e];
        x = r.x;
        y = r.y;
        en = r.e;
        key = r.key;
      } else {
        const StSite r = st.mg[e];
        x = r.x;
        y = r.y;
        key = r.key;
        g = r.g;
      }
      const uint32_t pl = key & (PB_SIZE - 1u), q = key >> PB_SHIFT;
      if (pl >= nh || q >= lo[pl + 1] - lo[pl]) {  // seq not below its history's count
        atomicOr(status, ST_SITE_SEQ);
        continue;
      }
      const uint32_t p = lo[pl] + q;  // place within the bucket's positions
      if (p >= cnt) {  // offsets not increasing: an inconsistent scan
        atomicOr(status, ST_SCAN);
        continue;
      }
      int bx = (int)floor((x - T.geo.x0) / T.geo.width * (double)T.ent_nx);
      int by = (int)floor((y - T.geo.y0) / T.geo.height * (double)T.ent_ny);
      bx = bx < 0 ? 0 : (bx > T.ent_nx - 1 ? T.ent_nx - 1 : bx);
      by = by < 0 ? 0 : (by > T.ent_ny - 1 ? T.ent_ny - 1 : by);
      if (in_lds)
        atomicAdd(&h[by * T.ent_nx + bx], 1u);
      else
        atomicAdd(&hist[by * T.ent_nx + bx], 1u);
      if (fits) {
        if (atomicOr(&seen[p >> 5], 1u << (p & 31u)) & (1u << (p & 31u)))
          atomicOr(status, ST_SCAN);  // position claimed twice
        lx[p] = x;
        ly[p] = y;
        lg[p] = g;
        if (CE) le[p] = en;
      } else {
        // a bucket larger than the LDS: this site's canonical entry and the
        // source entries combed from it, written directly
        const uint32_t k = base + p;
        if (cx) {
          cx[k] = x;
          cy[k] = y;
          cg[k] = g;
          if (CE) ce[k] = en;
        }
        const uint32_t i1 = comb_first(k + 1u, xi0, m, n);
        for (uint32_t i = comb_first(k, xi0, m, n); i < i1; ++i) {
          sx[i] = x;
          sy[i] = y;
          sg[i] = g;
          if (CE) se[i] = en;
        }
      }
    }
    __syncthreads();
    if (fits) {
      if (cx)  // the canonical bank itself is kept only when asked for
        for (uint32_t t = threadIdx.x; t < cnt; t += blockDim.x) {
          cx[base + t] = lx[t];
          cy[base + t] = ly[t];
          cg[base + t] = lg[t];
          if (CE) ce[base + t] = le[t];
        }
      const uint32_t i1 = range[1];
      for (uint32_t i = range[0] + threadIdx.x; i < i1; i += blockDim.x) {
        const uint32_t k = comb_pick(i, xi0, m, n) - base;
        sx[i] = lx[k];
        sy[i] = ly[k];
        sg[i] = lg[k];
        if (CE) se[i] = le[k];
      }
    }
    __syncthreads();  // the next bucket reuses the LDS arrays and the range
  }
  if (in_lds)
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
      if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Exact wave-wide sums (one wave of 64 lanes, one stripe per lane).
__device__ __forceinline__ void wave_sum128(unsigned long long& w0, unsigned long long& w1) {
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o0 = __shfl_xor(w0, off), o1 = __shfl_xor(w1, off);
    const unsigned long long t = w0 + o0;
    w1 += o1 + (t < w0 ? 1ull : 0ull);
    w0 = t;
  }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Neumaier pair (s, c) plus (x, cx).
__device__ __forceinline__ void neu_add(double& s, double& c, double x, double cx) {
  const double t = s + x;
  c += cx + (fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s);
  s = t;
}

// Generation totals (one wave): k estimators from the exact accumulators
// (multigroup track length from the per-block production sums of
// k_gen_tallies, in block order), event counters, bank size, the k used by
// the next generation and the combing offset.
__global__ void __launch_bounds__(64) k_gen_totals(Tables T, uint32_t gen, uint32_t n, Accum A,
                                                   const double* tl_part, int n_part,
                                                   double* gen_k, unsigned long long* gen_cnt,
                                                   uint32_t* gen_m, double* k_used, double* xi0) {
  static_assert(STRIPES == 64, "one accumulator stripe per lane");
  const int lane = (int)threadIdx.x;
  const double inv_q[3] = {1.0 / T.q_kcol, T.ce ? 1.0 / T.q_ktl : 0.0, 1.0 / T.q_kabs};
  // every load first: the stores below could alias them, so loads left in
  // the loops would wait one memory round trip each
  unsigned long long kw[3][2], cw[N_CNT_ALL];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    kw[e][0] = A.k[((size_t)e * STRIPES + lane) * 2];
    kw[e][1] = A.k[((size_t)e * STRIPES + lane) * 2 + 1];
  }
#pragma unroll
  for (int c = 0; c < N_CNT_ALL; ++c) cw[c] = A.cnt[c * STRIPES + lane];
  double kv[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    wave_sum128(kw[e][0], kw[e][1]);
    kv[e] = u128_to_double(kw[e][0], kw[e][1]) * inv_q[e];
  }
#pragma unroll
  for (int c = 0; c < N_CNT_ALL; ++c) {
    const unsigned long long v = wave_sum_u64(cw[c]);
    if (lane == 0) gen_cnt[(size_t)gen * N_CNT_ALL + c] = v;
    if (lane == 0 && c == CNT_SEG && v >= (1ull << 32)) atomicOr(A.status, ST_TALLY);
  }
  // multigroup track-length estimator: lane-strided partials, then a
  // fixed-order butterfly
  double ts = 0.0, tc = 0.0;
  if (!T.ce) {
    for (int b = lane; b < n_part; b += 64) neu_add(ts, tc, tl_part[2 * b], tl_part[2 * b + 1]);
    for (int off = 32; off > 0; off >>= 1) {
      const double os = __shfl_xor(ts, off), oc = __shfl_xor(tc, off);
      if (lane & off) {
        double s2 = os, c2 = oc;
        neu_add(s2, c2, ts, tc);
        ts = s2;
        tc = c2;
      } else {
        neu_add(ts, tc, os, oc);
      }
    }
  }
  if (lane != 0) return;
  gen_k[3 * gen + 0] = kv[0] / (double)n;
  gen_k[3 * gen + 1] = T.ce ? kv[1] / (double)n : (ts + tc) / (double)n;
  gen_k[3 * gen + 2] = kv[2] / (double)n;
  gen_m[gen] = *A.n_fis;
  if (!T.fixed_source) *k_used = gen_k[3 * gen + 0];
  Stream rs(T.seed, TAG_RESAMPLE, 0, gen, T.prob, 0);
  *xi0 = rs.next();
}

// Generation tallies per source particle: flux from the exact sums and the
// production nu_sig_f(bin) * flux.  A block takes GT_BINS consecutive bins,
// lane l of every wave bin l, the waves splitting the stripes (coalesced
// reads of each stripe's row), then one wave finishes the exact sums; each
// block leaves the compensated sum of its production terms (a fixed-order
// tree) for the track-length k estimator.
constexpr int GT_BINS = 64;
constexpr int GT_WAVES = 8;

// Exact sum over the stripes st = w, w + GT_WAVES, ... of bin b: the
// 128-bit pairs of the event kernels and the (low-half, high-half) sums of
// the tail kernels; (0, 0) for b >= nb.
__device__ __forceinline__ void bin_sum_stripes(const unsigned long long* pairs,
                                                const unsigned long long* halves, int n_stripes,
                                                int nb, int b, int w, unsigned long long* o0,
                                                unsigned long long* o1) {
  const size_t stride = 2 * (size_t)nb;
  unsigned long long w0 = 0, w1 = 0;
  if (b < nb) {
    for (int st = w; st < n_stripes; st += GT_WAVES) {
      const unsigned long long* pr = pairs + (size_t)st * stride + 2 * (size_t)b;
      const unsigned long long* hv = halves + (size_t)st * stride + 2 * (size_t)b;
      unsigned long long t = w0 + pr[0];
      w1 += pr[1] + (t < w0 ? 1ull : 0ull);
      w0 = t;
      const unsigned long long a = hv[0], c = hv[1];  // a + c * 2^32
      t = w0 + a;
      w1 += t < w0 ? 1ull : 0ull;
      w0 = t;
      t = w0 + (c << 32);
      w1 += (t < w0 ? 1ull : 0ull) + (c >> 32);
      w0 = t;
    }
  }
  *o0 = w0;
  *o1 = w1;
}

__global__ void __launch_bounds__(64 * GT_WAVES) k_gen_tallies(Tables T, uint32_t gen, uint32_t n,
                                                                Accum A, double* gen_tal,
                                                                double* tl_part) {
  __shared__ unsigned long long s0[GT_WAVES][GT_BINS], s1[GT_WAVES][GT_BINS];
  const int nb = T.n_bins;
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
  const int b = (int)blockIdx.x * GT_BINS + lane;
  // the flux accumulators, and in the continuous-energy time-dependent
  // mode the density ones
  const bool dens = A.dens != nullptr;
  unsigned long long v[2][2];  // [flux, density][w0, w1]: w1 * 2^64 + w0
  for (int a = 0; a < (dens ? 2 : 1); ++a) {
    bin_sum_stripes(a ? A.dens : A.tally, a ? A.dens_t : A.tally_t, T.tally_stripes, nb, b, w,
                    &v[a][0], &v[a][1]);
    s0[w][lane] = v[a][0];
    s1[w][lane] = v[a][1];
    __syncthreads();
    if (w == 0)
      for (int k = 1; k < GT_WAVES; ++k) {
        const unsigned long long t = v[a][0] + s0[k][lane];
        v[a][1] += s1[k][lane] + (t < v[a][0] ? 1ull : 0ull);
        v[a][0] = t;
      }
    __syncthreads();
  }
  if (w != 0) return;
  double prod = 0.0;
  if (b < nb) {
    const double flux = u128_to_double(v[0][0], v[0][1]) / T.q_flux;
    const int per_cell = T.geo.mr1 * T.G * T.nt;
    const int cell = b / per_cell;
    const int r = (b / (T.G * T.nt)) % T.geo.mr1;
    const int g = (b / T.nt) % T.G;
    const int m = T.geo.mats[T.geo.pin_map[cell] * T.geo.mr1 + r];
    // continuous energy: nu_sig_f varies inside a bin, so there is no
    // production tally; the time-dependent mode reports the density there
    if (T.ce)
      prod = dens ? u128_to_double(v[1][0], v[1][1]) / T.q_dens : 0.0;
    else
      prod = T.nusf[m * T.G + g] * flux;
    gen_tal[(size_t)gen * 2 * nb + b] = flux / (double)n;
    gen_tal[(size_t)gen * 2 * nb + nb + b] = prod / (double)n;
  }
  // fixed-order butterfly over the wave's 64 production terms
  double ps = prod, pc = 0.0;
  for (int off = 32; off > 0; off >>= 1) {
    const double os = __shfl_xor(ps, off), oc = __shfl_xor(pc, off);
    if (lane & off) {
      double s2 = os, c2 = oc;
      neu_add(s2, c2, ps, pc);
      ps = s2;
      pc = c2;
    } else {
      neu_add(ps, pc, os, oc);
    }
  }
  if (lane == 0) {
    tl_part[2 * blockIdx.x] = ps;
    tl_part[2 * blockIdx.x + 1] = pc;
  }
}

int gen_tally_blocks(int n_bins) { return (n_bins + GT_BINS - 1) / GT_BINS; }

// H = -sum_b p_b log2 p_b: the terms in parallel, summed in a fixed-order
// tree.
__global__ void __launch_bounds__(256) k_entropy_final(Tables T, uint32_t gen,
                                                      const uint32_t* hist, const uint32_t* n_p,
                                                      double* gen_h) {
  __shared__ double red[256];
  const uint32_t m = *n_p;
  const int nb = T.ent_nx * T.ent_ny;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    if (m > 0 && hist[b] > 0) {
      const double p = (double)hist[b] / (double)m;
      acc += p * log2(p);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) gen_h[gen] = -red[0];
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

// The event kernels run on LDS copies of the tables when they fit.
static size_t mg_lds_bytes(int prec, const Tables& T) {
  const size_t b = lds_tables_bytes(T, prec == 0 ? sizeof(double) : sizeof(float));
  return b <= LDS_TABLES_MAX ? b : 0;
}

template <class R, bool REC>
static void advance_k(dim3 g, dim3 b, size_t lb, hipStream_t s, const Tables& T, uint32_t gen,
                      uint32_t flights, const Bank& in, const uint32_t* n_in, const Bank& live,
                      uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                      const Records& Rc, uint32_t* clr_live, uint32_t* clr_col) {
  if (lb)
    hipLaunchKernelGGL((k_advance<R, REC, true>), g, b, lb, s, T, gen, flights, in, n_in, live,
                       n_live, col, n_col, A, Rc, clr_live, clr_col);
  else
    hipLaunchKernelGGL((k_advance<R, REC, false>), g, b, 0, s, T, gen, flights, in, n_in, live,
                       n_live, col, n_col, A, Rc, clr_live, clr_col);
}

hipError_t launch_advance(int prec, bool rec, const Tables& T, uint32_t gen, uint32_t flights,
                          const Bank& in, const uint32_t* n_in, const Bank& live,
                          uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                          const Records& Rc, uint32_t* clr_live, uint32_t* clr_col,
                          uint32_t bound, int block, hipStream_t s) {
  const dim3 g(std::max(1u, nblk(bound, block))), b(block);
  const size_t lb = mg_lds_bytes(prec, T);
  if (prec == 0) {
    if (rec)
      advance_k<double, true>(g, b, lb, s, T, gen, flights, in, n_in, live, n_live, col, n_col, A,
                              Rc, clr_live, clr_col);
    else
      advance_k<double, false>(g, b, lb, s, T, gen, flights, in, n_in, live, n_live, col, n_col,
                               A, Rc, clr_live, clr_col);
  } else {
    if (rec)
      advance_k<float, true>(g, b, lb, s, T, gen, flights, in, n_in, live, n_live, col, n_col, A,
                             Rc, clr_live, clr_col);
    else
      advance_k<float, false>(g, b, lb, s, T, gen, flights, in, n_in, live, n_live, col, n_col,
                              A, Rc, clr_live, clr_col);
  }
  return hipGetLastError();
}

template <class R, bool REC>
static void advance_lt_k(dim3 g, dim3 b, size_t lb, hipStream_t s, const Tables& T, uint32_t gen,
                         uint32_t flights, const Bank& in, const uint32_t* n_in, const Bank& live,
                         uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                         const Records& Rc, uint32_t* clr_live, uint32_t* clr_col) {
  hipLaunchKernelGGL((k_advance_lt<R, REC>), g, b, lb, s, T, gen, flights, in, n_in, live, n_live,
                     col, n_col, A, Rc, clr_live, clr_col);
}

// Resident blocks per compute unit of the LDS-staged advance kernel for this
// block size and LDS size (registers and LDS), at least 1.
int advance_lt_blocks_per_cu(int prec, bool rec, int block, size_t lds) {
  int n = 0;
  hipError_t e;
  if (prec == 0)
    e = rec ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_advance_lt<double, true>, block, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_advance_lt<double, false>, block, lds);
  else
    e = rec ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_advance_lt<float, true>, block, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_advance_lt<float, false>, block, lds);
  return (e == hipSuccess && n > 0) ? n : 1;
}

size_t advance_lt_lds_bytes(int prec, const Tables& T) {
  const size_t tb = mg_lds_bytes(prec, T);
  if (tb == 0) return 0;
  return ((tb + 15) & ~(size_t)15) + 16 * (size_t)T.n_bins;
}

hipError_t launch_advance_lt(int prec, bool rec, const Tables& T0, uint32_t gen, uint32_t flights,
                             const Bank& in, const uint32_t* n_in, const Bank& live,
                             uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                             const Records& Rc, uint32_t* clr_live, uint32_t* clr_col,
                             uint32_t bound, int block, int max_grid, hipStream_t s) {
  const size_t tb = mg_lds_bytes(prec, T0);
  if (tb == 0 || T0.probs || T0.ce || block < 64 || block > 1024 || block % 64 || max_grid < 1)
    return hipErrorInvalidValue;
  Tables T = T0;
  T.lds_tally_off = (uint32_t)((tb + 15) & ~(size_t)15);
  T.lds_bin_lo = 0;
  T.lds_bin_n = (uint32_t)T.n_bins;
  const size_t lb = advance_lt_lds_bytes(prec, T0);
  const unsigned nb = std::max(1u, nblk(bound, (unsigned)block));
  const dim3 g(std::min(nb, (unsigned)max_grid)), b(block);
  if (prec == 0) {
    if (rec)
      advance_lt_k<double, true>(g, b, lb, s, T, gen, flights, in, n_in, live, n_live, col, n_col,
                                 A, Rc, clr_live, clr_col);
    else
      advance_lt_k<double, false>(g, b, lb, s, T, gen, flights, in, n_in, live, n_live, col,
                                  n_col, A, Rc, clr_live, clr_col);
  } else {
    if (rec)
      advance_lt_k<float, true>(g, b, lb, s, T, gen, flights, in, n_in, live, n_live, col, n_col,
                                A, Rc, clr_live, clr_col);
    else
      advance_lt_k<float, false>(g, b, lb, s, T, gen, flights, in, n_in, live, n_live, col,
                                 n_col, A, Rc, clr_live, clr_col);
  }
  return hipGetLastError();
}

template <class R, bool REC>
static void advance_r_k(dim3 g, dim3 b, size_t lb, hipStream_t s, const Tables& T, uint32_t gen,
                        uint32_t flights, uint32_t rounds, const Bank& in, const uint32_t* n_in,
                        const Bank& live, uint32_t* n_live, const Bank& col, uint32_t* n_col,
                        const Accum& A, const Records& Rc, uint32_t* clr_live,
                        uint32_t* clr_col) {
  if (lb)
    hipLaunchKernelGGL((k_advance_r<R, REC, true>), g, b, lb, s, T, gen, flights, rounds, in,
                       n_in, live, n_live, col, n_col, A, Rc, clr_live, clr_col);
  else
    hipLaunchKernelGGL((k_advance_r<R, REC, false>), g, b, 0, s, T, gen, flights, rounds, in,
                       n_in, live, n_live, col, n_col, A, Rc, clr_live, clr_col);
}

hipError_t launch_advance_refill(int prec, bool rec, const Tables& T, uint32_t gen,
                                 uint32_t flights, uint32_t rounds, const Bank& in,
                                 const uint32_t* n_in, const Bank& live, uint32_t* n_live,
                                 const Bank& col, uint32_t* n_col, const Accum& A,
                                 const Records& Rc, uint32_t* clr_live, uint32_t* clr_col,
                                 uint32_t bound, int block, hipStream_t s) {
  if (rounds < 1 || rounds * (uint32_t)block > ADV_CHUNK_MAX) return hipErrorInvalidValue;
  const dim3 g(std::max(1u, nblk(bound, (unsigned)block * rounds))), b(block);
  const size_t lb = mg_lds_bytes(prec, T);
  if (prec == 0) {
    if (rec)
      advance_r_k<double, true>(g, b, lb, s, T, gen, flights, rounds, in, n_in, live, n_live, col,
                                n_col, A, Rc, clr_live, clr_col);
    else
      advance_r_k<double, false>(g, b, lb, s, T, gen, flights, rounds, in, n_in, live, n_live,
                                 col, n_col, A, Rc, clr_live, clr_col);
  } else {
    if (rec)
      advance_r_k<float, true>(g, b, lb, s, T, gen, flights, rounds, in, n_in, live, n_live, col,
                               n_col, A, Rc, clr_live, clr_col);
    else
      advance_r_k<float, false>(g, b, lb, s, T, gen, flights, rounds, in, n_in, live, n_live,
                                col, n_col, A, Rc, clr_live, clr_col);
  }
  return hipGetLastError();
}

template <class R, bool REC>
static void collide_k(dim3 g, dim3 b, size_t lb, hipStream_t s, const Tables& T, uint32_t gen,
                      const Bank& in, const uint32_t* n_in, const Bank& live, uint32_t* n_live,
                      const Accum& A, const Records& Rc) {
  if (lb)
    hipLaunchKernelGGL((k_collide<R, REC, true>), g, b, lb, s, T, gen, in, n_in, live, n_live, A,
                       Rc);
  else
    hipLaunchKernelGGL((k_collide<R, REC, false>), g, b, 0, s, T, gen, in, n_in, live, n_live, A,
                       Rc);
}

int collide_blocks_per_cu(int prec, bool rec, const Tables& T, int block) {
  const size_t lb = mg_lds_bytes(prec, T);
  int n = 0;
  hipError_t e;
  if (prec == 0) {
    if (rec)
      e = lb ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_collide<double, true, true>, block, lb)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_collide<double, true, false>, block, 0);
    else
      e = lb ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_collide<double, false, true>, block, lb)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_collide<double, false, false>, block, 0);
  } else {
    if (rec)
      e = lb ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_collide<float, true, true>, block, lb)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_collide<float, true, false>, block, 0);
    else
      e = lb ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_collide<float, false, true>, block, lb)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_collide<float, false, false>, block, 0);
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_collide(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                          const uint32_t* n_in, const Bank& live, uint32_t* n_live,
                          const Accum& A, const Records& Rc, uint32_t bound, int block,
                          int max_grid, hipStream_t s) {
  uint32_t nb = std::max(1u, nblk(bound, block));
  if (max_grid > 0) nb = std::min<uint32_t>(nb, (uint32_t)max_grid);
  const dim3 g(nb), b(block);
  const size_t lb = mg_lds_bytes(prec, T);
  if (prec == 0) {
    if (rec)
      collide_k<double, true>(g, b, lb, s, T, gen, in, n_in, live, n_live, A, Rc);
    else
      collide_k<double, false>(g, b, lb, s, T, gen, in, n_in, live, n_live, A, Rc);
  } else {
    if (rec)
      collide_k<float, true>(g, b, lb, s, T, gen, in, n_in, live, n_live, A, Rc);
    else
      collide_k<float, false>(g, b, lb, s, T, gen, in, n_in, live, n_live, A, Rc);
  }
  return hipGetLastError();
}

template <class R, bool REC>
static void tail_k(dim3 g, dim3 b, size_t lb, hipStream_t s, const Tables& T, uint32_t gen,
                   const Bank& in, const uint32_t* n_in, const Accum& A, const Records& Rc) {
  if (lb)
    hipLaunchKernelGGL((k_tail<R, REC, true>), g, b, lb, s, T, gen, in, n_in, A, Rc);
  else
    hipLaunchKernelGGL((k_tail<R, REC, false>), g, b, 0, s, T, gen, in, n_in, A, Rc);
}

hipError_t launch_tail(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                       const uint32_t* n_in, const Accum& A, const Records& Rc, uint32_t bound,
                       hipStream_t s) {
  const dim3 g(std::max(1u, nblk(bound, 64))), b(64);
  const size_t lb = mg_lds_bytes(prec, T);
  if (prec == 0) {
    if (rec)
      tail_k<double, true>(g, b, lb, s, T, gen, in, n_in, A, Rc);
    else
      tail_k<double, false>(g, b, lb, s, T, gen, in, n_in, A, Rc);
  } else {
    if (rec)
      tail_k<float, true>(g, b, lb, s, T, gen, in, n_in, A, Rc);
    else
      tail_k<float, false>(g, b, lb, s, T, gen, in, n_in, A, Rc);
  }
  return hipGetLastError();
}

template <class R, bool REC>
static void mono_k(dim3 g, dim3 b, size_t lb, hipStream_t s, const Tables& T, uint32_t gen,
                   const Bank& in, const uint32_t* n_in, const Bank& out, uint32_t* n_out,
                   const Accum& A, const Records& Rc, uint32_t* clr_out) {
  if (lb)
    hipLaunchKernelGGL((k_mono<R, REC, true>), g, b, lb, s, T, gen, in, n_in, out, n_out, A, Rc,
                       clr_out);
  else
    hipLaunchKernelGGL((k_mono<R, REC, false>), g, b, 0, s, T, gen, in, n_in, out, n_out, A, Rc,
                       clr_out);
}

hipError_t launch_mono(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                       const uint32_t* n_in, const Bank& out, uint32_t* n_out, const Accum& A,
                       const Records& Rc, uint32_t* clr_out, uint32_t bound, int block,
                       hipStream_t s) {
  const dim3 g(std::max(1u, nblk(bound, block))), b(block);
  const size_t lb = mg_lds_bytes(prec, T);
  if (prec == 0) {
    if (rec)
      mono_k<double, true>(g, b, lb, s, T, gen, in, n_in, out, n_out, A, Rc, clr_out);
    else
      mono_k<double, false>(g, b, lb, s, T, gen, in, n_in, out, n_out, A, Rc, clr_out);
  } else {
    if (rec)
      mono_k<float, true>(g, b, lb, s, T, gen, in, n_in, out, n_out, A, Rc, clr_out);
    else
      mono_k<float, false>(g, b, lb, s, T, gen, in, n_in, out, n_out, A, Rc, clr_out);
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

hipError_t launch_gen_totals(const Tables& T, uint32_t gen, uint32_t n, const Accum& A,
                             const double* tl_part, double* gen_k, unsigned long long* gen_cnt,
                             uint32_t* gen_m, double* k_used, double* xi0, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_totals, dim3(1), dim3(64), 0, s, T, gen, n, A, tl_part,
                     gen_tally_blocks(T.n_bins), gen_k, gen_cnt, gen_m, k_used, xi0);
  return hipGetLastError();
}

hipError_t launch_gen_tallies(const Tables& T, uint32_t gen, uint32_t n, const Accum& A,
                              double* gen_tal, double* tl_part, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_tallies, dim3(std::max(1, gen_tally_blocks(T.n_bins))),
                     dim3(64 * GT_WAVES), 0, s, T, gen, n, A, gen_tal, tl_part);
  return hipGetLastError();
}

uint32_t bank_buckets(uint32_t n_hist) { return nblk(n_hist, (int)PB_SIZE); }

hipError_t launch_bank_end(const Tables& T, uint32_t gen, const Sites& fis, const uint32_t* n_fis,
                           const uint32_t* offs, const uint32_t* total, uint32_t n_hist,
                           uint32_t cap, uint32_t* bk_fill, const Staging& st, uint32_t n,
                           const double* xi0, double* cx, double* cy, int32_t* cg, double* ce,
                           double* sx, double* sy, int32_t* sg, double* se, uint32_t* hist,
                           double* gen_h, uint32_t* status, hipStream_t s) {
  // the staging records carved decide the form (cx/cy/cg/ce may be null)
  const bool is_ce = st.ce != nullptr;
  if (is_ce ? (st.mg != nullptr || !fis.e || !se) : (st.mg == nullptr || se != nullptr))
    return hipErrorInvalidValue;
  if (!bk_fill || !hist || !total || (cx && (!cy || !cg || (is_ce && !ce))))
    return hipErrorInvalidValue;
  const unsigned g1 = std::max(1u, std::min(nblk(cap, 256), 8192u));
  if (is_ce)
    hipLaunchKernelGGL((k_bucket<true>), dim3(g1), dim3(256), 0, s, fis, n_fis, offs, total,
                       n_hist, cap, bk_fill, st, status);
  else
    hipLaunchKernelGGL((k_bucket<false>), dim3(g1), dim3(256), 0, s, fis, n_fis, offs, total,
                       n_hist, cap, bk_fill, st, status);
  const unsigned g2 = std::max(1u, std::min(bank_buckets(n_hist), 1024u));
  const int nb = T.ent_nx * T.ent_ny;
  const size_t lh = nb <= PLACE_HIST ? sizeof(uint32_t) * (size_t)std::max(nb, 1) : 0;
  if (is_ce)
    hipLaunchKernelGGL((k_place<true>), dim3(g2), dim3(256), lh, s, T, n_fis, total, cap, n_hist,
                       n, xi0, offs, bk_fill, st, cx, cy, cg, ce, sx, sy, sg, se, hist, status);
  else
    hipLaunchKernelGGL((k_place<false>), dim3(g2), dim3(256), lh, s, T, n_fis, total, cap,
                       n_hist, n, xi0, offs, bk_fill, st, cx, cy, cg, ce, sx, sy, sg, se, hist,
                       status);
  hipLaunchKernelGGL(k_entropy_final, dim3(1), dim3(256), 0, s, T, gen, hist, n_fis, gen_h);
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
