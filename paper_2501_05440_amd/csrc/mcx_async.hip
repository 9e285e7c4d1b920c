// mcx_async.hip - asynchronous engine: persistent workgroups that pull work
// from global per-event-type queues, with no grid-wide barrier and no
// launch per event.
//
// The paper's runtime offers, besides the event-based schedule it measures,
// an asynchronous schedule in which resident threads keep choosing among
// pending work by event type (Sec. 2).  Here one launch runs every history
// of a generation (or of a batch of fixed-source problems): particle state
// lives in a global pool indexed by the history, and two global queues of
// history indices hold the particles waiting for a flight (advance) and for
// a collision.  Each workgroup loops: it takes up to one block of items from
// the fuller queue (or, when both run low, gives birth to the next block of
// histories), processes them one per lane with the same operations as the
// event kernels, and appends every survivor to the queue of its next event.
// The launch ends when every history has ended.  Results are identical to
// the other engines: the random streams are per history and every sum is
// exact.
//
// Queues are rings of capacity >= the history count (a history sits in at
// most one queue at a time).  A producer reserves positions with one atomic
// on the tail, writes its entries (waiting, if needed, until the consumer of
// the previous round has emptied the slot), then publishes the count; a
// consumer reserves published items from that count, claims positions with
// one atomic on the head, and waits for each entry to be written.  Every
// wait is bounded: past the bound the engine sets an abort flag that every
// workgroup reads, and the run reports an error instead of hanging.
//
// Cross-workgroup visibility (the L2 of each XCD is separate): everything
// that passes between workgroups during the launch (queue entries and
// counters, the particle pool and the per-history counters) is read and
// written with device-scope relaxed atomic loads and stores, which go to
// the device's coherence point.  A lane publishes the queue entry of a
// particle only after its own stores of that particle's state have
// completed (a wait on its memory counter), and a consumer reads the state
// at addresses that depend on the entry it read.  Device-scope release and
// acquire fences would write back and invalidate a whole L2 at every
// hand-over, which is what they cost on this chip.
#include "mcx_kernels_common.hpp"

namespace mcx {

constexpr uint32_t Q_EMPTY = 0xFFFFFFFFu;

struct AsyncQueue {
  uint32_t* slot;            // [mask + 1] history index or Q_EMPTY
  unsigned long long* tail;  // positions reserved by producers
  unsigned long long* head;  // positions claimed by consumers
  unsigned long long* avail; // published items not yet claimed (two's complement)
  uint32_t mask;
};

// Particle state between events, indexed by the global history index; the
// per-history counters and estimator sums live in the HistOut arrays.
struct AsyncPool {
  double* x;
  double* y;
  void* u;
  void* v;
  uint32_t* cell;
  uint32_t* gs;
  uint32_t* ctr;
  uint32_t* prob;
};

struct AsyncCtl {
  AsyncQueue q[2];                // 0: advance, 1: collide
  unsigned long long* born;       // histories given birth (or reserved for it)
  unsigned long long* remaining;  // histories not yet ended
  uint32_t* abort;                // set when a wait exceeds its bound
  uint64_t spin_limit;            // polls before a wait gives up
};

enum : uint32_t { AT_EXIT = 0, AT_IDLE = 1, AT_ADV = 2, AT_COL = 3, AT_BIRTH = 4 };

// An idle workgroup sleeps k x 127 x 64 cycles after its k-th idle poll in a
// row, k at most IDLE_SLEEP_MAX (about 50 us); it gives up after
// spin_limit / IDLE_SLEEP_MAX polls in a row (seconds).
constexpr uint32_t IDLE_SLEEP_MAX = 16;

__device__ __forceinline__ uint64_t ld_dev(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_dev32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// coherent (device-scope relaxed) load and store of shared state
template <class T>
__device__ __forceinline__ T ldc(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void stc(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reserve up to want published items of queue Q; returns the count.
__device__ __forceinline__ uint32_t q_reserve(const AsyncQueue& Q, uint32_t want) {
  const long long a = (long long)ld_dev(Q.avail);
  if (a <= 0) return 0;
  const long long w = a < (long long)want ? a : (long long)want;
  const long long old = (long long)atomicAdd(Q.avail, (unsigned long long)(-w));
  if (old >= w) return (uint32_t)w;
  const long long got = old > 0 ? old : 0;
  atomicAdd(Q.avail, (unsigned long long)(w - got));
  return (uint32_t)got;
}

template <class R>
__device__ __forceinline__ Part<R> pool_load(const AsyncPool& S, const HistOut& H, uint32_t h,
                                             uint32_t id) {
  Part<R> p;
  p.x = ldc(S.x + h);
  p.y = ldc(S.y + h);
  p.u = ldc(static_cast<const R*>(S.u) + h);
  p.v = ldc(static_cast<const R*>(S.v) + h);
  const uint32_t c = ldc(S.cell + h);
  p.i = cell_i(c);
  p.j = cell_j(c);
  p.r = cell_r(c);
  const uint32_t gs = ldc(S.gs + h);
  p.g = (int)(gs & 0xFFFFu);
  p.nsite = gs >> 16;
  p.ctr = ldc(S.ctr + h);
  p.id = id;
  p.nseg = ldc(H.cnt + (size_t)h * HO_N + HO_SEG);
  p.t = 0.0;
  return p;
}

template <class R>
__device__ __forceinline__ void pool_store(const AsyncPool& S, uint32_t h, const Part<R>& p) {
  stc(S.x + h, p.x);
  stc(S.y + h, p.y);
  stc(static_cast<R*>(S.u) + h, p.u);
  stc(static_cast<R*>(S.v) + h, p.v);
  stc(S.cell + h, (uint32_t)pack_cell(p.i, p.j, p.r));
  stc(S.gs + h, (uint32_t)p.g | (p.nsite << 16));
  stc(S.ctr + h, p.ctr);
}

__device__ __forceinline__ void async_death(const HistOut& H, const Accum& A, uint32_t h,
                                            uint32_t nsite, int fate, uint64_t q_kabs) {
  A.nsite_id[h] = nsite;
  stc(H.kabs + h, (unsigned long long)q_kabs);
  stc(H.cnt + (size_t)h * HO_N + HO_SITES, nsite);
  stc(H.cnt + (size_t)h * HO_N + HO_FATE, (uint32_t)fate);
}

// Append the lanes with `push` set to queue Q (every thread of the block
// calls it).  Each pushing lane must have stored its particle's state
// (coherent stores) before the call; its entry is written once those
// stores have completed.
template <int PB>
__device__ __forceinline__ void q_push(const AsyncQueue& Q, bool push, uint32_t h,
                                       uint32_t* lds, unsigned long long* lds_pos,
                                       const AsyncCtl& C) {
  uint32_t total;
  const uint32_t off = block_excl_scan(push ? 1u : 0u, lds, &total);
  if (total == 0) return;  // uniform across the block
  if (threadIdx.x == 0) *lds_pos = atomicAdd(Q.tail, (unsigned long long)total);
  __syncthreads();
  const unsigned long long pos = *lds_pos;
  if (push) {
    // this lane's stores of the particle's state have completed
    __builtin_amdgcn_s_waitcnt(0);
    uint32_t* s = Q.slot + (uint32_t)((pos + off) & Q.mask);
    // the previous round's entry of this slot has been claimed; wait until
    // its consumer has emptied it
    uint64_t n = 0;
    while (ld_dev32(s) != Q_EMPTY) {
      if (++n > C.spin_limit || ld_dev32(C.abort)) {
        st_dev32(C.abort, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    st_dev32(s, h);
  }
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(Q.avail, (unsigned long long)total);
}

// Read the history index at claimed position pos of Q (waits until written)
// and empty the slot.
__device__ __forceinline__ uint32_t q_take(const AsyncQueue& Q, unsigned long long pos,
                                           const AsyncCtl& C, bool* ok) {
  uint32_t* s = Q.slot + (uint32_t)(pos & Q.mask);
  uint32_t h;
  uint64_t n = 0;
  while ((h = ld_dev32(s)) == Q_EMPTY) {
    if (++n > C.spin_limit || ld_dev32(C.abort)) {
      st_dev32(C.abort, 1u);
      *ok = false;
      return 0;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  st_dev32(s, Q_EMPTY);
  *ok = true;
  return h;
}

template <class R, int PB, bool LDS>
__global__ void __launch_bounds__(PB) k_async(Tables T0, uint32_t gen, Accum A, HistOut H,
                                              AsyncPool S, AsyncCtl C, uint32_t flights,
                                              const double* sx, const double* sy,
                                              const int32_t* sg, const uint32_t* prev_status) {
  const Tables T = kernel_tables<R, LDS>(T0);
  const ProbDesc* P = T.probs;
  const uint64_t total = T.n_hist_total;
  const double k_used = *A.k_used;
  const Records Rc{};
  __shared__ uint32_t sh_kind, sh_n;
  __shared__ unsigned long long sh_pos;
  __shared__ uint32_t lds[MAX_WAVES + 2];
  __shared__ uint32_t sh_dead;
  __shared__ uint64_t sh_idle;

  // after a failed generation (or a source that could not be sampled before
  // this launch) the generation runs empty, as in the other engines
  if ((prev_status && *prev_status != 0u) || (sx && (*A.status & ST_SOURCE))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(A.status, ST_SKIPPED);
    return;
  }
  if (threadIdx.x == 0) sh_idle = 0;

  for (;;) {
    // ---------------- choose the next task ----------------
    if (threadIdx.x == 0) {
      uint32_t kind = AT_IDLE, n = 0;
      unsigned long long pos = 0;
      if (ld_dev32(C.abort)) {
        kind = AT_EXIT;
      } else {
        const long long a_adv = (long long)ld_dev(C.q[0].avail);
        const long long a_col = (long long)ld_dev(C.q[1].avail);
        const uint64_t b = ld_dev(C.born);
        // the fuller queue first, then the other one, then births; births
        // first while both queues hold less than a block of items
        int order[3] = {1, 0, -1};
        if (b < total && a_adv < PB && a_col < PB) {
          order[0] = -1;
          order[1] = 0;
          order[2] = 1;
        } else if (a_adv > a_col) {
          order[0] = 0;
          order[1] = 1;
        }
        for (int t = 0; t < 3 && kind == AT_IDLE; ++t) {
          const int qi = order[t];
          if (qi < 0) {
            if (b < total) {
              const unsigned long long h0 = atomicAdd(C.born, (unsigned long long)PB);
              if (h0 < total) {
                kind = AT_BIRTH;
                pos = h0;
                n = (uint32_t)min((uint64_t)PB, total - h0);
              }
            }
          } else {
            n = q_reserve(C.q[qi], PB);
            if (n) {
              kind = qi == 0 ? AT_ADV : AT_COL;
              pos = atomicAdd(C.q[qi].head, (unsigned long long)n);
            }
          }
        }
        if (kind == AT_IDLE) {
          if (ld_dev(C.remaining) == 0ull) {
            kind = AT_EXIT;
          } else if (++sh_idle > C.spin_limit / IDLE_SLEEP_MAX) {
            st_dev32(C.abort, 1u);
            kind = AT_EXIT;
          }
        } else {
          sh_idle = 0;
        }
      }
      sh_kind = kind;
      sh_n = n;
      sh_pos = pos;
      sh_dead = 0;
    }
    __syncthreads();
    const uint32_t kind = sh_kind, n = sh_n;
    const unsigned long long pos = sh_pos;
    __syncthreads();
    if (kind == AT_EXIT) break;
    if (kind == AT_IDLE) {
      // back off: every idle poll is a device-scope load that competes with
      // the working blocks' queue traffic
      const uint32_t naps = (uint32_t)min<uint64_t>(sh_idle, IDLE_SLEEP_MAX);
      for (uint32_t z = 0; z < naps; ++z) __builtin_amdgcn_s_sleep(127);
      continue;
    }
    const uint32_t t = threadIdx.x;
    const bool valid = t < n;
    bool to_adv = false, to_col = false;
    uint32_t h = 0;

    if (kind == AT_BIRTH) {
      // ---------------- birth ----------------
      if (valid) {
        h = (uint32_t)(pos + t);
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
        pool_store(S, h, p);
        stc(S.prob + h, (uint32_t)pi);
        uint32_t* cnt = H.cnt + (size_t)h * HO_N;
        for (int e = 0; e < HO_N; ++e) stc(cnt + e, 0u);
        stc(H.kcol + 2 * (size_t)h, 0ull);
        stc(H.kcol + 2 * (size_t)h + 1, 0ull);
        stc(H.kabs + h, 0ull);
        to_adv = true;
      }
    } else {
      // ---------------- take the items ----------------
      bool ok = true;
      if (valid) h = q_take(C.q[kind == AT_ADV ? 0 : 1], pos + t, C, &ok);
      const bool live = valid && ok;
      const int pi = live && P ? (int)ldc(S.prob + h) : 0;
      const uint64_t seed = P ? P[pi].seed : T.seed;
      const uint64_t prob = P ? P[pi].prob : T.prob;
      const uint32_t id = live ? (uint32_t)(h - (P ? P[pi].hist_base : 0ull)) : 0u;
      if (kind == AT_ADV) {
        // ---------------- advance ----------------
        if (live) {
          const Geo L = P ? P[pi].geo : T.geo;
          Part<R> p = pool_load<R>(S, H, h, id);
          uint32_t* cnt = H.cnt + (size_t)h * HO_N;
          uint32_t ncross = ldc(cnt + HO_CROSS), nrefl = ldc(cnt + HO_REFL);
          Stream rs(seed, TAG_TRANSPORT, id, gen, prob, p.ctr);
          int ev = EV_NONE;
          for (uint32_t f = 0; f < flights; ++f) {
            if ((int64_t)p.nseg >= T.max_events) {
              ev = EV_KILL;
              break;
            }
            bool refl = false;
            ev = segment<R, false, false>(T, L, p, rs, A, Rc, &refl);
            p.nseg += 1;
            ncross += (ev == EV_CROSS || ev == EV_LEAK) ? 1u : 0u;
            nrefl += refl ? 1u : 0u;
            if (ev != EV_CROSS) break;
          }
          p.ctr = rs.draw;
          stc(cnt + HO_SEG, p.nseg);
          stc(cnt + HO_CROSS, ncross);
          stc(cnt + HO_REFL, nrefl);
          if (ev == EV_KILL || ev == EV_LEAK || ev == EV_CENSUS) {
            async_death(H, A, h, p.nsite,
                        ev == EV_KILL ? FATE_KILLED : ev == EV_LEAK ? FATE_LEAKED : FATE_CENSUS, 0);
            atomicAdd(&sh_dead, 1u);
          } else {
            pool_store(S, h, p);
            to_adv = ev == EV_CROSS;
            to_col = ev == EV_COLLIDE;
          }
        }
      } else {
        // ---------------- collide ----------------
        Part<R> p;
        ColXS<R> x{0, R(1), R(0)};
        uint32_t nf = 0;
        Stream rs(T.seed, TAG_TRANSPORT, 0, gen, T.prob, 0);
        if (live) {
          const Geo L = P ? P[pi].geo : T.geo;
          p = pool_load<R>(S, H, h, id);
          rs = Stream(seed, TAG_TRANSPORT, id, gen, prob, p.ctr);
          x = col_xs(T, L, p);
          const uint64_t q = quantize((double)(x.nusf / x.st), T.q_kcol);
          unsigned long long* kc = H.kcol + 2 * (size_t)h;
          stc(kc, ldc(kc) + (q & 0xFFFFFFFFull));
          stc(kc + 1, ldc(kc + 1) + (q >> 32));
          uint32_t* cc = H.cnt + (size_t)h * HO_N + HO_COL;
          stc(cc, ldc(cc) + 1u);
          nf = fission_count(T, x, rs, k_used);
        }
        const uint32_t slot = block_reserve(nf, A.n_fis, lds);
        if (live) {
          uint64_t qa = 0;
          const bool alive = collide_rest<R, false>(T, p, rs, x, nf, slot, A, &qa);
          p.ctr = rs.draw;
          if (alive) {
            uint32_t* cs = H.cnt + (size_t)h * HO_N + HO_SCAT;
            stc(cs, ldc(cs) + 1u);
            pool_store(S, h, p);
            to_adv = true;
          } else {
            async_death(H, A, h, p.nsite, FATE_ABSORBED, qa);
            atomicAdd(&sh_dead, 1u);
          }
        }
      }
    }
    // hand the survivors over (q_push publishes an entry once the lane's
    // state stores have completed)
    q_push<PB>(C.q[0], to_adv, h, lds, &sh_pos, C);
    q_push<PB>(C.q[1], to_col, h, lds, &sh_pos, C);
    __syncthreads();
    if (threadIdx.x == 0 && sh_dead) atomicAdd(C.remaining, (unsigned long long)(-(long long)sh_dead));
  }
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------

template <class R, int PB>
static hipError_t launch_a(unsigned grid, size_t lb, const Tables& T, uint32_t gen,
                           const Accum& A, const HistOut& H, const AsyncPool& S,
                           const AsyncCtl& C, uint32_t flights, const double* sx,
                           const double* sy, const int32_t* sg, const uint32_t* prev_status,
                           hipStream_t s) {
  if (lb)
    hipLaunchKernelGGL((k_async<R, PB, true>), dim3(grid), dim3(PB), lb, s, T, gen, A, H, S, C,
                       flights, sx, sy, sg, prev_status);
  else
    hipLaunchKernelGGL((k_async<R, PB, false>), dim3(grid), dim3(PB), 0, s, T, gen, A, H, S, C,
                       flights, sx, sy, sg, prev_status);
  return hipGetLastError();
}

hipError_t launch_async(int prec, int grid, const Tables& T, uint32_t gen, const Accum& A,
                        unsigned long long* h_kcol, unsigned long long* h_kabs, uint32_t* h_cnt,
                        const AsyncBufs& B, uint32_t flights, uint64_t spin_limit,
                        const double* sx, const double* sy, const int32_t* sg,
                        const uint32_t* prev_status, hipStream_t s) {
  const HistOut H{h_kcol, h_kabs, h_cnt};
  AsyncPool S{B.x, B.y, B.u, B.v, B.cell, B.gs, B.ctr, B.prob};
  AsyncCtl C;
  for (int q = 0; q < 2; ++q) {
    C.q[q].slot = B.slot[q];
    C.q[q].tail = B.ctl + 3 * q + 0;
    C.q[q].head = B.ctl + 3 * q + 1;
    C.q[q].avail = B.ctl + 3 * q + 2;
    C.q[q].mask = B.mask;
  }
  C.born = B.ctl + 6;
  C.remaining = B.ctl + 7;
  C.abort = reinterpret_cast<uint32_t*>(B.ctl + 8);
  C.spin_limit = spin_limit;
  // the tables go to LDS when they fit (batches keep them in global memory)
  const size_t tb = lds_tables_bytes(T, prec == 0 ? sizeof(double) : sizeof(float));
  const size_t lb = (!T.probs && tb <= LDS_TABLES_MAX) ? tb : 0;
  const unsigned g = (unsigned)std::max(1, grid);
  if (prec == 0) return launch_a<double, 256>(g, lb, T, gen, A, H, S, C, flights, sx, sy, sg, prev_status, s);
  return launch_a<float, 256>(g, lb, T, gen, A, H, S, C, flights, sx, sy, sg, prev_status, s);
}

// Set the queues and counters up for a launch: every slot empty, counters
// zero, `remaining` = the history count.
__global__ void k_async_init(uint32_t* slot0, uint32_t* slot1, uint32_t n_slots,
                             unsigned long long* ctl, unsigned long long n_hist) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t i = k; i < n_slots; i += gridDim.x * blockDim.x) {
    slot0[i] = Q_EMPTY;
    slot1[i] = Q_EMPTY;
  }
  if (k < ASYNC_CTL_WORDS) ctl[k] = k == 7 ? n_hist : 0ull;
}

// The abort flag of the last launch as a status bit of the generation.
__global__ void k_async_status(const unsigned long long* ctl, uint32_t* status) {
  if (reinterpret_cast<const uint32_t*>(ctl + 8)[0]) atomicOr(status, ST_ASYNC);
}

hipError_t launch_async_status(const AsyncBufs& B, uint32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_async_status, dim3(1), dim3(1), 0, s, B.ctl, status);
  return hipGetLastError();
}

hipError_t launch_async_init(const AsyncBufs& B, uint64_t n_hist, hipStream_t s) {
  const uint32_t n = B.mask + 1;
  const unsigned g = (unsigned)std::min<uint32_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_async_init, dim3(std::max(1u, g)), dim3(256), 0, s, B.slot[0], B.slot[1],
                     n, B.ctl, (unsigned long long)n_hist);
  return hipGetLastError();
}

}  // namespace mcx
