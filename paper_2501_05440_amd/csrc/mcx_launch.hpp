// mcx_launch.hpp - host-side launchers of the transport kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "mcx_device.hpp"

namespace mcx {

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s);
hipError_t launch_source(const Tables& T, uint32_t gen, uint32_t n, double* sx, double* sy,
                         int32_t* sg, uint32_t* status, hipStream_t s);
// prec: 0 = FP64, 1 = FP32-mixed
hipError_t launch_birth(int prec, const Tables& T, uint32_t gen, uint32_t n, const double* sx,
                        const double* sy, const int32_t* sg, const Bank& out, uint32_t* cnt_live,
                        uint32_t* cnt_col, const uint32_t* prev_status, uint32_t* status,
                        hipStream_t s);
hipError_t launch_gen_check(const Tables& T, const uint32_t* n_fis, const uint32_t* scan_total,
                            uint32_t* status, hipStream_t s);
hipError_t launch_advance(int prec, bool rec, const Tables& T, uint32_t gen, uint32_t flights,
                          const Bank& in, const uint32_t* n_in, const Bank& live,
                          uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                          const Records& Rc, uint32_t* clr_live, uint32_t* clr_col,
                          uint32_t bound, int block, hipStream_t s);
// advance with the flux tally staged in LDS: blocks of `block` threads walk
// the bank grid-stride (at most max_grid blocks) and add each bin to device
// memory once; results identical to launch_advance.  Multigroup, tables in
// LDS; advance_lt_lds_bytes gives its dynamic LDS per block (0: tables do
// not fit)
size_t advance_lt_lds_bytes(int prec, const Tables& T);
int advance_lt_blocks_per_cu(int prec, bool rec, int block, size_t lds);
hipError_t launch_advance_lt(int prec, bool rec, const Tables& T, uint32_t gen, uint32_t flights,
                             const Bank& in, const uint32_t* n_in, const Bank& live,
                             uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                             const Records& Rc, uint32_t* clr_live, uint32_t* clr_col,
                             uint32_t bound, int block, int max_grid, hipStream_t s);
// advance with lanes refilled from a chunk of rounds x block items per
// block (rounds x block <= 4096); results identical to launch_advance
hipError_t launch_advance_refill(int prec, bool rec, const Tables& T, uint32_t gen,
                                 uint32_t flights, uint32_t rounds, const Bank& in,
                                 const uint32_t* n_in, const Bank& live, uint32_t* n_live,
                                 const Bank& col, uint32_t* n_col, const Accum& A,
                                 const Records& Rc, uint32_t* clr_live, uint32_t* clr_col,
                                 uint32_t bound, int block, hipStream_t s);
// max_grid > 0: at most that many blocks, which walk the bank grid-stride
int collide_blocks_per_cu(int prec, bool rec, const Tables& T, int block);
hipError_t launch_collide(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                          const uint32_t* n_in, const Bank& live, uint32_t* n_live,
                          const Accum& A, const Records& Rc, uint32_t bound, int block,
                          int max_grid, hipStream_t s);
hipError_t launch_tail(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in, const uint32_t* n_in, const Accum& A, const Records& Rc,
                       uint32_t bound, hipStream_t s);
// monolithic event: one segment of every particle per launch, collision or
// crossing in the same kernel (in -> out, the count of out cleared at clr_out
// for the launch after)
hipError_t launch_mono(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                       const uint32_t* n_in, const Bank& out, uint32_t* n_out, const Accum& A,
                       const Records& Rc, uint32_t* clr_out, uint32_t bound, int block,
                       hipStream_t s);
uint32_t scan_chunks(uint32_t n);
hipError_t launch_scan(const uint32_t* in, uint32_t n, uint32_t* chunk_sum, uint32_t* out,
                       uint32_t* total, hipStream_t s);
// k_gen_tallies leaves one (sum, compensation) pair per block in tl_part
// (gen_tally_blocks(n_bins) pairs); k_gen_totals, launched after it, sums
// them into the track-length estimator.
int gen_tally_blocks(int n_bins);
hipError_t launch_gen_tallies(const Tables& T, uint32_t gen, uint32_t n, const Accum& A,
                              double* gen_tal, double* tl_part, hipStream_t s);
hipError_t launch_gen_totals(const Tables& T, uint32_t gen, uint32_t n, const Accum& A,
                             const double* tl_part, double* gen_k, unsigned long long* gen_cnt,
                             uint32_t* gen_m, double* k_used, double* xi0, hipStream_t s);
// Generation end of a k-eigenvalue run, after the scan of the per-history
// site counts (offs, their sum at total) and k_gen_totals (xi0): the
// canonical bank in cx/cy/cg/ce (not written when cx is null), the entropy of
// generation gen, and the combed source of the next one in sx/sy/sg/se.
// bk_fill holds bank_buckets(n_hist) zeroed counters and the staging array
// cap records.
uint32_t bank_buckets(uint32_t n_hist);
hipError_t launch_bank_end(const Tables& T, uint32_t gen, const Sites& fis, const uint32_t* n_fis,
                           const uint32_t* offs, const uint32_t* total, uint32_t n_hist,
                           uint32_t cap, uint32_t* bk_fill, const Staging& st, uint32_t n,
                           const double* xi0, double* cx, double* cy, int32_t* cg, double* ce,
                           double* sx, double* sy, int32_t* sg, double* se, uint32_t* hist,
                           double* gen_h, uint32_t* status, hipStream_t s);
hipError_t launch_stats(int n_bins2, int n_gen, int n_inactive, const double* gen_tal,
                        double* tal_mean, double* tal_sigma, const double* gen_k, double* k_stat,
                        hipStream_t s);
// Persistent engine configuration: threads per workgroup, LDS particle
// slots per workgroup, workgroups, and the refill threshold as a fraction of
// the slots (refill when fewer slots than that are live).
struct PersistentCfg {
  int block = 256;
  int slots = 512;
  int grid = 512;
  double tau = 0.75;
  int sort = 0;  // 1: collisions in fissile material first in the collide list
};
bool persistent_config_valid(int block, int slots);
size_t persistent_lds_bytes(int prec, int block, int slots);
hipError_t launch_persistent(int prec, const PersistentCfg& cfg, const Tables& T, uint32_t gen,
                             const Accum& A, unsigned long long* h_kcol,
                             unsigned long long* h_kabs, uint32_t* h_cnt, uint32_t* work,
                             const double* sx, const double* sy, const int32_t* sg,
                             const uint32_t* prev_status, hipStream_t s);
// Asynchronous engine: global particle pool and two global queues (advance,
// collide) of history indices; ctl holds ASYNC_CTL_WORDS words: per queue
// tail, head, published count, then births, remaining histories, abort flag.
constexpr int ASYNC_CTL_WORDS = 9;
struct AsyncBufs {
  double* x = nullptr;
  double* y = nullptr;
  void* u = nullptr;
  void* v = nullptr;
  uint32_t* cell = nullptr;
  uint32_t* gs = nullptr;
  uint32_t* ctr = nullptr;
  uint32_t* prob = nullptr;
  uint32_t* slot[2] = {nullptr, nullptr};
  unsigned long long* ctl = nullptr;
  uint32_t mask = 0;  // queue capacity - 1 (a power of two >= the history count)
};
hipError_t launch_async_init(const AsyncBufs& B, uint64_t n_hist, hipStream_t s);
hipError_t launch_async_status(const AsyncBufs& B, uint32_t* status, hipStream_t s);
hipError_t launch_async(int prec, int grid, const Tables& T, uint32_t gen, const Accum& A,
                        unsigned long long* h_kcol, unsigned long long* h_kabs, uint32_t* h_cnt,
                        const AsyncBufs& B, uint32_t flights, uint64_t spin_limit,
                        const double* sx, const double* sy, const int32_t* sg,
                        const uint32_t* prev_status, hipStream_t s);
hipError_t launch_hist_reduce(const Tables& T, int n_probs, unsigned long long* h_kcol,
                              unsigned long long* h_kabs, uint32_t* h_cnt, const Accum& A,
                              unsigned long long* prob_cnt, unsigned long long* prob_k,
                              hipStream_t s);
hipError_t launch_batch_results(const Tables& T, int n_probs, const Accum& A,
                                const unsigned long long* prob_k, double* flux, double* prod,
                                double* k_out, hipStream_t s);
// continuous energy (event engine; prec 0 = FP64, 1 = FP32-mixed)
hipError_t launch_ce_source(int prec, const Tables& T, uint32_t gen, uint32_t n, double* sx, double* sy,
                            double* se, uint32_t* status, hipStream_t s);
hipError_t launch_ce_birth(int prec, const Tables& T, uint32_t gen, uint32_t n, const double* sx,
                           const double* sy, const double* se, const Bank& out,
                           uint32_t* cnt_live, uint32_t* cnt_col, const uint32_t* prev_status,
                           uint32_t* status, hipStream_t s);
hipError_t launch_ce_advance(int prec, bool rec, const Tables& T, uint32_t gen, uint32_t flights,
                             const Bank& in, const uint32_t* n_in, const Bank& live,
                             uint32_t* n_live, const Bank& col, uint32_t* n_col, const Accum& A,
                             const Records& Rc, uint32_t* clr_live, uint32_t* clr_col,
                             uint32_t bound, int block, hipStream_t s);
hipError_t launch_ce_collide(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                             const uint32_t* n_in, const Bank& live, uint32_t* n_live,
                             const Accum& A, const Records& Rc, uint32_t bound, int block,
                             hipStream_t s);
hipError_t launch_ce_tail(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                          const uint32_t* n_in, const Accum& A, const Records& Rc, uint32_t bound,
                          hipStream_t s);
hipError_t launch_ce_mono(int prec, bool rec, const Tables& T, uint32_t gen, const Bank& in,
                          const uint32_t* n_in, const Bank& out, uint32_t* n_out, const Accum& A,
                          const Records& Rc, uint32_t* clr_out, uint32_t bound, int block,
                          hipStream_t s);
hipError_t launch_diag_math(int which, const double* in, double* out, int64_t n, hipStream_t s);
hipError_t launch_diag_philox(const uint64_t* in, uint64_t* out, int64_t n, hipStream_t s);
void host_math(int which, const double* in, double* out, int64_t n);

}  // namespace mcx
