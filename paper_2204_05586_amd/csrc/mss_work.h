// Work sets: the descriptor format shared by the batched path and the
// serving loop.  A work set is a list of sequences (simulations).  Each
// sequence may ask for
//   * integration of a range of its intervals [k_first, k_first + k_count)
//     (interval operators U_k written at their global index k, node times
//     from the global k, so a range gives exactly the operators the whole
//     simulation would), and/or
//   * the ordered product over all of its K_total operators (scan), writing
//     its states and final state.
// Descriptors carry absolute device pointers, so sequences may live in
// unrelated allocations (one block per served request).
#pragma once

#include <vector>

#include "mss_internal.h"
#include "mss_work_device.h"

namespace mss {

// Scan geometry of a sequence of K operators with tiles of `tile`
// (= 64 E) operators: levels above 0 and the scratch (bytes) of levels 1..top.
int scan_top(int64_t K, int tile = kScanTile);
size_t scan_scratch_bytes(int N, int64_t K, int tile = kScanTile);

// Host-side builder: fills item offsets and the scan tile tables, then
// packs everything for one upload.
struct WorkSet {
  int scan_e = kScanPerLane;  // operators per lane in the scan: 2, 4 or 8
  // chained runs (states formed in the integrator's launch): every sequence
  // is integrated whole (k_first = 0, k_count = K_total) and finalize()
  // builds the interleaved item order (IntegrateWorkArgs)
  bool chained = false;
  int64_t n_units = 0;                           // chained units (64 / S intervals each)
  std::vector<int32_t> order;                    // sequences by decreasing unit count
  std::vector<int64_t> group_item0, group_round0;
  std::vector<int32_t> group_count;
  std::vector<SimDesc> sims;
  std::vector<mss_term> terms;
  int64_t n_items = 0;
  int n_levels = 0;                                  // max top over scanning sequences
  std::vector<std::vector<int64_t>> reduce_tiles;    // [level][n + 1] prefix (levels 0..n_levels-1)
  std::vector<std::vector<int64_t>> apply_tiles;     // [level][n + 1] prefix (levels 0..n_levels)

  // Append a sequence; terms are copied unless identical to the previous
  // sequence's list.  Pointers may be filled later (patch_pointers).
  void add(const mss_problem& p, int slices_log2, int64_t k_first, int64_t k_count, bool scan);
  // Compute item offsets and tile tables (call after the last add).
  void finalize();
  // Bytes of the packed descriptor image and the image itself.
  size_t packed_bytes() const;
  void pack(char* dst, size_t* o_sims, size_t* o_terms, std::vector<size_t>* o_reduce,
            std::vector<size_t>* o_apply, size_t* o_chain = nullptr) const;

 private:
  const mss_term* last_terms_ = nullptr;
  int last_n_terms_ = -1, last_term_off_ = -1;
};

// Device view of an uploaded work set.
struct DevWork {
  const SimDesc* sims = nullptr;
  const mss_term* terms = nullptr;
  std::vector<const int64_t*> reduce_tiles, apply_tiles;
  std::vector<int64_t> reduce_total, apply_total;
  int32_t n_sims = 0;
  int64_t n_items = 0;
  int n_levels = 0;
  int scan_e = kScanPerLane;
  // chained runs
  int64_t n_units = 0;
  int32_t n_groups = 0;
  const int64_t* group_item0 = nullptr;
  const int64_t* group_round0 = nullptr;
  const int32_t* group_count = nullptr;
  const int32_t* order = nullptr;
};

DevWork device_view(const WorkSet& w, const char* dev_base, size_t o_sims, size_t o_terms,
                    const std::vector<size_t>& o_reduce, const std::vector<size_t>& o_apply,
                    size_t o_chain = 0);

// Enqueue the integrator (counter cleared by a kernel first, unless the
// caller's stream has already zeroed it: counter_zeroed) over every range of
// the work set; grid_blocks 256-thread workgroups.  user_fn: the work
// integrator of a user sampler's module (field from the sampler,
// descriptors carry no terms), or null for the field-program kernel.
hipError_t launch_work_integrate(const DevWork& w, unsigned long long* counter, int grid_blocks,
                                 hipStream_t st, hipFunction_t user_fn = nullptr,
                                 bool counter_zeroed = false);
// Enqueue the scan of every scanning sequence (reduce up, apply down).
hipError_t launch_work_scan(const DevWork& w, hipStream_t st);

// Enqueue a chained run of a chained work set: a reset kernel (unit counter,
// failure word and every slot word to 0) and the persistent integrator that
// also forms the states.  ws starts with a ChainSync block followed by one
// ChainSlot per sequence (chain_workspace_bytes).  user_fn: the chained
// work integrator of a user sampler's module, or null for the field-program
// kernel.  wait_ticks: bound of one wait (100 MHz real-time counter).
size_t chain_workspace_bytes(int32_t n_sims);
hipError_t launch_work_chained(const DevWork& w, void* ws, int grid_blocks, hipStream_t st,
                               hipFunction_t user_fn = nullptr,
                               unsigned long long wait_ticks = kChainWaitTicks);

}  // namespace mss
