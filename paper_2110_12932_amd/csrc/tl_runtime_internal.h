// Internal interface between the serving loop (tl_server.cpp) and the solver
// runtime (tl_runtime.cpp).  Not part of the public interface.
#pragma once
#include <stddef.h>

#include <string>
#include <vector>

#include "../../include/tl.h"

namespace tl {

// Device and pinned tables for batched solves over up to max_slots
// simulations (solve items and per-item scalars).
struct BatchTables {
  void* impl = nullptr;
};
size_t batch_tables_bytes(int max_slots);
tl_status batch_tables_init(BatchTables* bt, void* dev_area, int max_slots,
                            void* hip_stream);
void batch_tables_free(BatchTables* bt);

// One macro step of every listed simulation in lockstep with batched
// solves.  errs[q] is empty on success, else the failure message of
// simulation q (whose state is then undefined).  Returns TL_EDEVICE on a
// HIP runtime error.
tl_status step_many(const std::vector<tl_sim*>& sims, BatchTables* bt,
                    std::vector<std::string>& errs);

// Sampled event timing of the batched fine CG kernel of a server.
tl_status batch_set_profiling(BatchTables* bt, int sample_every);
void batch_get_profile(BatchTables* bt, int64_t* launches, double* ms,
                       double* bytes);

tl_status validate_request(const tl_mesh* mesh, const tl_material* material,
                           const tl_scan_path* scan, const tl_options* opts);
void set_last_error(const std::string& msg);
size_t tl_sim_nodes(tl_sim* s, int level);

}  // namespace tl
