// Batched Lanczos over many independent effective Hamiltonians.
#include <vector>

#include "../../include/mrdmrg.h"
#include "internal.hpp"

struct dm_batch {
  std::vector<dm_heff_plan*> plans;
};

extern "C" int dm_batch_create(int32_t n, dm_heff_plan* const* plans, dm_stream stream,
                               dm_batch** out) {
  (void)stream;
  if (!out || n <= 0 || !plans) {
    mrd::set_last_error("dm_batch_create: bad arguments");
    return DM_ERR_ARG;
  }
  auto* b = new dm_batch;
  b->plans.assign(plans, plans + n);
  for (auto* p : b->plans)
    if (!p) {
      delete b;
      mrd::set_last_error("dm_batch_create: null plan");
      return DM_ERR_ARG;
    }
  *out = b;
  return DM_OK;
}

extern "C" void dm_batch_destroy(dm_batch* b) { delete b; }

extern "C" int lanczos_ground_batched(dm_batch* b, void* const* thetas, int32_t max_iter,
                                      double tol, double* energies, int32_t* iters,
                                      double* done_us, dm_stream stream) {
  if (!b || !thetas || !energies || !iters) {
    mrd::set_last_error("lanczos_ground_batched: null argument");
    return DM_ERR_ARG;
  }
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const int rc = lanczos_ground(b->plans[i], thetas[i], max_iter, tol, &energies[i], &iters[i], stream);
    if (rc != DM_OK) return rc;
    if (done_us) done_us[i] = 0.0;
  }
  return DM_OK;
}
