// Tiled Q1 cell loops (fast path); see launch_cell_q1_* below.
#include "common.h"

namespace pff {

pf_status launch_cell_q1_d(const Geom&, const CellParams&, int, const double*, const double*, const double*,
                           const uint8_t*, double*, hipStream_t, bool* handled) {
  *handled = false;
  return PF_OK;
}
pf_status launch_cell_q1_f(const Geom&, const CellParams&, int, const float*, const float*, const float*,
                           const uint8_t*, float*, hipStream_t, bool* handled) {
  *handled = false;
  return PF_OK;
}

}  // namespace pff
