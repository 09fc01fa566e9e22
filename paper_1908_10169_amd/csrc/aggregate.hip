// Progressive aggregation (Sec. 3.5) of consecutive blocks after the sweep.
#include "internal.h"

namespace bilu {

bilu_status aggregate_device(bilu_handle* h) {
  return fail(h, BILU_ERR_INVALID, "progressive aggregation is not built yet; set use_aggregation = 0");
}

}  // namespace bilu
