// Weighted graphs (positive integer arc lengths): placeholder until the
// weighted engine lands.
#include "bcd_host_internal.h"

namespace bcd {

bcd_status run_weighted(Graph *, Workspace *, const std::vector<int32_t> &, const std::vector<int32_t> &, bool,
                        SourceRun &) {
  return fail(BCD_ERR_UNSUPPORTED, "weighted graphs are not supported yet");
}

bcd_status multi_source_pass_weighted(Graph *, const int32_t *, int64_t, uint64_t *, uint64_t *, double *) {
  return fail(BCD_ERR_UNSUPPORTED, "weighted graphs are not supported yet");
}

}  // namespace bcd
