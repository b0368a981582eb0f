// Dense range-scan observation update (placeholder until the MFMA path lands).
#include "scan.hpp"

namespace mcl {

size_t scan_work_bytes(int, int) { return 0; }
ScanWork scan_work_carve(void*, int, int) { return ScanWork(); }
ScanTable scan_table_carve(Carver&, const mcl_map_desc*, int, bool) { return ScanTable(); }
mcl_status scan_table_build(ScanTable&, const mcl_map_desc*, int, hipStream_t) { return MCL_OK; }

}  // namespace mcl

mcl_status scan_apply(mcl_filter, const float*, int32_t, double) { return MCL_ESTATE; }
mcl_status scan_sqdist(mcl_filter, const float*, int32_t, int32_t*) { return MCL_ESTATE; }
