// wcc_timeline_2d.hip -- diagnostic build of the 2D half-step kernels with per-wave timestamps
// (linked into libwcc_timeline.so in place of wcc2d_kernels.hip; see wcc_timeline.hpp).
#include "wcc_timeline.hpp"

#define step_time(...) step_time_tl(__VA_ARGS__)
#define publish(...) publish_tl(__VA_ARGS__)
#include "wcc2d_kernels.hip"
#undef step_time
#undef publish

WCC_TIMELINE_ENTRY_POINTS(2d)
