// Circle-structured Sinkhorn (Algorithm 3).
#include "host.h"

namespace mot {
int circle_create(mot_plan_s *, const mot_fastsum_params *) { return MOT_EUNSUPPORTED; }
int circle_run_sweeps(mot_plan_s *, int) { return MOT_EUNSUPPORTED; }
int circle_marginals(mot_plan_s *, double *) { return MOT_EUNSUPPORTED; }
void circle_destroy(mot_plan_s *) {}
size_t circle_footprint(int, const int64_t *, int, int) { return 0; }
}  // namespace mot
