// Host build of the device two-body flow (CC_KEPLER), for checking it on the CPU.
#include <math.h>
#define CC_KEPLER_FN static inline
#include "../paper_1407_7105_amd/csrc/cc_kepler.h"

// rv[6] = (r, v) advanced by t under mu; returns 1 on success.
extern "C" int kepler_flow_host(double mu, double *rv, double t)
{
    return cck::kepler_flow(mu, rv[0], rv[1], rv[2], rv[3], rv[4], rv[5], t) ? 1 : 0;
}
