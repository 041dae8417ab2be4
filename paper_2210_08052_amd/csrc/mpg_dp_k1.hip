// DP kernel instantiations with 1 protein column(s) per lane.
#include "mpg_dp.h"

namespace mpg {

hipError_t launch_dp_k1(hipStream_t s, int W, bool tb, const DevParams& P, const PairJob* jobs,
                        const int32_t* order, int count, const uint8_t* prot, const uint8_t* desc,
                        int2* bnd, uint8_t* tbbuf, mpg_dev_result* out) {
    return dev::launch_dp_k<1>(s, W, tb, P, jobs, order, count, prot, desc, bnd, tbbuf, out);
}

}  // namespace mpg
