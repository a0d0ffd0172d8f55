// FFT pass kernels instantiated for float.
#include "fft_kernels.hpp"

namespace lgf {

template size_t fft_xy_lds_bytes<float>(const geom &);
template hipError_t launch_fft_xy<float>(const geom &, void *, int, const void *,
                                         const dev_status *, hipStream_t);
template zt_plan plan_zt<float>(const geom &, size_t);
template void fft_set_max_lds<float>(const geom &, const zt_plan &);
template bool xy_acc_fusable<float>(const geom &);
template hipError_t launch_fft_xy_inv_acc<float>(const geom &, void *, const void *, const void *,
                                                 void *, double, bool, const dev_status *,
                                                 hipStream_t);
template hipError_t launch_fft_zt<float>(const geom &, void *, int, const void *, const float *,
                                         float, const zt_plan &, const dev_status *, hipStream_t);

}  // namespace lgf
