// FFT pass kernels instantiated for float.
#include "fft_kernels.hpp"

namespace lgf {

template hipError_t launch_fft_xy<float>(const geom &, void *, int, const void *, const fft_plan &,
                                         const dev_status *, hipStream_t);
template fft_plan plan_fft<float>(const geom &, size_t, int);
template void fft_set_max_lds<float>(const geom &, const fft_plan &);
template bool xy_acc_fusable<float>(const geom &, const fft_plan &);
template hipError_t launch_fft_xy_inv_acc<float>(const geom &, void *, const void *,
                                                 const fft_plan &, const void *, void *, double,
                                                 bool, const dev_status *, hipStream_t);
template hipError_t launch_fft_zt<float>(const geom &, void *, int, const void *, const float *,
                                         float, const fft_plan &, const dev_status *, hipStream_t);

}  // namespace lgf
