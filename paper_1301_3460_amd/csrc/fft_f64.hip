// FFT pass kernels instantiated for double.
#include "fft_kernels.hpp"

namespace lgf {

template hipError_t launch_fft_xy<double>(const geom &, void *, int, const void *, const fft_plan &,
                                          const dev_status *, hipStream_t);
template fft_plan plan_fft<double>(const geom &, size_t, int);
template void fft_set_max_lds<double>(const geom &, const fft_plan &);
template hipError_t launch_fft_zt<double>(const geom &, void *, int, const void *, const double *,
                                          double, const fft_plan &, const dev_status *, hipStream_t);

}  // namespace lgf
