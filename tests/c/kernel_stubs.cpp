// Stand-ins for the kernel launchers (test code): the host-only plan paths
// never launch, so a host build of plan.cpp and compiler.cpp links against
// these for the sanitizer runs; every launcher reports "not supported".
#include "kernels.hpp"

namespace nbs {

hipError_t launch_two_point(int, const TwoPointArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_absmax(const void*, unsigned*, long long, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fill_u32(unsigned*, unsigned, long long, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_scale_exps(const unsigned*, int*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_channel_scale(const int*, const int*, double*, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_nbb(int, const NbbArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fft_pass(int, const FftArgs&, hipStream_t) { return hipErrorNotSupported; }
bool fft_line_supported(int, int) { return false; }
int fft_plane_fields(int, long long, int) { return 0; }
int fft_cube_fields(int, long long, int) { return 0; }
hipError_t launch_fft_cube(int, int, const FftPlaneArgs&, hipStream_t) { return hipErrorNotSupported; }
bool fft_cube_inv_supported(int, int) { return false; }
hipError_t launch_fft_cube_inv(int, const FftArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fft_plane(int, int, const FftPlaneArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fft_line(int, const FftArgs&, hipStream_t) { return hipErrorNotSupported; }
size_t contract_lds_bytes(int, int, int, int, int) { return 0; }
size_t contract_seg_lds_bytes(int, int, int, int, int, int) { return 0; }
int contract_waves(int prec) { return prec == 0 ? 8 : 4; }
hipError_t launch_contract(int, const ContractArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t prepare_kernels(int, int, size_t, int) { return hipErrorNotSupported; }

}  // namespace nbs
