// placeholder: adjoint kernels
#include "esim_internal.h"
namespace esim {
size_t backward_scratch_bytes(const ClipDev& hc, int64_t n) { (void)hc; return static_cast<size_t>(n) * 8; }
hipError_t launch_backward(const BackwardArgs& a, hipStream_t s) { (void)a; (void)s; return hipErrorNotSupported; }
}
