// The SVD harness links the host offline stage without the GPU kernel-tensor generator;
// these definitions satisfy the linker and are never called by the harness.
#include "../../paper_2511_03109_amd/csrc/ph_host.hpp"

namespace ph {

GpuTensorGen::GpuTensorGen(const TreeData&, ph_kernel, const double*, int) : p_(nullptr) {
  fail(PH_EUNSUPPORTED, "the SVD harness has no GPU kernel-tensor generation");
}
GpuTensorGen::~GpuTensorGen() {}
void GpuTensorGen::near(const std::vector<NearJob>&, int, double*, int64_t) {}
void GpuTensorGen::far(const std::vector<double>&, int, int, double*) {}
void GpuTensorGen::near_qr(const std::vector<NearJob>&, int, int64_t, double*) {}
void GpuTensorGen::near_factors(const std::vector<NearJob>&, int, const std::vector<double>&,
                                const std::vector<int64_t>&, const std::vector<int32_t>&,
                                const std::vector<int64_t>&, int64_t, double*) {}

}  // namespace ph
