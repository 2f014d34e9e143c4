// Workspace for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc): a fixed array in the
// library's device image, one copy per GPU, bound to a context by
// fr_sg_init_static.  Every context bound on a GPU shares that GPU's array.
#include <mutex>
#include <string>

#include "internal.hpp"

namespace {

constexpr int64_t kStaticWorkspaceBytes = int64_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

// the array itself; host code never passes this name to a kernel or a copy (on the
// host it only stands for the symbol): the device address comes from
// hipGetSymbolAddress, once per device
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

}  // namespace

extern "C" fr_sg_status fr_sg_init_static(const fr_sg_problem* problem, void* hip_stream, fr_sg_ctx** out) {
  if (!out) {
    frsg::set_init_error("out is NULL");
    return FRSG_EINVAL;
  }
  *out = nullptr;
  int64_t need = 0;
  const fr_sg_status st = fr_sg_workspace_size(problem, &need);  // validates; sets the error text
  if (st != FRSG_OK) return st;
  if (need > kStaticWorkspaceBytes) {
    frsg::set_init_error("problem needs a workspace of " + std::to_string(need) +
                         " bytes; the static workspace holds " + std::to_string(kStaticWorkspaceBytes) +
                         " (use fr_sg_init with a caller-allocated workspace)");
    return FRSG_EUNSUPPORTED;
  }
  int dev = -1;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    frsg::set_init_error(std::string("no current HIP device: ") + hipGetErrorString(he));
    return FRSG_EDEVICE;
  }
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (he != hipSuccess || !p) {
        frsg::set_init_error(std::string("hipGetSymbolAddress of the static workspace failed: ") +
                             hipGetErrorString(he));
        return FRSG_EDEVICE;
      }
      g_scratch_ptr[dev] = p;
    }
    ptr = g_scratch_ptr[dev];
  }
  return frsg::init_with_workspace(problem, hip_stream, ptr, kStaticWorkspaceBytes, out, false);
}
