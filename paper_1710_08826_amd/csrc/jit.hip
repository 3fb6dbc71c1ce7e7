// hipRTC compilation and the per-process program cache.
#include "jit.hpp"

#include <hip/hip_ext.h>
#include <hip/hiprtc.h>

#include <map>
#include <mutex>
#include <utility>

#include "internal.hpp"

namespace fn {

// Device headers embedded at build time (generated source).
extern const int kEmbeddedCount;
extern const char* const kEmbeddedNames[];
extern const char* const kEmbeddedTexts[];

JitProgram::~JitProgram() {
  if (mod) (void)hipModuleUnload(mod);
}

std::vector<char> jit_compile(const std::string& source, const std::string& arch) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, source.c_str(), "fn_model.hip", kEmbeddedCount, kEmbeddedTexts, kEmbeddedNames) !=
      HIPRTC_SUCCESS)
    throw Error(FN_E_INVALID, "hiprtcCreateProgram failed");
  const std::string arch_opt = "--offload-arch=" + arch;
  // the same code-generation flags as the library's own kernels
  const char* opts[] = {arch_opt.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  std::vector<char> code;
  if (rc != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    throw Error(FN_E_INVALID, "runtime compilation of the model kernels failed: " + log);
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  code.resize(n);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return code;
}

static std::string device_arch(int dev) {
  hipDeviceProp_t p;
  hip_check(hipGetDeviceProperties(&p, dev), "hipGetDeviceProperties");
  std::string a = p.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::shared_ptr<JitProgram> jit_load(const std::string& source, const std::vector<std::string>& names) {
  static std::mutex mu;
  static std::map<std::pair<int, std::string>, std::shared_ptr<JitProgram>> cache;
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  std::string key = source;
  for (const auto& n : names) key += "\n//kernel " + n;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({dev, key});
  if (it != cache.end()) return it->second;
  const std::vector<char> code = jit_compile(source, device_arch(dev));
  auto prog = std::make_shared<JitProgram>();
  hip_check(hipModuleLoadData(&prog->mod, code.data()), "hipModuleLoadData");
  for (const auto& n : names) {
    hipFunction_t f = nullptr;
    hip_check(hipModuleGetFunction(&f, prog->mod, n.c_str()), "hipModuleGetFunction");
    prog->fns.push_back(f);
  }
  cache[{dev, key}] = prog;
  return prog;
}

void jit_launch(hipFunction_t f, unsigned grid, unsigned block, hipStream_t s, void** args, hipEvent_t start,
                hipEvent_t stop) {
  if (start || stop) {
    const uint64_t items = (uint64_t)grid * block;
    if (items > 0xffffffffull) throw Error(FN_E_INVALID, "launch too large for a timed dispatch");
    hip_check(hipExtModuleLaunchKernel(f, (uint32_t)items, 1, 1, block, 1, 1, 0, s, args, nullptr, start, stop, 0),
              "hipExtModuleLaunchKernel");
    return;
  }
  hip_check(hipModuleLaunchKernel(f, grid, 1, 1, block, 1, 1, 0, s, args, nullptr), "hipModuleLaunchKernel");
}

}  // namespace fn
