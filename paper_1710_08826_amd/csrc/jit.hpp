// Runtime specialization of the hot kernels: a model's structure (which
// resonance sits in which pair with which spin, ...) becomes compile-time
// constants of a kernel compiled with hipRTC when the model is created, so the
// per-event code carries no branches or selects on the structure.  The device
// headers of the library are embedded in it at build time.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

namespace fn {

struct JitProgram {
  hipModule_t mod = nullptr;
  std::vector<hipFunction_t> fns;  // in the order the names were given
  ~JitProgram();
};

// Code object of `source` (which may include the embedded device headers) for
// `arch` (e.g. "gfx950"); throws Error(FN_E_INVALID) with the compiler log on
// failure.  Needs no device.
std::vector<char> jit_compile(const std::string& source, const std::string& arch);

// Compiled and loaded on the current device, with the kernels `names`;
// programs are cached per (device, source) for the life of the process.
std::shared_ptr<JitProgram> jit_load(const std::string& source, const std::vector<std::string>& names);

// Launch of a loaded kernel; args are pointers to the argument values.
// Launches f on grid x block; with start/stop events the dispatch itself
// records the kernel's start and end times into them (hipExtModuleLaunchKernel).
void jit_launch(hipFunction_t f, unsigned grid, unsigned block, hipStream_t s, void** args,
                hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

}  // namespace fn
