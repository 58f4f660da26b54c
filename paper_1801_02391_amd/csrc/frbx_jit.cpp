// Kernels specialised at run time: the float32 fringe kernel compiled by
// hipRTC for the IF lattice of a search (the rows of the first MBD pass that
// hold an IF), so that the pass reads and transforms only those rows.  The
// device code is the same source as the statically built kernel
// (frbx_fringe.h, embedded by the build as frbx_rtc_source.inc) and
// computes the same sums (a separate compilation: multiply-add fusion, and
// so the last bits, may differ).  Modules stay loaded until the process
// ends; one per (device, J, M, rows).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "frbx_internal.h"
#include "frbx_rtc_source.inc"

namespace frbx {
namespace {

struct JitEntry {
  hipModule_t module = nullptr;
  hipFunction_t fn = nullptr;
  std::string err;
};

std::mutex g_mu;
std::map<std::tuple<int, int, int, unsigned>, JitEntry> g_cache;

// Compile fringe_kernel<J, M, false, false, false, rows> for the current
// device's architecture; fills e.fn or e.err.
void compile(int J, int M, unsigned rows, JitEntry &e) {
  const std::string expr = "frbx::fringe_kernel<" + std::to_string(J) + ", " + std::to_string(M) +
                           ", false, false, false, " + std::to_string(rows) + "u>";
  hiprtcProgram prog = nullptr;
  if (hiprtcCreateProgram(&prog, kFringeRtcSource, "frbx_fringe_rtc.hip", 0, nullptr, nullptr) !=
      HIPRTC_SUCCESS) {
    e.err = "hiprtcCreateProgram failed";
    return;
  }
  if (hiprtcAddNameExpression(prog, expr.c_str()) != HIPRTC_SUCCESS) {
    e.err = "hiprtcAddNameExpression failed";
    hiprtcDestroyProgram(&prog);
    return;
  }
  // the options of the static build: gfx950, packed FP32 kept out
  const char *opts[] = {"--offload-arch=gfx950", "-O3",      "-std=c++17",       "-ffp-contract=fast",
                        "-Xclang",               "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult cr = hiprtcCompileProgram(prog, int(sizeof(opts) / sizeof(opts[0])), opts);
  if (cr != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    e.err = std::string("hipRTC compile: ") + hiprtcGetErrorString(cr) + ": " + log.substr(0, 400);
    hiprtcDestroyProgram(&prog);
    return;
  }
  const char *lowered = nullptr;
  size_t code_size = 0;
  if (hiprtcGetLoweredName(prog, expr.c_str(), &lowered) != HIPRTC_SUCCESS || !lowered ||
      hiprtcGetCodeSize(prog, &code_size) != HIPRTC_SUCCESS || code_size == 0) {
    e.err = "hipRTC: no code for " + expr;
    hiprtcDestroyProgram(&prog);
    return;
  }
  const std::string name(lowered);
  std::vector<char> code(code_size);
  const hiprtcResult gr = hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  if (gr != HIPRTC_SUCCESS) {
    e.err = "hiprtcGetCode failed";
    return;
  }
  hipError_t he = hipModuleLoadData(&e.module, code.data());
  if (he != hipSuccess) {
    e.err = std::string("hipModuleLoadData: ") + hipGetErrorString(he);
    e.module = nullptr;
    return;
  }
  he = hipModuleGetFunction(&e.fn, e.module, name.c_str());
  if (he != hipSuccess) {
    e.err = std::string("hipModuleGetFunction: ") + hipGetErrorString(he);
    e.fn = nullptr;
  }
}

}  // namespace

hipFunction_t fringe_rows_kernel(int device, int n_chan, int n_mbd, unsigned rows, std::string *err) {
  std::lock_guard<std::mutex> lock(g_mu);
  JitEntry &e = g_cache[std::make_tuple(device, n_chan, n_mbd, rows)];
  if (!e.fn && e.err.empty()) compile(n_chan, n_mbd, rows, e);
  if (!e.fn && err) *err = e.err;
  return e.fn;
}

hipError_t launch_fringe_rows(hipFunction_t fn, const FringeArgs &a, size_t lds_bytes, int grid,
                              hipStream_t s) {
  (void)hipGetLastError();
  if (!fn || grid <= 0) return grid <= 0 ? hipSuccess : hipErrorInvalidValue;
  FringeArgs arg = a;
  void *params[] = {&arg};
  return hipModuleLaunchKernel(fn, unsigned(grid), 1, 1, unsigned(kBlock), 1, 1, unsigned(lds_bytes), s, params,
                               nullptr);
}

}  // namespace frbx
