// Run-time specialisation (hipRTC) of the pooled projection kernel and of
// the planner's round kernels: the robot's joint constants (twists, offsets,
// joint types, limits, base and tool frames, collision spheres) and the
// constraint's locked axes are written into the kernel source as constants,
// so the compiler folds them (zero twists and offsets drop out of the frame
// updates, prismatic tests and free-axis branches disappear: 42% fewer
// vector instructions for the 7-DOF arm on a plane).  The device code is the
// library's own (device.h, project.h, project_pool.h, collide.h,
// plan_device.h, handed to hipRTC as in-memory headers); only the policy
// class that supplies the constants is generated.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cerrno>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iterator>
#include <string>
#include <vector>

#include <sys/stat.h>
#include <unistd.h>

#include "cprrtc.h"
#include "device.h"
#include "handles.h"
#include "kernels.h"
#include "plan_device.h"
#include "rtc_sources.h"   // generated at build time: the headers above as strings

namespace cprrtc {
namespace {

std::string lit(float v) {
  char b[48];
  std::snprintf(b, sizeof b, "%.9ef", (double)v);   // round-trips a float exactly
  return b;
}

// The robot's device copy already holds rotation entries near 0 or +-1 as
// exactly those values (cp_robot_create), so the constants written here are
// the ones the library kernel reads.
std::string array(const char* name, const float* v, int n) {
  std::string s = std::string("    constexpr float ") + name + "[" + std::to_string(n) + "] = {";
  for (int i = 0; i < n; ++i) s += (i ? ", " : "") + lit(v[i]);
  return s + "};\n";
}

// The constant policy (same static functions as RobotMem) and the kernel.
std::string kernel_source(const RobotDev& h, int kind, unsigned mask, const float* spheres,
                          int n_spheres, bool with_pool, bool with_plan) {
  const int n = h.dof;
  std::string s;
  s += "#include \"device.h\"\n#include \"project.h\"\n#include \"project_pool.h\"\n"
       "#include \"plan_device.h\"\n";
  s += "using namespace cprrtc;\n";
  s += "struct RtcPolicy {\n";
  auto fn = [&](const char* name, const float* v, int cnt) {
    s += std::string("  static __device__ __forceinline__ float ") + name +
         "(const RobotDev*, int j) {\n" + array("v", v, cnt) + "    return v[j];\n  }\n";
  };
  fn("ca", h.ca, n);
  fn("sa", h.sa, n);
  fn("a", h.a, n);
  fn("d0", h.d0, n);
  fn("th0", h.th0, n);
  fn("lo", h.lo, n);
  fn("hi", h.hi, n);
  s += "  static __device__ __forceinline__ bool prismatic(const RobotDev*, int j) {\n"
       "    constexpr bool v[" + std::to_string(n) + "] = {";
  for (int j = 0; j < n; ++j) s += std::string(j ? ", " : "") + (h.prismatic[j] ? "true" : "false");
  s += "};\n    return v[j];\n  }\n";
  // a revolute joint whose limits (plus offset) stay within +-3.2 rad takes
  // the hardware sine and cosine
  s += "  static __device__ __forceinline__ bool short_angle(const RobotDev*, int j) {\n"
       "    constexpr bool v[" + std::to_string(n) + "] = {";
  for (int j = 0; j < n; ++j) s += std::string(j ? ", " : "") + (h.short_angle[j] ? "true" : "false");
  s += "};\n    return v[j];\n  }\n";
  const int b1 = h.n_chains > 1 ? h.chain_begin[1] : n;
  s += "  static __device__ __forceinline__ int chain1(const RobotDev*, int) { return " +
       std::to_string(b1) + "; }\n";
  for (const char* which : {"base", "tool"}) {
    const bool is_base = which[0] == 'b';
    float m[kMaxChains * 12];
    for (int c = 0; c < kMaxChains; ++c)
      for (int i = 0; i < 12; ++i) m[c * 12 + i] = is_base ? h.base[c][i] : h.tool[c][i];
    s += std::string("  static __device__ __forceinline__ float ") + which +
         "(const RobotDev*, int c, int i) {\n" + array("v", m, kMaxChains * 12) +
         "    return v[c * 12 + i];\n  }\n";
  }
  s += "  static __device__ __forceinline__ bool lock(const ConDev&, int i) {\n    constexpr bool v[6] = {";
  for (int i = 0; i < 6; ++i) s += std::string(i ? ", " : "") + ((mask >> i) & 1 ? "true" : "false");
  s += "};\n    return v[i];\n  }\n";
  // collision spheres (the planner validates its own motions)
  s += "  static __device__ __forceinline__ int n_chains(const RobotDev*) { return " +
       std::to_string(h.n_chains) + "; }\n";
  auto ints = [&](const char* name, const int* v, int cnt, const char* arg) {
    s += std::string("  static __device__ __forceinline__ int ") + name + "(const RobotDev*, int " +
         arg + ") {\n    constexpr int v[" + std::to_string(cnt) + "] = {";
    for (int i = 0; i < cnt; ++i) s += (i ? ", " : "") + std::to_string(v[i]);
    s += std::string("};\n    return v[") + arg + "];\n  }\n";
  };
  ints("chain_begin", h.chain_begin, kMaxChains + 1, "c");
  ints("sph_begin", h.sph_begin, kMaxDof + 1, "j");
  s += "  static __device__ __forceinline__ float4 sphere(const float4*, int i) {\n"
       "    constexpr float v[" + std::to_string(4 * std::max(1, n_spheres)) + "] = {";
  for (int i = 0; i < 4 * n_spheres; ++i) s += (i ? ", " : "") + lit(spheres[i]);
  s += "};\n    return make_float4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);\n  }\n};\n";
  if (with_pool) {
  s += "extern \"C\" __global__ __launch_bounds__(64) void cp_rtc_pool(\n"
       "    const RobotDev* __restrict__ rob, ConDev con, ProjDev prm, int n_motions,\n"
       "    const float* __restrict__ q_from, const float* __restrict__ q_to, float* __restrict__ xi,\n"
       "    int* __restrict__ status, int* __restrict__ iters, unsigned long long* __restrict__ work) {\n";
  s += "  project_pool_body<" + std::to_string(n) + ", " + std::to_string(kind) + ", 0, " +
       std::to_string(kPoolSlots) +
       ", RtcPolicy>(rob, con, prm, n_motions, q_from, q_to, nullptr, xi, status, iters, work);\n}\n";
    // FK + CC of independent configurations (fk_cc_batch without distances)
    for (int b : {4, 8})
      s += "extern \"C\" __global__ __launch_bounds__(256) void cp_rtc_fkcc" + std::to_string(b) +
           "(const RobotDev* __restrict__ rob, const float4* __restrict__ sph, EnvDev env,\n"
           "    int n_cfg, const float* __restrict__ q, unsigned char* __restrict__ collide, int early) {\n"
           "  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;\n"
           "  const bool on = i < n_cfg;\n"
           "  const float* qi = q + (on ? i : 0) * " + std::to_string(n) + ";\n"
           "  uint64_t hits;\n  float msd;\n  CcWork cw;\n  cc_work_clear(cw);\n"
           "  collide_config<" + std::to_string(b) + ", false, false, false, RtcPolicy>(rob, sph, env, qi, on,\n"
           "      0ull, early != 0, hits, msd, cw);\n"
           "  if (on) collide[i] = (unsigned char)((hits >> (threadIdx.x & 63)) & 1u);\n}\n";
    for (int b : {4, 8, 16})
      s += "extern \"C\" __global__ __launch_bounds__(256) void cp_rtc_validate" + std::to_string(b) +
           "(const RobotDev* __restrict__ rob, const float4* __restrict__ sph, EnvDev env, int W,\n"
           "    int n_motions, const float* __restrict__ xi, int* __restrict__ status,\n"
           "    unsigned long long* __restrict__ work, int early) {\n"
           "  validate_body<" + std::to_string(b) + ", true, RtcPolicy>(rob, sph, env, W, n_motions, xi,\n"
           "      status, work, early, (int64_t)blockIdx.x * 256 + threadIdx.x);\n}\n";
  }
  for (int b : {4, 8}) {
    if (!with_plan) break;
    s += "extern \"C\" __global__ __launch_bounds__(kPlanBlock) void cp_rtc_plan" + std::to_string(b) +
         "(const RobotDev* __restrict__ rob, const float4* __restrict__ sph, EnvDev env, ConDev con,\n"
         "    ProjDev prm, PlanDev pd) {\n"
         "  const int g = (int)((blockIdx.x * kPlanBlock + threadIdx.x) >> 6);\n"
         "  if (g >= pd.n_groups) return;\n"
         "  plan_extend<" + std::to_string(n) + ", " + std::to_string(kind) + ", " + std::to_string(b) +
         ", RtcPolicy>(rob, sph, env, con, prm, pd, pd.sample_base, g);\n}\n";
  }
  return s;
}

unsigned mask_bits(const ConDev& con) {
  unsigned m = 0;
  for (int i = 0; i < 6; ++i)
    if (con.mask[i] != 0.0f) m |= 1u << i;
  return m;
}

}  // namespace

bool rtc_find(cp_robot* robot, const ConDev& con, RtcFns* out) {
  std::lock_guard<std::mutex> g(robot->rtc_lock);
  const unsigned m = mask_bits(con);
  for (const RtcKernel& k : robot->rtc)
    if (k.kind == con.kind && k.mask == m) {
      *out = k.fns;
      return true;
    }
  return false;
}

hipError_t launch_rtc_pool(const RtcFns& k, const cp_robot* robot, const ConDev& con,
                           const ProjDev& prm, int n_motions, const float* q_from,
                           const float* q_to, float* xi, int* status, int* iters,
                           unsigned long long* work, hipStream_t stream) {
  const RobotDev* rob = robot->dev;
  ConDev c = con;
  ProjDev p = prm;
  void* args[] = {&rob, &c, &p, &n_motions, &q_from, &q_to, &xi, &status, &iters, &work};
  return hipModuleLaunchKernel(k.pool, pool_blocks(n_motions), 1, 1, 64, 1, 1, 0, stream, args,
                               nullptr);
}

hipError_t launch_rtc_fk_cc(const RtcFns& k, const cp_robot* robot, const EnvDev& env, int n_cfg,
                            const float* q, uint8_t* collide, bool early, int batch,
                            hipStream_t stream) {
  const RobotDev* rob = robot->dev;
  const float4* sph = robot->spheres;
  EnvDev e = env;
  int n = n_cfg, ea = early ? 1 : 0;
  void* args[] = {&rob, &sph, &e, &n, &q, &collide, &ea};
  const unsigned nb = (unsigned)(((int64_t)n_cfg + 255) / 256);
  return hipModuleLaunchKernel(k.fkcc[batch == 4 ? 0 : 1], nb, 1, 1, 256, 1, 1, 0, stream, args,
                               nullptr);
}

bool rtc_find_validate(cp_robot* robot, RtcFns* out) {
  std::lock_guard<std::mutex> g(robot->rtc_lock);
  for (const RtcKernel& k : robot->rtc)
    if (k.fns.validate[0]) {
      *out = k.fns;
      return true;
    }
  return false;
}

hipError_t launch_rtc_validate(const RtcFns& k, const cp_robot* robot, const EnvDev& env, int W,
                               int n_motions, const float* xi, int* status,
                               unsigned long long* work, bool early, int batch,
                               hipStream_t stream) {
  const RobotDev* rob = robot->dev;
  const float4* sph = robot->spheres;
  EnvDev e = env;
  int early_i = early ? 1 : 0;
  void* args[] = {&rob, &sph, &e, &W, &n_motions, &xi, &status, &work, &early_i};
  const unsigned nb = (unsigned)(((int64_t)n_motions * W + 255) / 256);
  return hipModuleLaunchKernel(k.validate[batch == 4 ? 0 : batch == 8 ? 1 : 2], nb, 1, 1, 256,
                               1, 1, 0, stream,
                               args, nullptr);
}

hipError_t launch_rtc_plan_round(const RtcFns& k, const cp_robot* robot, const EnvDev& env,
                                 const ConDev& con, const ProjDev& prm, const PlanDev& pd,
                                 int sphere_batch, unsigned blocks, size_t lds,
                                 hipStream_t stream) {
  const RobotDev* rob = robot->dev;
  const float4* sph = robot->spheres;
  EnvDev e = env;
  ConDev c = con;
  ProjDev p = prm;
  PlanDev d = pd;
  void* args[] = {&rob, &sph, &e, &c, &p, &d};
  return hipModuleLaunchKernel(k.plan[sphere_batch == 4 ? 0 : 1], blocks, 1, 1, kPlanBlock, 1, 1,
                               (unsigned)lds, stream, args, nullptr);
}

void rtc_release(cp_robot* robot) {
  std::lock_guard<std::mutex> g(robot->rtc_lock);
  for (RtcKernel& k : robot->rtc)
    for (hipModule_t m : k.modules) (void)hipModuleUnload(m);
  robot->rtc.clear();
}

// Compiled code objects are kept on disk, keyed by a hash of everything the
// compilation sees (the generated source, the library's device headers, the
// options, the target and the run-time compiler's version), so a later
// process skips the compiler.  The directory is $CPRRTC_RTC_CACHE (the
// value 0 turns the cache off), else $XDG_CACHE_HOME/cprrtc, else
// $HOME/.cache/cprrtc; a missing or unusable directory, or an unreadable
// entry, just means compiling.
uint64_t fnv1a(uint64_t h, const char* p, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    h ^= (unsigned char)p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

std::string cache_dir() {
  const char* e = std::getenv("CPRRTC_RTC_CACHE");
  if (e) return std::string(e) == "0" ? std::string() : std::string(e);
  const char* x = std::getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/cprrtc";
  const char* h = std::getenv("HOME");
  return h && *h ? std::string(h) + "/.cache/cprrtc" : std::string();
}

// mkdir -p of an absolute or relative directory; false if it is not usable
bool make_dirs(const std::string& d) {
  if (d.empty()) return false;
  for (size_t i = 1; i <= d.size(); ++i) {
    if (i == d.size() || d[i] == '/') {
      const std::string part = d.substr(0, i);
      if (mkdir(part.c_str(), 0755) != 0 && errno != EEXIST) return false;
    }
  }
  return access(d.c_str(), W_OK) == 0;
}

std::string cache_key(const std::string& src, const char* const* opts, int n_opts) {
  uint64_t a = 0xcbf29ce484222325ull, b = 0x84222325cbf29ce4ull;
  auto add = [&](const char* p, size_t n) {
    a = fnv1a(a, p, n);
    b = fnv1a(b ^ n, p, n);
  };
  add(src.data(), src.size());
  for (int i = 0; i < kRtcHeaderCount; ++i) {
    add(kRtcHeaderNames[i], std::strlen(kRtcHeaderNames[i]));
    add(kRtcHeaders[i], std::strlen(kRtcHeaders[i]));
  }
  for (int i = 0; i < n_opts; ++i) add(opts[i], std::strlen(opts[i]));
  // a code object from another run-time compiler is not reused
  int ver[2] = {0, 0};
  if (hiprtcVersion(&ver[0], &ver[1]) == HIPRTC_SUCCESS)
    add(reinterpret_cast<const char*>(ver), sizeof ver);
  char k[40];
  std::snprintf(k, sizeof k, "%016llx%016llx", (unsigned long long)a, (unsigned long long)b);
  return k;
}

std::vector<char> cache_read(const std::string& path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return {};
  return std::vector<char>(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
}

void cache_write(const std::string& dir, const std::string& path, const std::vector<char>& code) {
  if (!make_dirs(dir)) return;
  const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return;
    f.write(code.data(), (std::streamsize)code.size());
    if (!f) {
      std::remove(tmp.c_str());
      return;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

}  // namespace cprrtc

using namespace cprrtc;

extern "C" {

int cp_robot_specialize(cp_robot* robot, const cp_constraint* constraint, int32_t what,
                        double* compile_ms) {
  try {
    if (!robot) return api_fail(CP_E_ARG, "cp_robot_specialize: NULL robot");
    ConDev con;
    int rc = api_constraint(constraint, robot, &con);
    if (rc != CP_OK) return rc;
    const int dof = robot->host.dof;
    if (!dof_supported(dof)) return api_fail(CP_E_UNSUPPORTED, "cp_robot_specialize: dof %d", dof);
    if (con.kind == KIND_REL && dof % 2)
      return api_fail(CP_E_UNSUPPORTED, "cp_robot_specialize: relative pose needs an even dof");
    if (what == 0) what = CP_SPECIALIZE_PROJECT;
    if (what & ~(CP_SPECIALIZE_PROJECT | CP_SPECIALIZE_PLAN))
      return api_fail(CP_E_ARG, "cp_robot_specialize: what = %d", what);
    RtcFns have;
    rtc_find(robot, con, &have);
    const bool need_pool = (what & CP_SPECIALIZE_PROJECT) && !have.pool;
    const bool need_plan = (what & CP_SPECIALIZE_PLAN) && !have.plan[0];
    if (!need_pool && !need_plan) {
      if (compile_ms) *compile_ms = 0.0;
      return CP_OK;
    }
    const auto t0 = std::chrono::steady_clock::now();
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    hipDeviceProp_t props;
    if (he == hipSuccess) he = hipGetDeviceProperties(&props, dev);
    if (he != hipSuccess) return api_hip_fail(he, "cp_robot_specialize");
    // the spheres as stored on the device (grouped by link)
    std::vector<float4> sph(robot->host.n_spheres);
    he = hipMemcpy(sph.data(), robot->spheres, sizeof(float4) * sph.size(), hipMemcpyDeviceToHost);
    if (he != hipSuccess) return api_hip_fail(he, "cp_robot_specialize: spheres");
    const std::string src = kernel_source(robot->host, con.kind, mask_bits(con),
                                          reinterpret_cast<const float*>(sph.data()),
                                          robot->host.n_spheres, need_pool, need_plan);
    const std::string arch = std::string("--offload-arch=") + props.gcnArchName;
    // packed FP32 instructions stay out of every kernel, as in the library;
    // finite values without signed-zero distinctions let products with the
    // zero constants fold away (for finite operands x * 0 + y is exactly y,
    // so the results are those of the library kernel)
    const char* opts[] = {arch.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops", "-fno-signed-zeros",
                          "-ffinite-math-only"};
    const int n_opts = (int)(sizeof opts / sizeof opts[0]);
    const std::string dir = cache_dir();
    const std::string entry = dir.empty() ? std::string() : dir + "/" + cache_key(src, opts, n_opts) + ".co";
    hipModule_t module = nullptr;
    std::vector<char> code = entry.empty() ? std::vector<char>() : cache_read(entry);
    if (!code.empty() && hipModuleLoadData(&module, code.data()) != hipSuccess) module = nullptr;
    if (!module) {
      hiprtcProgram prog = nullptr;
      hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "cprrtc_rtc_pool.hip", kRtcHeaderCount,
                                           kRtcHeaders, kRtcHeaderNames);
      if (r != HIPRTC_SUCCESS)
        return api_fail(CP_E_RTC, "hiprtcCreateProgram: %s", hiprtcGetErrorString(r));
      r = hiprtcCompileProgram(prog, n_opts, opts);
      if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        if (log.size() > 400) log.resize(400);
        return api_fail(CP_E_RTC, "hiprtcCompileProgram: %s", log.c_str());
      }
      size_t size = 0;
      hiprtcGetCodeSize(prog, &size);
      code.assign(size, '\0');
      hiprtcGetCode(prog, code.data());
      hiprtcDestroyProgram(&prog);
      he = hipModuleLoadData(&module, code.data());
      if (he == hipSuccess && !entry.empty()) cache_write(dir, entry, code);
    }
    hipFunction_t pool = nullptr, plan4 = nullptr, plan8 = nullptr, val4 = nullptr, val8 = nullptr,
                  val16 = nullptr;
    if (he == hipSuccess && need_pool) he = hipModuleGetFunction(&pool, module, "cp_rtc_pool");
    if (he == hipSuccess && need_pool) he = hipModuleGetFunction(&val4, module, "cp_rtc_validate4");
    if (he == hipSuccess && need_pool) he = hipModuleGetFunction(&val8, module, "cp_rtc_validate8");
    if (he == hipSuccess && need_pool) he = hipModuleGetFunction(&val16, module, "cp_rtc_validate16");
    hipFunction_t fk4 = nullptr, fk8 = nullptr;
    if (he == hipSuccess && need_pool) he = hipModuleGetFunction(&fk4, module, "cp_rtc_fkcc4");
    if (he == hipSuccess && need_pool) he = hipModuleGetFunction(&fk8, module, "cp_rtc_fkcc8");
    if (he == hipSuccess && need_plan) he = hipModuleGetFunction(&plan4, module, "cp_rtc_plan4");
    if (he == hipSuccess && need_plan) he = hipModuleGetFunction(&plan8, module, "cp_rtc_plan8");
    if (he != hipSuccess) {
      if (module) (void)hipModuleUnload(module);
      return api_hip_fail(he, "cp_robot_specialize: loading the compiled kernel");
    }
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    {
      // one entry per (kind, mask); kernels compiled later join it (the
      // entry keeps every module it uses)
      std::lock_guard<std::mutex> g(robot->rtc_lock);
      RtcKernel* e = nullptr;
      for (RtcKernel& k : robot->rtc)
        if (k.kind == con.kind && k.mask == mask_bits(con)) e = &k;
      if (!e) {
        robot->rtc.emplace_back();
        e = &robot->rtc.back();
        e->kind = con.kind;
        e->mask = mask_bits(con);
      }
      e->modules.push_back(module);
      if (pool) {
        e->fns.pool = pool;
        e->fns.validate[0] = val4;
        e->fns.validate[1] = val8;
        e->fns.validate[2] = val16;
        e->fns.fkcc[0] = fk4;
        e->fns.fkcc[1] = fk8;
      }
      if (plan4) {
        e->fns.plan[0] = plan4;
        e->fns.plan[1] = plan8;
      }
      e->compile_ms += ms;
    }
    if (compile_ms) *compile_ms = ms;
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_robot_specialize: unexpected exception");
  }
}

}  // extern "C"
