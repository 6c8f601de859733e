// compose.cpp -- user environment kinds compiled at run time (arXiv
// 2408.00930, Sec. 2: the framework is environment-agnostic; App. B: user
// environments are compiled for the device and run in the same GPU-resident
// loop -- there with Numba, here with the HIP run-time compiler).
//
// A user kind is the source of a `struct UserEnv` with the interface of the
// built-in kinds (envs.h). Registration wraps it into a program that includes
// the fused roll-out's templates (rollout_kernels.h), compiles k_fused and
// k_reset for UserEnv with hipRTC for the current device, loads the code
// object and records the kind. From then on the kind goes through the same
// entry points as a built-in one; its launches use the loaded functions.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "wsx.h"

namespace wsx {

namespace {

struct UserKind {
    int kind;
    KindInfo info;
    Variant v;          // the one compiled shape
    int device;
    hipModule_t mod;
    hipFunction_t fused, reset;
};

std::mutex g_mu;
std::vector<UserKind> g_kinds;   // kind kUserKindBase + i

// The fused kernel's shape for a policy format and width: the built-in
// kinds' default shape of that format (split-M head for heads wider than 16).
bool user_shape(int dtype, int hidden, int n_head, int& nw, int& nt, int& hs, int& occ) {
    const bool wide = n_head > 16;
    if (dtype == WSX_F32 && hidden == 64 && !wide) { nw = 4; nt = 1; hs = 0; occ = 1; return true; }
    if (dtype == WSX_BF16 && hidden == 256) {
        if (wide) { nw = 8; nt = 8; hs = 1; occ = 2; } else { nw = 8; nt = 5; hs = 0; occ = 2; }
        return true;
    }
    return false;
}

// The directory of this library's sources: <package>/csrc next to libwsx.so.
std::string source_dir() {
    Dl_info info{};
    if (!dladdr(reinterpret_cast<void*>(&source_dir), &info) || !info.dli_fname) return "";
    std::string p = info.dli_fname;
    const size_t slash = p.rfind('/');
    return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/csrc";
}

const UserKind* find_kind(int kind) {
    const int i = kind - kUserKindBase;
    return i >= 0 && i < (int)g_kinds.size() ? &g_kinds[i] : nullptr;
}

// The kernels of a kind are loaded on the device current at registration.
bool on_device(int device) {
    int cur = -1;
    return hipGetDevice(&cur) == hipSuccess && cur == device;
}

}  // namespace

bool user_kind_info(int kind, KindInfo& k) {
    std::lock_guard<std::mutex> lk(g_mu);
    const UserKind* u = find_kind(kind);
    if (!u) return false;
    k = u->info;
    return true;
}

bool user_variant(int kind, Variant& v) {
    std::lock_guard<std::mutex> lk(g_mu);
    const UserKind* u = find_kind(kind);
    if (!u) return false;
    v = u->v;
    return true;
}

hipError_t launch_user_fused(const Variant& v, const Batch& batch, int grid, hipStream_t s) {
    hipFunction_t f = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        const UserKind* u = find_kind(v.kind);
        if (!u) return hipErrorInvalidValue;
        if (!on_device(u->device)) return hipErrorInvalidDevice;
        f = u->fused;
    }
    void* args[] = {const_cast<Batch*>(&batch)};
    return hipModuleLaunchKernel(f, grid, 1, 1, v.waves * 64, 1, 1, 0, s, args, nullptr);
}

hipError_t launch_user_reset(int kind, const EnvArgs& env, hipStream_t s) {
    hipFunction_t f = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        const UserKind* u = find_kind(kind);
        if (!u) return hipErrorInvalidValue;
        if (!on_device(u->device)) return hipErrorInvalidDevice;
        f = u->reset;
    }
    const int threads = 256;
    const unsigned blocks = (unsigned)((env.n_rows + threads - 1) / threads);
    void* args[] = {const_cast<EnvArgs*>(&env)};
    return hipModuleLaunchKernel(f, blocks, 1, 1, threads, 1, 1, 0, s, args, nullptr);
}

int user_blocks_per_cu(const Variant& v) {
    hipFunction_t f = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        const UserKind* u = find_kind(v.kind);
        if (!u) return 1;
        f = u->fused;
    }
    int n = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, v.waves * 64, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace wsx

using namespace wsx;

extern "C" int wsx_user_kind_register(const wsx_user_kind_desc* d, const char* source,
                                      int32_t* kind) {
    if (!d || !source || !kind) return fail(WSX_EINVAL, "desc, source and kind must not be NULL");
    if (d->state_dim < 1 || d->state_dim > 64 || d->obs_dim < 1 || d->obs_dim > 64)
        return fail(WSX_EINVAL, "state_dim and obs_dim must lie in 1..64");
    if (d->n_actions != 0 && (d->n_actions < 2 || d->n_actions > 255))
        return fail(WSX_EINVAL, "n_actions must be 0 (Gaussian) or 2..255 (categorical)");
    const int n_head = (d->n_actions ? d->n_actions : 1) + 1;
    int nw, nt, hs, occ;
    if (!user_shape(d->dtype, d->hidden, n_head, nw, nt, hs, occ))
        return fail(WSX_EUNSUPPORTED,
                    "user kinds run FP32 policies of width 64 (heads <= 16) or BF16 policies of "
                    "width 256 (got dtype %d, width %d, %d head outputs)",
                    d->dtype, d->hidden, n_head);
    const std::string dir = source_dir();
    if (dir.empty()) return fail(WSX_EINVAL, "cannot locate the library's sources");

    std::lock_guard<std::mutex> lk(g_mu);
    const int id = kUserKindBase + (int)g_kinds.size();
    char asserts[512];
    std::snprintf(asserts, sizeof asserts,
                  "namespace wsx {\n"
                  "static_assert(UserEnv::KIND == WSX_USER_KIND, \"UserEnv::KIND must be WSX_USER_KIND\");\n"
                  "static_assert(UserEnv::SD == %d && UserEnv::OD == %d && UserEnv::NACT == %d,"
                  " \"UserEnv's sizes differ from the descriptor\");\n"
                  "static_assert(UserEnv::SR >= UserEnv::SD && UserEnv::LANES >= 1, \"UserEnv::SR, LANES\");\n"
                  "}\n",
                  d->state_dim, d->obs_dim, d->n_actions);
    const std::string program = std::string("#include \"rollout_kernels.h\"\nnamespace wsx {\n#line 1 \"user_env\"\n") +
                                source + "\n}\n" + asserts;
    char fused_name[160], reset_name[64];
    std::snprintf(fused_name, sizeof fused_name,
                  "wsx::k_fused<wsx::UserEnv, wsx::UserEnv, %d, %d, %d, %d, %d, %d>", d->dtype,
                  d->hidden, nw, nt, hs, occ);
    std::snprintf(reset_name, sizeof reset_name, "wsx::k_reset<wsx::UserEnv>");

    // the current device's architecture (the library's own target when none)
    std::string arch = "gfx950";
    int device = -1;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&device) == hipSuccess && hipGetDeviceProperties(&prop, device) == hipSuccess)
        arch = prop.gcnArchName;
    else
        device = -1;
    const std::string o_arch = "--offload-arch=" + arch, o_inc = "-I" + dir;
    const std::string o_kind = "-DWSX_USER_KIND=" + std::to_string(id);
    const char* opts[] = {o_arch.c_str(), "-O3", "-std=c++17", "-ffp-contract=on", "-Xclang",
                          "-target-feature", "-Xclang", "-packed-fp32-ops", o_inc.c_str(),
                          o_kind.c_str()};
    hiprtcProgram prog = nullptr;
    if (hiprtcCreateProgram(&prog, program.c_str(), "user_env.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        return fail(WSX_EINVAL, "hiprtcCreateProgram failed");
    hiprtcAddNameExpression(prog, fused_name);
    hiprtcAddNameExpression(prog, reset_name);
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        if (log.size() > 1500) log.resize(1500);
        return fail(WSX_EINVAL, "the environment source does not compile:\n%s", log.c_str());
    }
    const char* lf = nullptr;
    const char* lr = nullptr;
    hiprtcGetLoweredName(prog, fused_name, &lf);
    hiprtcGetLoweredName(prog, reset_name, &lr);
    const std::string fname = lf ? lf : "", rname = lr ? lr : "";
    size_t size = 0;
    hiprtcGetCodeSize(prog, &size);
    std::vector<char> code(size);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    if (device < 0) return fail(WSX_EHIP, "compiled, but no HIP device to load the kernels on");

    UserKind u{};
    u.kind = id;
    u.info = KindInfo{d->state_dim, d->obs_dim, d->n_actions, d->dtype, d->hidden, 16 * nt, nw, occ};
    u.v = Variant{id, d->dtype, d->hidden, nw, 16 * nt, occ, 0};
    u.device = device;
    hipError_t e = hipModuleLoadData(&u.mod, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&u.fused, u.mod, fname.c_str());
    if (e == hipSuccess) e = hipModuleGetFunction(&u.reset, u.mod, rname.c_str());
    if (e != hipSuccess) {
        if (u.mod) (void)hipModuleUnload(u.mod);
        return hip_fail(e, "wsx_user_kind_register (load)");
    }
    g_kinds.push_back(u);
    *kind = id;
    return WSX_OK;
}
