// The C ABI's host-side paths (argument validation, sizing, the tuning
// table's text format, the server's checks) with the library's host code
// built under AddressSanitizer and UndefinedBehaviorSanitizer, by
// tests/test_host_sanitizers.py. Runs without a GPU: every call here must
// return an error code or a host-computed value, never touch device memory.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "wsx.h"

#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "%s:%d: check failed: %s (last error: %s)\n",    \
                         __FILE__, __LINE__, #c, wsx_last_error());               \
            std::exit(1);                                                         \
        }                                                                         \
    } while (0)

static bool says(const char* what) { return std::strstr(wsx_last_error(), what) != nullptr; }

int main(int argc, char** argv) {
    const char* tmp = argc > 1 ? argv[1] : "/tmp";
    size_t b = 0;
    // state block sizes
    CHECK(wsx_env_state_bytes(99, 10, 10, &b) == WSX_EINVAL && says("unknown environment kind"));
    CHECK(wsx_env_state_bytes(WSX_PENDULUM, 0, 0, &b) == WSX_EINVAL);
    CHECK(wsx_env_state_bytes(WSX_PENDULUM, 10, 12, &b) == WSX_EINVAL);
    CHECK(wsx_env_state_bytes(WSX_MARKET, 3, 300, nullptr) == WSX_EINVAL);
    for (int kind = WSX_CARTPOLE; kind <= WSX_REACTION; ++kind) {
        const int64_t rows = kind == WSX_MARKET ? 5000 : 1000;
        CHECK(wsx_env_state_bytes(kind, 1000, rows, &b) == WSX_OK && b % 256 == 0 && b > 0);
    }
    // create: every argument check before any device work
    wsx_env* env = nullptr;
    CHECK(wsx_env_create(nullptr, &env) == WSX_EINVAL);
    wsx_env_desc d{};
    d.kind = WSX_MARKET;
    d.n_envs = 3;
    d.state = reinterpret_cast<void*>(0x1000);
    CHECK(wsx_env_create(&d, &env) == WSX_EINVAL && says("agent_offsets"));
    std::vector<int32_t> off = {0, 5, 300, 310};   // an env of 295 agents
    d.agent_offsets = off.data();
    CHECK(wsx_env_create(&d, &env) != WSX_OK);
    d.kind = WSX_REACTION;
    d.agent_offsets = nullptr;
    CHECK(wsx_env_create(&d, &env) == WSX_EINVAL && says("params"));
    d.kind = WSX_PENDULUM;
    d.tile_rows = -1;
    CHECK(wsx_env_create(&d, &env) == WSX_EINVAL);
    d.tile_rows = 7;
    d.waves = 3;
    CHECK(wsx_env_create(&d, &env) != WSX_OK);
    CHECK(env == nullptr);
    // calls on a NULL handle
    CHECK(wsx_env_reset(nullptr, 0, nullptr) == WSX_EINVAL);
    CHECK(wsx_rollout(nullptr, nullptr, 1, nullptr, WSX_MODE_FUSED, nullptr) == WSX_EINVAL);
    CHECK(wsx_env_info(nullptr, nullptr, nullptr, nullptr) == WSX_EINVAL);
    CHECK(wsx_env_tiles(nullptr, nullptr, nullptr) == WSX_EINVAL);
    CHECK(wsx_env_set_step(nullptr, 3) == WSX_EINVAL);
    CHECK(wsx_env_set_chunk(nullptr, 3) == WSX_EINVAL);
    CHECK(wsx_env_destroy(nullptr) == WSX_EINVAL);
    CHECK(wsx_env_shape(nullptr, nullptr, nullptr, nullptr, nullptr) == WSX_EINVAL);
    CHECK(wsx_rollout_batch(nullptr, nullptr, nullptr, 0, 1, nullptr) == WSX_EINVAL);
    // returns / GAE
    float f = 0.0f;
    uint8_t u = 0;
    CHECK(wsx_compute_returns(&f, &f, &u, &f, -1, 1, 0.99, 0.95, 1, &f, &f, WSX_F32, nullptr) ==
          WSX_EINVAL);
    CHECK(wsx_compute_returns(&f, &f, &u, &f, 1, 1, 1.5, 0.95, 1, &f, &f, WSX_F32, nullptr) ==
          WSX_EINVAL);
    CHECK(wsx_compute_returns(&f, &f, &u, &f, 1, 1, 0.99, 0.95, 1, &f, &f, WSX_BF16, nullptr) ==
          WSX_EUNSUPPORTED);
    CHECK(wsx_compute_returns(nullptr, &f, &u, &f, 1, 1, 0.99, 0.95, 1, &f, &f, WSX_F32,
                              nullptr) == WSX_EINVAL);
    CHECK(wsx_compute_returns(nullptr, nullptr, nullptr, nullptr, 0, 5, 0.99, 0.95, 1, nullptr,
                              nullptr, WSX_F64, nullptr) == WSX_OK);   // nothing to do
    // policy checks
    wsx_policy p{};
    p.dtype = WSX_BF16;
    p.d_in = 3;
    p.h1 = p.h2 = 256;
    p.n_head = 2;
    // pointers the host only checks for NULL (never dereferenced here)
    p.w1 = p.w2 = p.w3 = &f;
    p.b1 = p.b2 = p.b3 = &f;
    p.log_std = &f;
    CHECK(wsx_policy_forward(nullptr, &f, 1, &f, nullptr) == WSX_EINVAL);
    CHECK(wsx_policy_forward(&p, &f, -1, &f, nullptr) == WSX_EINVAL);
    CHECK(wsx_policy_trace(nullptr, &p, &f, 1, &f, &f, &f, nullptr) == WSX_EINVAL);
    CHECK(wsx_quantize(7, 1.0f, &f, &f, 1, nullptr) == WSX_EINVAL);
    CHECK(wsx_quantize(WSX_FP8_E4M3, 3.0f, &f, &f, 1, nullptr) == WSX_EINVAL && says("power of two"));
    CHECK(wsx_quantize(WSX_BF16, 1.0f, &f, &f, -1, nullptr) == WSX_EINVAL);
    // the update: sizes are host arithmetic; FP8 is rejected
    CHECK(wsx_ac_grad_workspace_bytes(&p, 1000, &b) == WSX_OK && b > 1000 * 256 * 2);
    size_t b2 = 0;
    CHECK(wsx_ac_grad_workspace_bytes(&p, int64_t(1) << 30, &b2) == WSX_OK && b2 >= b);
    CHECK(wsx_ac_grad_workspace_bytes(&p, 0, &b) == WSX_EINVAL);
    wsx_grads g{};
    CHECK(wsx_ac_grad(&p, 0, &f, &f, &f, &f, 10, 0.5f, 0.0f, &g, nullptr, 0, nullptr) ==
          WSX_EINVAL);
    CHECK(wsx_ac_grad_static(&p, 0, &f, &f, &f, &f, WSX_AC_STATIC_MAX_SAMPLES + 1, 0.5f, 0.0f,
                             &g, nullptr) == WSX_EINVAL && says("at most"));
    p.dtype = WSX_FP8_E4M3;
    CHECK(wsx_ac_grad_workspace_bytes(&p, 10, &b) == WSX_EUNSUPPORTED);
    CHECK(wsx_adam_step(&f, &f, &f, &f, 1, 0, 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr, WSX_F32,
                        nullptr) == WSX_EINVAL);
    CHECK(wsx_adam_step(&f, &f, &f, &f, 1, 1, 1e-3f, 1.5f, 0.999f, 1e-8f, nullptr, WSX_F32,
                        nullptr) == WSX_EINVAL);
    CHECK(wsx_adam_step_many(nullptr, 0, 1, 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr) != WSX_OK);
    // the tuning table: save and load round trip through its text format
    wsx_tune_entry e{};
    CHECK(wsx_tune_lookup(WSX_PENDULUM, 123, 123, 256, &e) != WSX_OK);
    const std::string path = std::string(tmp) + "/wsx_tune_test.txt";
    {
        FILE* fp = std::fopen(path.c_str(), "w");
        CHECK(fp);
        std::fprintf(fp, "2 123 123 256 80 8 2 25 5.5\n4 7 300 256 128 8 2 0 41.0\n");
        std::fclose(fp);
    }
    CHECK(wsx_tune_load(path.c_str()) == WSX_OK);
    CHECK(wsx_tune_lookup(WSX_PENDULUM, 123, 123, 256, &e) == WSX_OK);
    CHECK(e.tile_rows == 80 && e.waves == 8 && e.occupancy == 2 && e.chunk_steps == 25);
    CHECK(wsx_tune_save(path.c_str()) == WSX_OK);
    CHECK(wsx_tune_load(path.c_str()) == WSX_OK);
    CHECK(wsx_tune_lookup(WSX_MARKET, 7, 300, 256, &e) == WSX_OK && e.tile_rows == 128);
    CHECK(wsx_tune_load("/nonexistent/dir/tune.txt") != WSX_OK);
    {
        FILE* fp = std::fopen(path.c_str(), "w");
        std::fprintf(fp, "2 1 2 3 not numbers\n");
        std::fclose(fp);
    }
    CHECK(wsx_tune_load(path.c_str()) != WSX_OK);
    std::remove(path.c_str());
    CHECK(wsx_autotune_workspace_bytes(nullptr, 10, &b) == WSX_EINVAL);
    // the server's argument checks
    wsx_server* srv = nullptr;
    wsx_server_desc sd{};
    CHECK(wsx_server_create(&sd, &srv) == WSX_EINVAL);
    CHECK(wsx_server_create(nullptr, &srv) == WSX_EINVAL);
    CHECK(wsx_server_submit(nullptr, nullptr, nullptr) == WSX_EINVAL);
    CHECK(wsx_server_wait(nullptr, 1, 0, nullptr) == WSX_EINVAL);
    CHECK(wsx_server_release(nullptr, 1) == WSX_EINVAL);
    CHECK(wsx_server_get_stats(nullptr, nullptr) == WSX_EINVAL);
    CHECK(wsx_server_destroy(nullptr) == WSX_EINVAL);
    // user kinds: descriptor checks
    wsx_user_kind_desc ud{};
    int32_t kind = 0;
    CHECK(wsx_user_kind_register(&ud, "struct UserEnv {};", &kind) == WSX_EINVAL);
    CHECK(wsx_user_kind_register(nullptr, "", &kind) == WSX_EINVAL);
    std::printf("abi host paths under sanitizers: ok\n");
    return 0;
}
