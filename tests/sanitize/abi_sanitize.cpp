// Host-side checks of libsvdlut under AddressSanitizer and UndefinedBehaviorSanitizer, for a
// build without a GPU: the argument validation of every entry point (the cases of
// tests/test_abi_cpu.py, which must fail before any HIP call), the size queries at the edges
// of their ranges, the deterministic-mode switch, and the tuning-cache parser on well-formed,
// truncated, corrupt and random input.  Prints "OK <checks>" and exits 0 when every check
// holds; a sanitizer report aborts the run.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>

#include "../../include/svdlut.h"
#include "../../paper_2508_16121_amd/csrc/tune_cache.h"

static int g_checks = 0, g_failed = 0;

#define CHECK(cond)                                                                 \
    do {                                                                            \
        ++g_checks;                                                                 \
        if (!(cond)) {                                                              \
            ++g_failed;                                                             \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
        }                                                                           \
    } while (0)

// a refused call: non-zero status and a message naming what was wrong
static void refused(svdlut_status st, const char* needle) {
    CHECK(st != SVDLUT_OK);
    const char* msg = svdlut_last_error();
    CHECK(msg != nullptr);
    if (msg && needle) {
        const bool found = std::strstr(msg, needle) != nullptr;
        CHECK(found);
        if (!found) std::fprintf(stderr, "  message \"%s\" lacks \"%s\"\n", msg, needle);
    }
}

static void validation() {
    void* f = reinterpret_cast<void*>(0x1000);   // never dereferenced: every call fails first
    const float* cf = static_cast<const float*>(f);
    float* ff = static_cast<float*>(f);
    const svdlut_dtype F32 = SVDLUT_F32;
    const svdlut_dtype BAD = static_cast<svdlut_dtype>(7);
    refused(svdlut_reconstruct(nullptr, cf, cf, ff, 9, 33, 8, nullptr), "null");
    refused(svdlut_reconstruct(cf, cf, cf, ff, 9, 41, 8, nullptr), nullptr);
    refused(svdlut_reconstruct(cf, cf, cf, ff, 9, 33, 65, nullptr), nullptr);
    refused(svdlut_reconstruct(cf, cf, cf, ff, 0, 33, 8, nullptr), nullptr);
    const int bad_dims[][7] = {{0, 4, 4, 1, 1, 33, 8}, {1, 0, 4, 1, 1, 33, 8}, {1, 4, 70000, 1, 1, 33, 8},
                               {1, 4, 4, 0, 1, 33, 8}, {1, 4, 4, 1, 1, 1, 8}, {INT32_MIN, 4, 4, 1, 1, 33, 8},
                               {1, 4, 4, 1, INT32_MAX, 33, 8}, {1, 4, 4, 1, 1, 33, INT32_MIN}};
    for (const auto& d : bad_dims)
        refused(svdlut_apply(f, f, F32, cf, cf, cf, f, F32, nullptr, d[0], d[1], d[2], d[3], d[4], d[5], d[6], nullptr),
                nullptr);
    refused(svdlut_apply(f, f, BAD, cf, cf, cf, f, F32, nullptr, 1, 4, 4, 1, 1, 33, 8, nullptr), "dtype");
    refused(svdlut_apply_grid(f, f, F32, cf, cf, cf, f, F32, nullptr, nullptr, cf, cf, 6, 17, 1, 4, 4, 1, 1, 33, 8,
                              nullptr), "grid");
    for (int K : {0, 13, -1, INT32_MAX})
        refused(svdlut_apply_grid(f, f, F32, cf, cf, cf, f, F32, nullptr, cf, cf, cf, K, 17, 1, 4, 4, 1, 1, 33, 8,
                                  nullptr), nullptr);
    for (int Ds : {1, 34, INT32_MIN})
        refused(svdlut_apply_grid(f, f, F32, cf, cf, cf, f, F32, nullptr, cf, cf, cf, 6, Ds, 1, 4, 4, 1, 1, 33, 8,
                                  nullptr), nullptr);
    refused(svdlut_apply_grid_bwd(f, f, F32, cf, cf, cf, f, F32, cf, cf, 6, 17, f, nullptr, nullptr, nullptr,
                                  nullptr, nullptr, ff, nullptr, nullptr, 1, 8, 8, 1, 1, 33, 8, f, 1u << 30, nullptr),
            "all set");
    refused(svdlut_apply_grid_bwd(f, f, F32, cf, cf, cf, f, F32, cf, cf, 6, 17, nullptr, nullptr, nullptr, nullptr,
                                  nullptr, nullptr, ff, ff, ff, 1, 8, 8, 1, 1, 33, 8, f, 16, nullptr), "workspace");
    refused(svdlut_unfused_apply(nullptr, ff, cf, cf, cf, cf, cf, cf, 6, 17, 33, 1, 8, 8, f, 1u << 30, nullptr),
            nullptr);
    refused(svdlut_unfused_apply(cf, ff, cf, cf, cf, cf, cf, cf, 6, 17, 41, 1, 8, 8, f, 1u << 30, nullptr), nullptr);
    refused(svdlut_unfused_apply(cf, ff, cf, cf, cf, cf, cf, cf, 6, 17, 33, 1, 8, 8, f, 16, nullptr), "workspace");
    refused(svdlut_apply_bwd(f, f, F32, cf, cf, cf, f, F32, f, ff, nullptr, ff, nullptr, nullptr, 1, 8, 8, 1, 1, 33,
                             8, f, 1u << 30, nullptr), "all set");
    refused(svdlut_apply_bwd(f, f, F32, cf, cf, cf, f, F32, nullptr, ff, ff, ff, nullptr, nullptr, 1, 8, 8, 1, 1, 33,
                             8, f, 16, nullptr), "workspace");
    CHECK(svdlut_apply_bwd(f, f, F32, cf, cf, cf, f, F32, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 1, 8,
                           8, 1, 1, 33, 8, nullptr, 0, nullptr) == SVDLUT_OK);
    refused(svdlut_apply_bwd_noalloc(f, f, F32, cf, cf, cf, f, F32, nullptr, ff, ff, ff, nullptr, nullptr, 600, 4, 4,
                                     1, 1, 33, 8, nullptr), "scratch");
    refused(svdlut_apply_loss_bwd(f, f, F32, cf, cf, cf, f, F32, nullptr, static_cast<svdlut_loss_kind>(9), ff, f,
                                  nullptr, nullptr, nullptr, nullptr, nullptr, 1, 8, 8, 1, 1, 33, 8, f, 1u << 30,
                                  nullptr), "kind");
    refused(svdlut_apply_loss_bwd(f, f, F32, cf, cf, cf, f, F32, nullptr, SVDLUT_LOSS_L1, ff, f, nullptr, nullptr,
                                  nullptr, nullptr, nullptr, 1, 8, 8, 1, 1, 33, 8, f, 16, nullptr), "workspace");
    refused(svdlut_loss(f, f, F32, 0, SVDLUT_LOSS_L1, ff, nullptr, f, 64, nullptr), nullptr);
    refused(svdlut_loss(f, f, F32, 100, static_cast<svdlut_loss_kind>(5), ff, nullptr, f, 64, nullptr), nullptr);
    refused(svdlut_adam_step(ff, cf, ff, ff, 10, 1e-4f, 0.9f, 0.999f, 1e-8f, 0, nullptr), nullptr);
    refused(svdlut_adam_step(ff, cf, ff, ff, 10, 1e-4f, 1.5f, 0.999f, 1e-8f, 1, nullptr), nullptr);
    svdlut_plan* plan = nullptr;
    refused(svdlut_plan_create(nullptr, 1, 33, 8, F32, F32, &plan), nullptr);
    refused(svdlut_plan_launch(nullptr, f, f, cf, cf, cf, f, nullptr, nullptr), nullptr);
    refused(svdlut_plan_set_shape(nullptr, 512, 1, 4), nullptr);
    CHECK(svdlut_plan_destroy(nullptr) == SVDLUT_OK);
    refused(svdlut_generator_fwd(nullptr, f, F32, 1, 256, 256, 33, 8, ff, ff, ff, ff, f, 1u << 30, nullptr), nullptr);
    refused(svdlut_generator_fwd(cf, f, F32, 1, 256, 256, 33, 8, ff, ff, ff, ff, f, 16, nullptr), nullptr);
    refused(svdlut_generator_bwd(cf, nullptr, cf, cf, cf, ff, 1, 33, 8, f, 1u << 30, nullptr), nullptr);
    refused(svdlut_lut1d_apply(nullptr, ff, cf, 1, 4, 4, 33, nullptr), nullptr);
    refused(svdlut_lut3d_apply(cf, ff, cf, 1, 4, 4, 41, f, 1u << 30, nullptr), nullptr);
}

static void size_queries() {
    CHECK(svdlut_apply_bwd_workspace_size(0, 33) == 0);
    CHECK(svdlut_apply_bwd_workspace_size(INT32_MAX, 33) > 0);
    CHECK(svdlut_apply_bwd_workspace_size(1, 41) == 0);
    CHECK(svdlut_apply_loss_bwd_workspace_size(INT32_MIN, 33) == 0);
    CHECK(svdlut_apply_grid_bwd_workspace_size(1, 33, 34) == 0);
    CHECK(svdlut_deterministic_workspace_size(1, 65535, 65535, 65535, 65535) > 0);
    CHECK(svdlut_deterministic_workspace_size(INT32_MAX, 65535, 65535, 65535, 65535) > 0);
    CHECK(svdlut_deterministic_workspace_size(1, 0, 4, 4, 4) == 0);
    CHECK(svdlut_loss_workspace_size(-1) == 0 || svdlut_loss_workspace_size(-1) > 0);   // no UB either way
    CHECK(svdlut_loss_workspace_size(INT64_MAX / 8) > 0);
    CHECK(svdlut_generator_param_count(33, 8) > 0);
    CHECK(svdlut_paper_generator_param_count(33, 8, 6, 17) > 0);
    (void)svdlut_generator_workspace_size(INT32_MAX, 33, 8);
    (void)svdlut_paper_generator_workspace_size(INT32_MAX, 33, 8, 12, 33);
    (void)svdlut_unfused_workspace_size(INT32_MAX, 65535, 65535, 12, 33);
    (void)svdlut_lut3d_workspace_size(INT32_MAX, 40);
    CHECK(std::strlen(svdlut_version()) > 0);
}

static void deterministic_switch() {
    const int was = svdlut_get_deterministic();
    svdlut_set_deterministic(1);
    CHECK(svdlut_get_deterministic() == 1);
    void* f = reinterpret_cast<void*>(0x1000);
    const float* cf = static_cast<const float*>(f);
    float* ff = static_cast<float*>(f);
    refused(svdlut_apply_bwd(f, f, SVDLUT_F32, cf, cf, cf, f, SVDLUT_F32, nullptr, nullptr, nullptr, nullptr, ff,
                             nullptr, 2, 64, 64, 8, 8, 17, 4, nullptr, 0, nullptr), "deterministic");
    refused(svdlut_apply_bwd_noalloc(f, f, SVDLUT_F32, cf, cf, cf, f, SVDLUT_F32, nullptr, nullptr, nullptr, nullptr,
                                     ff, ff, 577, 4096, 4096, 4096, 4096, 33, 8, nullptr), "deterministic");
    svdlut_set_deterministic(was);
}

static void tune_cache() {
    using svdlut::TuneEntry;
    std::map<std::string, TuneEntry> m;
    CHECK(svdlut::parse_tune_cache("{\n  \"gfx950|a\": [512, 2],\n  \"gfx950|b\": [1024,1]\n}\n", m) == 2);
    CHECK(m["gfx950|a"].block == 512 && m["gfx950|a"].bpc == 2 && m["gfx950|a"].px == 4);
    // the third value: pixels per lane
    CHECK(svdlut::parse_tune_cache("{\"gfx950|c\": [256, 4, 8]}", m) == 1);
    CHECK(m["gfx950|c"].block == 256 && m["gfx950|c"].bpc == 4 && m["gfx950|c"].px == 8);
    // round trip
    std::map<std::string, TuneEntry> m2;
    CHECK(svdlut::parse_tune_cache(svdlut::format_tune_cache(m), m2) == 3);
    CHECK(m2.size() == 3 && m2["gfx950|b"].block == 1024 && m2["gfx950|c"].px == 8 && m2["gfx950|a"].px == 4);
    const char* bad[] = {"",
                         "{",
                         "\"",
                         "{\"k\"",
                         "{\"k\":",
                         "{\"k\": [",
                         "{\"k\": [512",
                         "{\"k\": [512,",
                         "{\"k\": [512, 2",
                         "{\"k\": [500, 2]}",
                         "{\"k\": [512, 0]}",
                         "{\"k\": [512, 33]}",
                         "{\"k\": [-512, 2]}",
                         "{\"k\": [99999999999999999999, 2]}",
                         "{\"k\": [512, 2.5]}",
                         "{\"k\": [\"512\", 2]}",
                         "{\"k\": {\"block\": 512}}",
                         "[512, 2]",
                         "\"k\" [512, 2]",
                         "{\"k\": [512 2]}",
                         "{\"k\": [512, 2, 6]}",
                         "{\"k\": [512, 2, 8, 1]}",
                         "{\"k\": [512, 2,]}",
                         "{\"k\": [512, 2, \"8\"]}",
                         "\xff\xfe\x00\x01"};
    for (const char* b : bad) {
        std::map<std::string, TuneEntry> mb;
        CHECK(svdlut::parse_tune_cache(std::string(b), mb) == 0);
        CHECK(mb.empty());
    }
    // a corrupt entry does not hide the valid ones around it
    std::map<std::string, TuneEntry> mc;
    CHECK(svdlut::parse_tune_cache("{\"a\": [512, 2], \"b\": [7, 7], \"c\": [64, 32]}", mc) == 2);
    CHECK(mc.count("a") == 1 && mc.count("b") == 0 && mc.count("c") == 1);
    // random bytes and random splices of a valid file: never out of bounds, entries valid
    const std::string good = svdlut::format_tune_cache(m);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    auto next = [&]() { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; };
    for (int it = 0; it < 20000; ++it) {
        std::string s;
        if (it & 1) {
            const size_t n = next() % 96;
            for (size_t i = 0; i < n; ++i) s.push_back(static_cast<char>(next() & 0xff));
        } else {
            s = good.substr(0, next() % (good.size() + 1));
            if (!s.empty()) s[next() % s.size()] = "\"[],:0123456789 -"[next() % 17];
        }
        std::map<std::string, TuneEntry> mr;
        svdlut::parse_tune_cache(s, mr);
        for (const auto& kv : mr) CHECK(svdlut::tune_entry_ok(kv.second));
    }
}

int main() {
    validation();
    size_queries();
    deterministic_switch();
    tune_cache();
    if (g_failed) {
        std::fprintf(stderr, "%d of %d checks failed\n", g_failed, g_checks);
        return 1;
    }
    std::printf("OK %d checks\n", g_checks);
    return 0;
}
