// Host sanitizer run of the C ABI's host-side argument and file checks,
// linked against a copy of libcoremaint built with AddressSanitizer and
// UndefinedBehaviorSanitizer on its host code (tests/test_sanitize.py).
// Only paths that need no GPU run here: defaults, status texts, argument
// rejection on null handles, and snapshot parsing (good and corrupt files;
// a good file then fails at device set-up when no GPU is present, or is
// restored when one is).
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/coremaint.h"

static int fails = 0;
#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);      \
            ++fails;                                              \
        }                                                         \
    } while (0)

static void put(const char *path, const std::vector<unsigned char> &bytes) {
    FILE *f = std::fopen(path, "wb");
    if (f) {
        std::fwrite(bytes.data(), 1, bytes.size(), f);
        std::fclose(f);
    }
}

static std::vector<unsigned char> snapshot_bytes(int32_t n, int32_t alive, int64_t m, const std::vector<int32_t> &w,
                                                 bool good_sum) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (int32_t x : w) {
        h ^= (uint64_t)(uint32_t)x;
        h *= 0x100000001b3ull;
    }
    if (!good_sum) h ^= 1;
    std::vector<unsigned char> b(8 + 4 * 4 + 8 + 8 + 4 * w.size());
    std::memcpy(b.data(), "CMSNAP01", 8);
    int32_t hdr[4] = {1, n, alive, 0};
    std::memcpy(b.data() + 8, hdr, 16);
    std::memcpy(b.data() + 24, &m, 8);
    std::memcpy(b.data() + 32, &h, 8);
    std::memcpy(b.data() + 40, w.data(), 4 * w.size());
    return b;
}

int main(int argc, char **argv) {
    const char *dir = argc > 1 ? argv[1] : ".";
    cm_config cfg;
    cm_config_default(&cfg);
    CHECK(cfg.strict == 1 && cfg.mode == CM_MODE_PLAIN);
    for (int code = 1; code >= -15; --code) CHECK(cm_strerror(code) != nullptr);
    CHECK(cm_create(nullptr, nullptr) == CM_E_ARG);
    CHECK(cm_load_graph(nullptr, 0, 0, nullptr, nullptr, 0) == CM_E_ARG);
    CHECK(cm_insert_edges(nullptr, 0, nullptr, nullptr, 0, nullptr) == CM_E_ARG);
    CHECK(cm_update_edges_noalloc(nullptr, 0, 0, nullptr, nullptr, nullptr) == CM_E_ARG);
    CHECK(cm_snapshot(nullptr, "x") == CM_E_ARG);
    CHECK(cm_debug_log(nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0) == CM_E_ARG);
    CHECK(std::strcmp(cm_last_error(nullptr), "") == 0);
    cm_destroy(nullptr);
    // snapshot parsing: a triangle plus an isolated id
    const std::vector<int32_t> good = {2, 2, 2, 0, 2, 2, 2, 0, 0, 0, 1, 1, 2, 2};
    char path[4096];
    std::snprintf(path, sizeof(path), "%s/s.snap", dir);
    cm_graph *g = nullptr;
    CHECK(cm_restore(nullptr, path, &g) == CM_E_IO && g == nullptr);  // missing file
    put(path, snapshot_bytes(4, 4, 3, good, false));
    CHECK(cm_restore(nullptr, path, &g) == CM_E_IO && g == nullptr);  // checksum
    auto trunc = snapshot_bytes(4, 4, 3, good, true);
    trunc.resize(trunc.size() - 3);
    put(path, trunc);
    CHECK(cm_restore(nullptr, path, &g) == CM_E_IO && g == nullptr);  // truncated
    put(path, snapshot_bytes(4, 3, 3, good, true));
    CHECK(cm_restore(nullptr, path, &g) == CM_E_IO && g == nullptr);  // live count
    put(path, snapshot_bytes(4, 4, 3, good, true));
    const int rc = cm_restore(nullptr, path, &g);  // parses; then needs a device
    CHECK(rc == CM_OK || rc == CM_E_DEVICE);
    if (g) cm_destroy(g);
    std::printf(fails ? "abi: %d failures\n" : "abi: ok\n", fails);
    return fails ? 1 : 0;
}
