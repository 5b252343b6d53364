// Autotuning table: the method that sr_autotune_closure / sr_autotune_mul /
// sr_batch_autotune measured fastest for an (architecture, operation, kind,
// size class), consulted by closure(), semiring_mul() and the batches before
// their built-in size rules.  A size class is the bit length of n - 1, i.e.
// the sizes (2^(c-1), 2^c]; an entry made at one size applies to its whole
// class.  The runtimes of the kernels do not depend on the matrix entries (no
// entry is ever skipped), so timing any input of the right shape is timing
// every input of it.  Entries are keyed by the device's architecture name
// (gfx950), so a table saved on one MI355X serves every other: JSON, one
// entry per line:
//
//   {"format": "libsemiring-autotune-1", "entries": [
//   {"arch": "gfx950", "op": 1, "kind": 2, "class": [11, 0, 0], "choice": 256},
//   ...
//   ]}
//
// op: 1 closure (class of D), 2 product (classes of R, K, N), 3 batch
// (classes of the largest D and of the graph count); choice: the flags
// (SR_CLOSURE_*, SR_BOOL_*; for big pivot blocks the block / 64 in bits
// 16..23) or a batch's update-tile code.
#include <hip/hip_runtime_api.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sr_internal.h"

namespace sr {
namespace {

using Key = std::tuple<std::string, int, int, int, int, int>;  // arch, op, kind, c0, c1, c2

std::mutex g_mu;
std::map<Key, unsigned> g_table;
std::vector<std::string> g_arch;  // per device index, filled on first use
std::once_flag g_autoload;

// Architecture name of the current device ("gfx950"; "" without a device).
std::string current_arch() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0) return std::string();
    {
        std::lock_guard<std::mutex> g(g_mu);
        if ((size_t)d < g_arch.size() && !g_arch[(size_t)d].empty()) return g_arch[(size_t)d];
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, d) != hipSuccess) return std::string();
    std::string a(prop.gcnArchName);
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a.resize(colon);
    std::lock_guard<std::mutex> g(g_mu);
    if (g_arch.size() <= (size_t)d) g_arch.resize((size_t)d + 1);
    g_arch[(size_t)d] = a;
    return a;
}

const char *autotune_file() {
    const char *v = getenv("SR_AUTOTUNE_FILE");
    return (v && *v) ? v : nullptr;
}

void autoload() {
    std::call_once(g_autoload, [] {
        if (const char *f = autotune_file()) (void)tuned_load(f);
    });
}

// Writes the table; the caller holds g_mu.
int save_locked(const char *path) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return -1;
    fprintf(f, "{\"format\": \"libsemiring-autotune-1\", \"entries\": [\n");
    size_t i = 0;
    for (const auto &kv : g_table) {
        const Key &k = kv.first;
        fprintf(f, "{\"arch\": \"%s\", \"op\": %d, \"kind\": %d, \"class\": [%d, %d, %d], "
                   "\"choice\": %u}%s\n",
                std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                std::get<4>(k), std::get<5>(k), kv.second, ++i < g_table.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path) != 0) return -1;
    return 0;
}

}  // namespace

int size_class(int64_t n) {
    int c = 0;
    for (int64_t v = n - 1; v > 0; v >>= 1) c++;
    return c;
}

unsigned tuned_get(int op, int kind, int64_t a, int64_t b, int64_t c) {
    autoload();
    const Key k{current_arch(), op, kind, size_class(a), size_class(b), size_class(c)};
    std::lock_guard<std::mutex> g(g_mu);
    const auto it = g_table.find(k);
    return it == g_table.end() ? 0u : it->second;
}

void tuned_set(int op, int kind, int64_t a, int64_t b, int64_t c, unsigned choice) {
    autoload();
    const Key k{current_arch(), op, kind, size_class(a), size_class(b), size_class(c)};
    std::lock_guard<std::mutex> g(g_mu);
    g_table[k] = choice;
    if (const char *f = autotune_file()) (void)save_locked(f);
}

void tuned_clear() {
    std::lock_guard<std::mutex> g(g_mu);
    g_table.clear();
}

int tuned_save(const char *path) {
    std::lock_guard<std::mutex> g(g_mu);
    return save_locked(path);
}

int tuned_load(const char *path) {
    FILE *f = fopen(path, "r");
    if (!f) return -1;
    std::vector<std::pair<Key, unsigned>> got;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        // {"arch": "<name>", "op": .., "kind": .., "class": [.., .., ..], "choice": ..}
        const char *a = strstr(line, "{\"arch\": \"");
        if (!a) continue;
        a += strlen("{\"arch\": \"");
        const char *q = strchr(a, '"');
        if (!q || q - a > 63) continue;
        int op = 0, kind = 0, c0 = 0, c1 = 0, c2 = 0;
        unsigned choice = 0;
        if (sscanf(q, "\", \"op\": %d, \"kind\": %d, \"class\": [%d, %d, %d], \"choice\": %u}",
                   &op, &kind, &c0, &c1, &c2, &choice) == 6)
            got.emplace_back(Key{std::string(a, (size_t)(q - a)), op, kind, c0, c1, c2}, choice);
    }
    fclose(f);
    std::lock_guard<std::mutex> g(g_mu);
    for (const auto &e : got) g_table[e.first] = e.second;
    return (int)got.size();
}

}  // namespace sr
