// Autotuning table: the method that sr_autotune_closure / sr_autotune_mul
// measured fastest for a (device, operation, kind, size class), consulted by
// closure() and semiring_mul() before their built-in size rules.  A size class
// is the bit length of n - 1, i.e. the sizes (2^(c-1), 2^c]; an entry made at
// one size applies to its whole class.  The runtimes of the kernels do not
// depend on the matrix entries (no entry is ever skipped), so timing any
// input of the right shape is timing every input of it.
#include <hip/hip_runtime_api.h>

#include <map>
#include <mutex>
#include <tuple>

#include "sr_internal.h"

namespace sr {
namespace {

using Key = std::tuple<int, int, int, int, int, int>;  // device, op, kind, c0, c1, c2

std::mutex g_mu;
std::map<Key, unsigned> g_table;

int current_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return -1;
    return d;
}

}  // namespace

int size_class(int64_t n) {
    int c = 0;
    for (int64_t v = n - 1; v > 0; v >>= 1) c++;
    return c;
}

unsigned tuned_get(int op, int kind, int64_t a, int64_t b, int64_t c) {
    const Key k{current_device(), op, kind, size_class(a), size_class(b), size_class(c)};
    std::lock_guard<std::mutex> g(g_mu);
    const auto it = g_table.find(k);
    return it == g_table.end() ? 0u : it->second;
}

void tuned_set(int op, int kind, int64_t a, int64_t b, int64_t c, unsigned choice) {
    const Key k{current_device(), op, kind, size_class(a), size_class(b), size_class(c)};
    std::lock_guard<std::mutex> g(g_mu);
    g_table[k] = choice;
}

void tuned_clear() {
    std::lock_guard<std::mutex> g(g_mu);
    g_table.clear();
}

}  // namespace sr
