// svm_tune.cpp -- the shape autotuner of libsvmhip.so: launch shapes measured on the device
// per problem class and kept for the life of the process.  A class is the row layout, the
// kernel-value precision, whether values are all 1.0, whether shrinking is on, and the sizes
// n and d rounded up to powers of two.  The shapes tuned here (the SMO loop's workgroup
// count, a batched problem's team size) only change how work is spread: the selection is
// exact and f is updated row by row, so results are the same for every shape.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "svm_internal.h"

namespace svm {

namespace {

int log2_ceil(long long v) {
    int b = 0;
    while ((1ll << b) < v) ++b;
    return b;
}

using Key = std::tuple<int, int, int, int, int, int, int>;

struct TuneTable {
    std::mutex m;
    std::map<Key, int> shape;
};
TuneTable& table() {
    static TuneTable t;
    return t;
}

Key key_of(const TuneClass& c) {
    return Key(c.target, c.lay, c.kprec, c.pattern ? 1 : 0, c.shrink ? 1 : 0, log2_ceil(c.n), log2_ceil(c.d));
}

}  // namespace

int tuned_shape(const TuneClass& c) {
    TuneTable& t = table();
    std::lock_guard<std::mutex> lock(t.m);
    auto it = t.shape.find(key_of(c));
    return it == t.shape.end() ? 0 : it->second;
}

void set_tuned_shape(const TuneClass& c, int shape) {
    TuneTable& t = table();
    std::lock_guard<std::mutex> lock(t.m);
    t.shape[key_of(c)] = shape;
}

void clear_tuned_shapes() {
    TuneTable& t = table();
    std::lock_guard<std::mutex> lock(t.m);
    t.shape.clear();
}

}  // namespace svm
