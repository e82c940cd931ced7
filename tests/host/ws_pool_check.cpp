// Host-only check of the two-pass workspace registry: a buffer handed out
// before (and so possibly captured into a graph) stays allocated when a later
// request on the same stream needs more, streams never share a buffer, and a
// request that would allocate under capture fails instead.
#include <cstdio>
#include <cstdlib>
#include <set>

#include "tfft_workspace.hpp"

namespace {
std::set<void*> g_live;   // buffers the fake allocator has handed out
int g_fail_next = 0;

struct FakeAlloc {
    bool operator()(void** p, size_t bytes) const {
        if (g_fail_next) { g_fail_next = 0; *p = nullptr; return false; }
        *p = std::malloc(bytes ? bytes : 1);
        g_live.insert(*p);
        return *p != nullptr;
    }
};

int g_errors = 0;
#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); ++g_errors; } \
    } while (0)
}  // namespace

int main() {
    using tfft::WsResult;
    tfft::WorkspacePool<FakeAlloc> pool{FakeAlloc{}};
    const void* s1 = reinterpret_cast<const void*>(0x1000);
    const void* s2 = reinterpret_cast<const void*>(0x2000);
    void* a = nullptr;
    void* b = nullptr;
    void* c = nullptr;

    // nothing reserved: a captured request fails, an eager one allocates
    CHECK(pool.get(0, s1, 64 << 10, false, &a) == WsResult::kWouldAllocate);
    CHECK(pool.get(0, s1, 64 << 10, true, &a) == WsResult::kOk && a);
    // a smaller or equal request reuses the buffer, also under capture
    CHECK(pool.get(0, s1, 32 << 10, false, &b) == WsResult::kOk && b == a);
    // a larger eager request gets a new buffer; the old one is retired, not freed
    CHECK(pool.get(0, s1, 1 << 20, true, &b) == WsResult::kOk && b != a);
    CHECK(pool.retired().size() == 1 && pool.retired()[0] == a);
    CHECK(g_live.count(a) == 1);
    CHECK(pool.bytes(0, s1) == (size_t)(1 << 20));
    // another stream has its own buffer
    CHECK(pool.get(0, s2, 64 << 10, true, &c) == WsResult::kOk && c != b && c != a);
    // another device too
    void* d = nullptr;
    CHECK(pool.get(1, s1, 64 << 10, true, &d) == WsResult::kOk && d != b);
    // a failed allocation leaves the current buffer in place
    g_fail_next = 1;
    void* e = nullptr;
    CHECK(pool.get(0, s1, 4 << 20, true, &e) == WsResult::kNoMemory);
    CHECK(pool.get(0, s1, 1 << 20, false, &e) == WsResult::kOk && e == b);
    std::printf("%s (%d errors)\n", g_errors ? "FAILED" : "ok", g_errors);
    return g_errors ? 1 : 0;
}
