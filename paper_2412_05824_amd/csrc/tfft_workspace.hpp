// tfft_workspace.hpp -- the two-pass workspace registry (host code, no HIP).
//
// A length above the single-pass limit runs as a column pass that writes its
// intermediate into a workspace and a row pass that reads it back.  The
// library owns that workspace.  Rules kept here:
//   * one workspace per (device, stream): transforms running at the same time
//     on different streams never share an intermediate;
//   * grow only, never free while the library is loaded: a graph captured
//     from an earlier call keeps the buffer it was captured with, so a later,
//     larger eager request allocates a new buffer and retires the old one to
//     a list instead of freeing it (retired buffers are released with the
//     process);
//   * no allocation while the caller's stream is being captured: the request
//     fails with "would allocate" and the caller reserves beforehand.
// The allocator is a template parameter so the bookkeeping can be checked on
// the host with a fake allocator.
#pragma once

#include <cstddef>
#include <map>
#include <utility>
#include <vector>

namespace tfft {

enum class WsResult { kOk, kWouldAllocate, kNoMemory };

template <class Alloc> class WorkspacePool {
public:
    explicit WorkspacePool(Alloc alloc) : alloc_(alloc) {}

    // A buffer of at least `bytes` for (device, stream).  may_alloc false:
    // only an existing buffer may be returned.
    WsResult get(int device, const void* stream, size_t bytes, bool may_alloc, void** out) {
        Slot& s = cur_[std::make_pair(device, stream)];
        if (s.ptr && s.bytes >= bytes) {
            *out = s.ptr;
            return WsResult::kOk;
        }
        if (!may_alloc) return WsResult::kWouldAllocate;
        void* p = nullptr;
        if (!alloc_(&p, bytes) || !p) return WsResult::kNoMemory;
        if (s.ptr) retired_.push_back(s.ptr);   // a captured graph may still use it
        s.ptr = p;
        s.bytes = bytes;
        *out = p;
        return WsResult::kOk;
    }

    size_t bytes(int device, const void* stream) const {
        auto it = cur_.find(std::make_pair(device, stream));
        return it == cur_.end() ? 0 : it->second.bytes;
    }
    const std::vector<void*>& retired() const { return retired_; }

private:
    struct Slot {
        void* ptr = nullptr;
        size_t bytes = 0;
    };
    Alloc alloc_;
    std::map<std::pair<int, const void*>, Slot> cur_;
    std::vector<void*> retired_;
};

}  // namespace tfft
