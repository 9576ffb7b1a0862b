#pragma once
#include <map>
#include <mutex>
#include <vector>

namespace em {
struct FakeLog {
    std::mutex mu;
    std::vector<int> order;  // job tags in admission order
    int live = 0, max_live = 0;
    size_t bytes = 0, max_bytes = 0;
    int batches = 0, max_batch = 0;
    int stage_us = 200;
    std::map<const void *, size_t> footprint_of;  // job state -> footprint while in flight
    void reset()
    {
        std::lock_guard<std::mutex> g(mu);
        order.clear();
        live = max_live = 0;
        bytes = max_bytes = 0;
        batches = max_batch = 0;
    }
};
extern FakeLog g_log;
}  // namespace em
