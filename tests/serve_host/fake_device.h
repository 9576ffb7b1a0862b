#pragma once
#include <condition_variable>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace em {
struct FakeLog {
    std::mutex mu;
    std::vector<int> order;  // job tags in admission order
    int live = 0, max_live = 0;
    size_t bytes = 0, max_bytes = 0;
    int batches = 0, max_batch = 0;
    int stage_us = 200;
    int device_syncs = 0;                      // hipFree / hipHostFree calls (each waits for the device)
    std::vector<std::thread::id> device_threads;  // threads that ran stages or launches
    int64_t hang_n = -1;                       // a job of this many particles hangs its launch
    bool hang_released = false;
    std::condition_variable hang_cv;
    std::map<const void *, size_t> footprint_of;  // job state -> footprint while in flight
    void reset()
    {
        std::lock_guard<std::mutex> g(mu);
        order.clear();
        live = max_live = 0;
        bytes = max_bytes = 0;
        batches = max_batch = 0;
        device_syncs = 0;
        device_threads.clear();
        hang_n = -1;
        hang_released = false;
        footprint_of.clear();
    }
    void release_hang();
};
extern FakeLog g_log;
}  // namespace em
