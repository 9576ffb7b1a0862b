// Device primitives: device memory pool, exclusive scan of counts and a
// stable LSD radix sort (keys with 32-bit values), all written for wave64.
#include <algorithm>
#include <chrono>
#include <thread>

#include "em_internal.h"

namespace em {

// ---------------------------------------------------------------- workspace
Workspace::Workspace(int device) : device_(device), bufs_(S_NUM_SLOTS) {}

Workspace::~Workspace() { release(); }

void Workspace::use_arena(void *base, size_t bytes)
{
    release();
    arena_base_ = static_cast<char *>(base);
    arena_cap_ = bytes;
    arena_used_ = 0;
}

size_t Workspace::arena_free() const
{
    return arena_base_ ? arena_cap_ - arena_used_ : ~size_t(0);
}

void Workspace::release()
{
    if (arena_base_) {
        for (Buf &b : bufs_) b = Buf();
        arena_used_ = 0;
        held_.store(0);
        return;
    }
    for (Buf &b : bufs_)
        if (b.p) {
            if (stream_) (void)hipFreeAsync(b.p, stream_);
            else (void)hipFree(b.p);
            held_.fetch_sub(b.cap);
            b.p = nullptr;
            b.cap = 0;
        }
}

void Workspace::drop(int slot)
{
    if (arena_base_ || slot < 0 || slot >= (int)bufs_.size()) return;
    Buf &b = bufs_[slot];
    if (!b.p) return;
    if (stream_) (void)hipFreeAsync(b.p, stream_);
    else (void)hipFree(b.p);
    held_.fetch_sub(b.cap);
    b = Buf();
}

void *Workspace::get(int slot, size_t bytes)
{
    if (slot < 0 || slot >= (int)bufs_.size()) throw Error{MAP_EINVAL, "workspace slot out of range"};
    Buf &b = bufs_[slot];
    if (bytes == 0) bytes = 256;
    if (arena_base_) {
        if (b.cap >= bytes) return b.p;
        const size_t want = (bytes + 255) & ~size_t(255);
        if (want > arena_cap_ - arena_used_)
            throw Error{MAP_ENOMEM, "the fixed scratch buffer (" + std::to_string(arena_cap_ >> 20) +
                                        " MiB) is too small for this input: " + std::to_string(arena_used_ + want) +
                                        " bytes needed so far"};
        b.p = arena_base_ + arena_used_;
        b.cap = want;
        arena_used_ += want;
        held_.store(arena_used_);
        return b.p;
    }
    if (b.cap < bytes) {
        if (b.p) {
            if (stream_) EM_HIP(hipFreeAsync(b.p, stream_));
            else EM_HIP(hipFree(b.p));
        }
        held_.fetch_sub(b.cap);
        b.p = nullptr;
        b.cap = 0;
        // growth slack: a quarter, at most 256 MiB (buffers of tens of GB are not padded by a quarter)
        size_t want = bytes + std::min(bytes / 4, size_t(256) << 20) + 256;
        want = (want + 255) & ~size_t(255);
        hipError_t e = stream_ ? hipMallocAsync(&b.p, want, stream_) : hipMalloc(&b.p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            throw Error{MAP_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed"};
        }
        b.cap = want;
        held_.fetch_add(want);
    }
    return b.p;
}

size_t Workspace::bytes_held() const { return held_.load(); }

// ---------------------------------------------------------------- bounded stream waits
static thread_local double t_wait_limit_ms = 0.0;

void set_wait_limit_ms(double ms) { t_wait_limit_ms = ms > 0.0 ? ms : 0.0; }

void stream_sync(hipStream_t s)
{
    if (t_wait_limit_ms <= 0.0) {
        EM_HIP(hipStreamSynchronize(s));
        return;
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (int spin = 0;; spin++) {
        const hipError_t e = hipStreamQuery(s);
        if (e == hipSuccess) return;
        (void)hipGetLastError();  // a not-ready query is no error of the next call
        if (e != hipErrorNotReady)
            throw Error{MAP_EDEVICE, std::string("hipStreamQuery: ") + hipGetErrorString(e)};
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (ms > t_wait_limit_ms)
            throw Error{MAP_EDEVICE, std::string(kWaitLimitText) + " (" + std::to_string((long long)t_wait_limit_ms) +
                                         " ms)"};
        if (spin < 200) std::this_thread::yield();
        else std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

int device_cu_count()
{
    int dev = 0, cus = 0;
    EM_HIP(hipGetDevice(&dev));
    EM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return cus > 0 ? cus : 1;
}

// ---------------------------------------------------------------- fills
__global__ void k_iota_u32(uint32_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = (uint32_t)i;
}

__global__ void k_iota_i64(int64_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = i;
}

__global__ void k_zero_u64(uint64_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0;
}

__global__ void k_zero_u8(uint8_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

static int grid_for(int64_t n, int block, int cap = 65536)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

void fill_iota_u32(uint32_t *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    EM_HIP(hipGetLastError());
}

void fill_iota_i64(int64_t *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota_i64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    EM_HIP(hipGetLastError());
}

// Zero a buffer with a kernel (keeps the path free of memset nodes).
void fill_zero_bytes(void *p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return;
    size_t words = bytes / 8;
    if (words) hipLaunchKernelGGL(k_zero_u64, dim3(grid_for((int64_t)words, 256)), dim3(256), 0, s,
                                  static_cast<uint64_t *>(p), (int64_t)words);
    size_t tail = bytes - words * 8;
    if (tail) hipLaunchKernelGGL(k_zero_u8, dim3(1), dim3(64), 0, s, static_cast<uint8_t *>(p) + words * 8,
                                 (int64_t)tail);
    EM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- block scan helpers
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = SCAN_BLOCK * SCAN_ITEMS;

// exclusive scan of one value per thread across a 256-thread block (4 waves)
__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t *total)
{
    __shared__ int64_t wsum[SCAN_BLOCK / 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < SCAN_BLOCK / 64; w++) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    if (total) *total = all;
    return before + x - v;
}

__global__ void k_chunk_sums(const int64_t *in, int64_t n, int64_t *partial)
{
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++)
        if (base + k < n) s += in[base + k];
    int64_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// out[i+1] = prefix[block] + inclusive scan within the chunk; out[0] = 0
__global__ void k_chunk_scan(const int64_t *in, int64_t n, const int64_t *prefix, int64_t *out)
{
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int64_t ex = block_exclusive_scan(s, nullptr) + (prefix ? prefix[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        ex += v[k];
        if (base + k < n) out[base + k + 1] = ex;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}

static void scan_rec(int64_t *tmp, const int64_t *in, int64_t *out, int64_t n, hipStream_t s)
{
    int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(SCAN_BLOCK), 0, s, in, n, (const int64_t *)nullptr, out);
        EM_HIP(hipGetLastError());
        return;
    }
    int64_t *partial = tmp;
    int64_t *pscan = tmp + nb;
    int64_t *next = tmp + 2 * nb + 1;
    hipLaunchKernelGGL(k_chunk_sums, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, partial);
    EM_HIP(hipGetLastError());
    scan_rec(next, partial, pscan, nb, s);
    hipLaunchKernelGGL(k_chunk_scan, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, (const int64_t *)pscan, out);
    EM_HIP(hipGetLastError());
}

void scan_counts(Workspace &ws, const int64_t *in, int64_t *out, int64_t n, hipStream_t s)
{
    if (n <= 0) {
        fill_zero_bytes(out, sizeof(int64_t), s);
        return;
    }
    // scratch: sum over levels of (2 nb + 1)
    int64_t need = 0, m = n;
    while (m > SCAN_CHUNK) {
        int64_t nb = (m + SCAN_CHUNK - 1) / SCAN_CHUNK;
        need += 2 * nb + 1;
        m = nb;
    }
    int64_t *tmp = ws.get<int64_t>(S_SCAN_TMP, (size_t)need + 8);
    scan_rec(tmp, in, out, n, s);
}

// ---------------------------------------------------------------- radix sort
// LSD radix sort with digits of up to 10 bits: a key width of b bits takes
// ceil(b / 10) passes, the width split evenly between them (18-bit keys: two
// passes of 9 bits, so the result lands back in the input buffers).
constexpr int RS_BLOCK = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_MAX_BITS = 10;
constexpr int RS_MAX_BUCKETS = 1 << RS_MAX_BITS;

template <typename K>
__global__ void k_rs_hist(const K *keys, int64_t n, int shift, int rb, int64_t nblocks, int64_t *hist)
{
    __shared__ unsigned cnt[RS_MAX_BUCKETS];
    const int nb = 1 << rb;
    for (int t = threadIdx.x; t < nb; t += RS_BLOCK) cnt[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const unsigned mask = (unsigned)nb - 1u;
    for (int k = 0; k < RS_ITEMS; k++) {
        int64_t i = base + (int64_t)k * RS_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(unsigned)(keys[i] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nb; t += RS_BLOCK) hist[(int64_t)t * nblocks + blockIdx.x] = cnt[t];
}

// Stable scatter: items of a tile are taken in order, 256 at a time; the rank of
// an item among equal digits is (items of earlier chunks and blocks) + (equal
// digits in earlier waves of the chunk) + (equal digits in lower lanes).
template <typename K>
__global__ void k_rs_scatter(const K *keys, const uint32_t *vals, K *keys_out, uint32_t *vals_out, int64_t n,
                             int shift, int rb, int64_t nblocks, const int64_t *offsets)
{
    __shared__ int64_t run[RS_MAX_BUCKETS];
    __shared__ unsigned wcnt[RS_WAVES][RS_MAX_BUCKETS];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int nb = 1 << rb;
    const unsigned mask = (unsigned)nb - 1u;
    for (int q = t; q < nb; q += RS_BLOCK) {
        run[q] = offsets[(int64_t)q * nblocks + blockIdx.x];
        for (int w = 0; w < RS_WAVES; w++) wcnt[w][q] = 0;
    }
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_ITEMS; k++) {
        int64_t i = base + (int64_t)k * RS_BLOCK + t;
        bool valid = i < n;
        K key = valid ? keys[i] : K(0);
        uint32_t val = valid ? vals[i] : 0u;
        unsigned d = (unsigned)(key >> shift) & mask;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RS_MAX_BITS; b++) {
            if (b < rb) {
                unsigned long long bb = __ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? bb : ~bb;
            }
        }
        unsigned rank_in_wave = (unsigned)__popcll(peers & lt);
        if (valid && rank_in_wave == 0) wcnt[wave][d] = (unsigned)__popcll(peers);
        __syncthreads();
        if (valid) {
            int64_t dest = run[d] + rank_in_wave;
            for (int w = 0; w < wave; w++) dest += wcnt[w][d];
            keys_out[dest] = key;
            vals_out[dest] = val;
        }
        __syncthreads();
        for (int q = t; q < nb; q += RS_BLOCK) {
            unsigned add = 0;
            for (int w = 0; w < RS_WAVES; w++) {
                add += wcnt[w][q];
                wcnt[w][q] = 0;
            }
            run[q] += add;
        }
        __syncthreads();
    }
}

template <typename K>
static void radix_sort(Workspace &ws, K *keys, uint32_t *vals, K *keys2, uint32_t *vals2, int64_t n, int bits,
                       hipStream_t s)
{
    if (n <= 1 || bits <= 0) return;
    const int passes = (bits + RS_MAX_BITS - 1) / RS_MAX_BITS;
    const int rb = (bits + passes - 1) / passes;
    const int64_t nblocks = (n + RS_TILE - 1) / RS_TILE;
    int64_t *hist = ws.get<int64_t>(S_SORT_HIST, (size_t)(nblocks << rb) * 2 + 1);
    int64_t *offs = hist + (nblocks << rb);
    K *src_k = keys, *dst_k = keys2;
    uint32_t *src_v = vals, *dst_v = vals2;
    for (int p = 0; p < passes; p++) {
        const int shift = rb * p;
        hipLaunchKernelGGL(k_rs_hist<K>, dim3((unsigned)nblocks), dim3(RS_BLOCK), 0, s, src_k, n, shift, rb, nblocks,
                           hist);
        EM_HIP(hipGetLastError());
        scan_counts(ws, hist, offs, nblocks << rb, s);
        hipLaunchKernelGGL(k_rs_scatter<K>, dim3((unsigned)nblocks), dim3(RS_BLOCK), 0, s, src_k, src_v, dst_k,
                           dst_v, n, shift, rb, nblocks, (const int64_t *)offs);
        EM_HIP(hipGetLastError());
        std::swap(src_k, dst_k);
        std::swap(src_v, dst_v);
    }
    if (src_k != keys) {
        EM_HIP(hipMemcpyAsync(keys, src_k, sizeof(K) * n, hipMemcpyDeviceToDevice, s));
        EM_HIP(hipMemcpyAsync(vals, src_v, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
}

void radix_sort_u32(Workspace &ws, uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2, int64_t n,
                    int bits, hipStream_t s)
{
    radix_sort<uint32_t>(ws, keys, vals, keys2, vals2, n, bits, s);
}

void radix_sort_u64(Workspace &ws, uint64_t *keys, uint32_t *vals, uint64_t *keys2, uint32_t *vals2, int64_t n,
                    int bits, hipStream_t s)
{
    radix_sort<uint64_t>(ws, keys, vals, keys2, vals2, n, bits, s);
}

}  // namespace em
