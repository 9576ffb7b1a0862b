// map_particles_noalloc: the synchronous mapping with every intermediate
// buffer in one fixed device array (`scratch`), for callers that cannot
// allocate device memory (code under graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// `scratch` is a file-scope device array: each device the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never uses the array's name as an address (on the host it only stands for
// the symbol): at context creation, with the context's device current, the
// device address is looked up with hipGetSymbolAddress once per device and
// kept; the pipeline then works inside that address range through the
// workspace's arena mode, so no call below allocates or frees device memory.
// All calls on one device share its array: two calls that overlap in time on
// one device (from different contexts or threads) race and must not be made.
// Everything the pipeline needs zeroed is cleared by its own fill kernels at
// the start of each call.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "em_internal.h"
#include "em_runtime.h"

namespace em {

namespace {

constexpr int kMaxDevices = 64;

// 128 MiB: a mapping of about 10,000 box-clipped Voronoi cells and their
// particles (the 4,096-particle uniform case needs about 70 MB).
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_mu;
void *g_base[kMaxDevices] = {};

}  // namespace

void noalloc_attach(int device)
{
    EM_CHECK(device >= 0 && device < kMaxDevices, MAP_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_base[device]) return;
    void *p = nullptr;
    EM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    EM_CHECK(p != nullptr, MAP_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_base[device] = p;
}

static void *noalloc_base(int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return (device >= 0 && device < kMaxDevices) ? g_base[device] : nullptr;
}

}  // namespace em

using namespace em;

extern "C" int map_particles_noalloc(map_ctx *h, const map_particles_in *p, const map_cells_in *c, map_out *out)
{
    if (!h) return MAP_EINVAL;
    Ctx *C = reinterpret_cast<Ctx *>(h);
    std::lock_guard<std::mutex> guard(C->mu);
    try {
        EM_HIP(hipSetDevice(C->device));
        EM_CHECK(p && c && out, MAP_EINVAL, "null particle, cell or output descriptor");
        EM_CHECK(C->precision == MAP_FP64 || C->precision == MAP_MIXED, MAP_EINVAL,
                 "map_particles_noalloc runs at MAP_FP64 or MAP_MIXED");
        EM_CHECK(p->mem_kind == MAP_MEM_DEVICE && c->mem_kind == MAP_MEM_DEVICE && out->mem_kind == MAP_MEM_DEVICE,
                 MAP_EINVAL, "map_particles_noalloc takes device inputs and outputs only");
        check_host_args(p, c);
        // the parts of the footprint known before the pair search
        const double need = 80.0 * (double)c->n_face_verts + 88.0 * (double)c->n_cells + 64.0 * (double)p->n +
                            (double)(1 << 20);
        EM_CHECK(need <= (double)kNoallocScratchBytes, MAP_ENOMEM,
                 "input too large for the " + std::to_string(kNoallocScratchBytes >> 20) +
                     " MiB scratch of map_particles_noalloc (at least " + std::to_string((long long)need) +
                     " bytes needed); use map_particles");
        void *base = noalloc_base(C->device);
        EM_CHECK(base != nullptr, MAP_EDEVICE, "the scratch array of this device was not attached");
        Workspace ws(C->device);
        ws.use_arena(base, kNoallocScratchBytes);
        C->back.valid = false;
        run_mapping(*C, ws, p, c, out, C->precision, C->stream, true);
        // the pairs lived in the shared scratch: nothing is kept for map_back
        C->back.valid = false;
        C->err.clear();
        return MAP_OK;
    } catch (const Error &e) {
        C->back.valid = false;
        C->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        C->err = "host allocation failed";
        return MAP_ENOMEM;
    } catch (const std::exception &e) {
        C->err = e.what();
        return MAP_EDEVICE;
    }
}
