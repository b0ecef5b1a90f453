// The allocation-free variant of sapq_dslash (sapq_dslash_noalloc): its two staging vectors
// (the operand and the result in the internal layout) live in a static device array of the
// library instead of the context's arena, so a caller that cannot allocate (graph capture, a
// serving loop) needs no buffer of its own beyond its input and output.
//
// The array is file-scope and has a fixed size; every GPU the library runs on holds its own
// copy until the process ends.  Its device address is taken once per device with
// hipGetSymbolAddress, with that device current, when a context is created there, and only
// that address is ever handed to a kernel.  Calls that overlap on one GPU share the array and
// race.
#include <mutex>

#include "sapq_impl.h"

namespace sapq {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void *g_scratch_dev[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

size_t noalloc_scratch_bytes() { return NOALLOC_SCRATCH_BYTES; }

// Device address of `scratch` on device `dev` (the current device): looked up on the first
// call for that device and kept.  SAPQ_EHIP if the runtime cannot give it.
int noalloc_scratch_init(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("device index beyond the allocation-free entry point's table");
        return SAPQ_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[dev]) return SAPQ_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        return SAPQ_EHIP;
    }
    g_scratch_dev[dev] = p;
    return SAPQ_OK;
}

static void *scratch_of(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[dev];
}

}  // namespace sapq

using namespace sapq;

extern "C" int sapq_dslash_noalloc(sapq_ctx *h, double *out, const double *in, int prec) {
    if (!h || !out || !in) { set_error("null argument"); return SAPQ_EINVAL; }
    Ctx *c = &h->c;
    if (prec != SAPQ_FP64 && prec != c->prm.prec_inner) { set_error("prec must be SAPQ_FP64 or the context's prec_inner"); return SAPQ_EINVAL; }
    if (out == in) { set_error("in and out may not alias"); return SAPQ_EINVAL; }
    const size_t vec = ((c->nvec * elem_bytes(prec)) + 255) & ~(size_t)255;
    if (2 * vec > NOALLOC_SCRATCH_BYTES) {
        set_error("sapq_dslash_noalloc: the lattice needs " + std::to_string(2 * vec) + " bytes of staging, beyond the " +
                  std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte static scratch");
        return SAPQ_ENOMEM;
    }
    if (!c->have_U || !c->have_F) { set_error("gauge field and clover field must be loaded first"); return SAPQ_ESTATE; }
    char *base = (char *)scratch_of(c->device);
    if (!base) { set_error("no static scratch address for the context's device"); return SAPQ_ESTATE; }
    void *a = base, *b = base + vec;
    launch_pack_spinor(c, prec, a, in, 1.0);
    launch_dslash(c, prec, b, a);
    launch_unpack_spinor(c, prec, out, b, 1.0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("sapq_dslash_noalloc: ") + hipGetErrorString(e));
        return SAPQ_EHIP;
    }
    return SAPQ_OK;
}
