// Estimates that allocate nothing: the whole workspace of one estimate
// (probe and Lanczos blocks, coefficients, reduction partials, results)
// lives in one static device array per GPU instead of buffers the context
// allocates, for callers that cannot call hipMalloc (code under stream
// capture, tight serving loops, harnesses that forbid allocation).
//
// The array is a file-scope __device__ variable.  Host code never passes its
// name to a kernel or a copy: the name is a host-side stand-in, not a device
// address.  Its address on each device comes from hipGetSymbolAddress, taken
// once per device (with that device current) when the first context on the
// device is created, and kept here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx_internal.h"
#include "vne.h"

namespace vne {
namespace rt {

static __device__ __align__(256) unsigned char scratch[VNE_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<unsigned char *> g_scratch_ptr;   // per device; nullptr until resolved

// Carves 256-byte aligned ranges out of the scratch array, in the order the
// buffers are asked for; counts what does not fit.
struct Carver {
    unsigned char *base;
    size_t used = 0, need = 0;
    void take(DevBuf *b, size_t bytes) {
        if (bytes == 0) bytes = 256;
        const size_t at = (need + 255) & ~(size_t)255;
        need = at + bytes;
        if (need <= VNE_NOALLOC_SCRATCH_BYTES) {
            b->p = base + at;
            b->bytes = bytes;
            used = need;
        } else {
            b->p = nullptr;
            b->bytes = 0;
        }
    }
};

}  // namespace

// Device address of the scratch array on `device` (the current device).
vne_status noalloc_attach(int device, std::string *err) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize(device + 1, nullptr);
    if (g_scratch_ptr[device]) return VNE_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return VNE_EDEVICE;
    }
    g_scratch_ptr[device] = (unsigned char *)ptr;
    return VNE_OK;
}

static unsigned char *scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (size_t)device < g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

}  // namespace rt
}  // namespace vne

using namespace vne;
using namespace vne::rt;

extern "C" vne_status vne_entropy_estimate_noalloc(vne_ctx *c, int32_t gid, const vne_probes *pr, int32_t k,
                                                   uint32_t mode, vne_result *out) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (!pr || !out) return fail(c, VNE_EINVAL, "NULL argument");
    if (!get_graph(c, gid)) return fail(c, VNE_EINVAL, "unknown graph id");
    if (k < 1 || k > kMaxSteps) return fail(c, VNE_EINVAL, "k_steps must be in [1, 128]");
    if (pr->m < 1) return fail(c, VNE_EINVAL, "probe count m must be >= 1");
    if (pr->kind != VNE_PROBE_RADEMACHER && pr->kind != VNE_PROBE_COLORING && pr->kind != VNE_PROBE_DENSE)
        return fail(c, VNE_ENOTSUP, "the allocation-free estimate takes RADEMACHER, COLORING or DENSE probes");
    VNE_TRY(check_mode(c, mode));
    HIP_TRY(c, hipSetDevice(c->device));
    unsigned char *base = scratch_of(c->device);
    if (!base) return fail(c, VNE_EDEVICE, "scratch array of the device not resolved");
    // the graph's device arrays were built at registration
    auto sit = c->sets.find(std::vector<int32_t>{gid});
    if (sit == c->sets.end()) return fail(c, VNE_EINVAL, "graph has no device arrays");
    GraphSet *set = sit->second.get();
    const bool fp64 = (mode & VNE_MODE_F64) != 0;
    const bool desing = (mode & VNE_MODE_DESING) != 0;
    if (desing && !set->zero_rowsum)
        return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs a matrix whose rows sum to zero (A 1 = 0)");
    const int m = pr->m;

    Plan p;
    VNE_TRY(plan_shape(c, set, &p, m, k, fp64, false));
    Carver cv{base};
    plan_buffers(set, &p, [&](DevBuf *b, size_t bytes) { cv.take(b, bytes); });
    // host colour / dense arrays are copied into the scratch array too
    const size_t es = fp64 ? 8 : 4;
    if (pr->kind == VNE_PROBE_COLORING && pr->location == VNE_HOST) cv.take(&p.colors, (size_t)set->n * 4);
    if (pr->kind == VNE_PROBE_DENSE && pr->location == VNE_HOST) cv.take(&p.dense, (size_t)set->n * m * es);
    if (cv.need > VNE_NOALLOC_SCRATCH_BYTES)
        return fail(c, VNE_ENOMEM, "workspace of " + std::to_string(cv.need) + " bytes exceeds the " +
                                       std::to_string((size_t)VNE_NOALLOC_SCRATCH_BYTES) +
                                       "-byte scratch array of the allocation-free estimate");
    // the array keeps the last call's contents: clear what must start at zero
    HIP_TRY(c, hipMemsetAsync(p.long_part.p, 0, p.long_part.bytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(p.seeds.p, 0, p.seeds.bytes, c->stream));
    p.h_graph_k = {k};
    p.h_graph_m = {m};
    ProbeSpec ps;
    int combine_kind = 0;
    VNE_TRY(make_probe_spec(c, set, &p, pr, m, fp64, &ps, &combine_kind));
    RunOpts o;
    o.collect = false;                   // no timing events
    o.direct = true;                     // no captured graph
    VNE_TRY(run_lanczos(c, set, &p, ps, desing, o));
    HIP_TRY(c, launch_combine_graphs((const double *)p.psi.p, p.m_pad, (const int32_t *)p.graph_m.p, 1,
                                     combine_kind, (double *)p.estimate.p, c->stream));
    // results straight into the caller's buffers (column c of alpha / beta at
    // c * k: the plan's layout for one graph)
    hipStream_t s = c->stream;
    int32_t fl = 0;
    HIP_TRY(c, hipMemcpyAsync(&out->estimate, p.estimate.p, 8, hipMemcpyDeviceToHost, s));
    if (out->quad) HIP_TRY(c, hipMemcpyAsync(out->quad, p.psi.p, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    if (out->norm2) HIP_TRY(c, hipMemcpyAsync(out->norm2, p.norm2.p, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    if (out->k_eff) HIP_TRY(c, hipMemcpyAsync(out->k_eff, p.k_eff.p, (size_t)m * 4, hipMemcpyDeviceToHost, s));
    if (out->alpha) HIP_TRY(c, hipMemcpyAsync(out->alpha, p.alpha.p, (size_t)m * k * 8, hipMemcpyDeviceToHost, s));
    if (out->beta) HIP_TRY(c, hipMemcpyAsync(out->beta, p.beta.p, (size_t)m * k * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(&fl, p.flags.p, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return check_flags(c, fl);
}
