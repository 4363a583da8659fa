// Allocation-free evaluation (mad_problem_eval_static): the evaluation of mad_problem_eval with every
// buffer that an evaluation writes and then reads back within itself -- per-patch energies, the
// per-component reduction, the persistent launch's queue head, the halo partials of shared entries,
// the FP64 redo queue, the vertex normals and the network outputs -- carved from one static device
// array instead of the problem's own buffers. The entry point calls no allocator, so it can run where
// allocation is not allowed (code under HIP graph capture, serving loops with a fixed memory budget).
//
// Each GPU holds its own copy of the array, at its own address, from the load of the library until the
// process ends. Every call on one GPU uses that GPU's copy: calls that overlap on one GPU (two streams,
// two threads) race on it and must be ordered by the caller.
#include <algorithm>
#include <mutex>
#include <string>

#include "mad_internal.hpp"

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

}  // namespace

// Host code must not pass this name to a kernel: on the host it is a stand-in, not a device address.
// The device address comes from hipGetSymbolAddress, once per device, below.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the device must be current); looked up once per
// device and kept.
int scratch_address(int dev, unsigned char** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return mad::fail(MAD_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return MAD_OK;
}

// Places the evaluation's buffers one after another (256-byte aligned) from `base`; with base NULL it
// only counts. Returns the bytes needed without the FP64 redo queue, which takes what is left (up to
// one entry per element).
size_t carve(const mad_problem* p, unsigned char* base, mad::EvalScratch& sc) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> unsigned char* {
        unsigned char* q = base ? base + off : nullptr;
        off += (std::max<size_t>(bytes, 16) + 255) & ~size_t(255);
        return q;
    };
    const size_t eb = p->prec == MAD_F32 ? 4 : 8;
    const size_t d = (size_t)p->d;
    const size_t np = (size_t)std::max(p->patches.n, 1);
    sc.partial = reinterpret_cast<double*>(
        take(sizeof(double) * std::max(np * std::max<size_t>(p->terms.size(), 1), (size_t)p->n_color_slots)));
    sc.comp_energy =
        reinterpret_cast<double*>(take(sizeof(double) * std::max<size_t>(p->patches.comp_patch_ptr.size(), 1)));
    sc.work_counter = reinterpret_cast<int32_t*>(take(16));
    sc.fb_count = reinterpret_cast<int32_t*>(take(16));
    if (p->scatter == MAD_SCATTER_PATCH) {
        sc.halo_g = take((size_t)p->n_halo_v * d * eb);
        sc.halo_h = take((size_t)p->n_halo_b * d * d * eb);
    }
    if (p->shell) sc.normals = reinterpret_cast<double*>(take(sizeof(double) * 3 * (size_t)p->mesh->nv));
    for (size_t ti = 0; ti < p->terms.size() && ti < 8; ++ti) {
        const mad::Term& t = p->terms[ti];
        if (t.kind != MAD_MLP) continue;
        sc.psi[ti] = reinterpret_cast<float*>(take(sizeof(float) * (size_t)mad::kPsi * (size_t)t.n));
        sc.xh[ti] = reinterpret_cast<float*>(take(sizeof(float) * 6 * (size_t)t.n));
    }
    return off;
}

}  // namespace

extern "C" int32_t mad_problem_eval_static(mad_problem* p, const double* x, uint32_t mode, double* energy,
                                           void* grad, void* hess, void* stream) {
    int rc = mad::check_eval_args(p, x, mode, energy, grad, hess);
    if (rc != MAD_OK) return rc;
    int dev = -1;
    MAD_HIP_TRY(hipGetDevice(&dev));
    if (dev != p->device)
        return mad::fail(MAD_E_INVALID_ARG, "the problem lives on device " + std::to_string(p->device) +
                                                ", the current device is " + std::to_string(dev));
    if (dev < 0 || dev >= kMaxDevices) return mad::fail(MAD_E_UNSUPPORTED, "device index beyond 63");
    mad::EvalScratch sc;
    const size_t need = carve(p, nullptr, sc);
    if (need > kStaticScratchBytes)
        return mad::fail(MAD_E_CAPACITY, "the evaluation needs " + std::to_string(need) +
                                             " bytes of scratch; the static scratch holds " +
                                             std::to_string(kStaticScratchBytes));
    unsigned char* base = nullptr;
    if ((rc = scratch_address(dev, &base)) != MAD_OK) return rc;
    sc = mad::EvalScratch{};
    carve(p, base, sc);
    if (p->scatter == MAD_SCATTER_PATCH && p->prec == MAD_F32) {
        int64_t total = 0;
        for (const auto& t : p->terms) total += t.n;
        const size_t room = (kStaticScratchBytes - need) / sizeof(uint32_t);
        sc.fb_cap = (int32_t)std::min<int64_t>(total, (int64_t)std::min<size_t>(room, INT32_MAX));
        sc.fb_list = reinterpret_cast<uint32_t*>(base + need);
    }
    // per-stage profiling creates HIP events on first use: not recorded here
    const bool prof = p->profiling;
    p->profiling = false;
    rc = mad::eval_problem(p, x, mode, energy, grad, hess, (hipStream_t)stream, nullptr, nullptr, &sc);
    p->profiling = prof;
    return rc;
}
