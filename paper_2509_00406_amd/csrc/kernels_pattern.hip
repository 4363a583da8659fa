// Block sparsity pattern from topology, on the GPU (Sec. 6.1): enumerate the
// element-element couplings in parallel, prefix-sum the per-row counts into
// row offsets, then fill the columns.
//
// Every block row is owned by one 64-lane workgroup, which gathers the stencils
// of the elements incident to its vertex (from a vertex -> element incidence
// built by a count / scan / fill pass), sorts them and drops repeats; rows of
// any length (any vertex valence) are handled. The result is unique (sorted unique columns per row, diagonal always present),
// so the pattern is bit-exact regardless of the order in which atomics
// filled the incidence lists. Scans are exclusive three-phase scans
// (block sums, scan of block sums, block-local rescan) with int64 totals so
// int32 overflow is detected before the int32 row pointer is written.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mad_internal.hpp"

namespace mad {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

// ---- exclusive scan: out[i] = sum_{j<i} in[j], out[n] = total (int64) ---------------------------
template <typename TI>
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(const TI* in, int64_t n, int64_t* bsum) {
    __shared__ int64_t red[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int64_t acc = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < n) acc += (int64_t)in[i];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kScanThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// in-place exclusive scan of a thread-block-sized array in LDS; returns the block total
__device__ int64_t block_exclusive_scan(int64_t* s) {
    const int t = threadIdx.x;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int64_t v = (t >= off) ? s[t - off] : 0;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    const int64_t total = s[kScanThreads - 1];
    const int64_t incl = s[t];
    __syncthreads();
    s[t] = incl;   // inclusive
    __syncthreads();
    const int64_t excl = (t == 0) ? 0 : s[t - 1];
    __syncthreads();
    s[t] = excl;
    __syncthreads();
    return total;
}

// single workgroup: exclusive scan of the block sums, carrying across chunks of kScanThreads
__global__ __launch_bounds__(kScanThreads) void k_scan_bsum(int64_t* bsum, int64_t nb, int64_t* total_out) {
    __shared__ int64_t s[kScanThreads];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        s[threadIdx.x] = (i < nb) ? bsum[i] : 0;
        const int64_t tot = block_exclusive_scan(s);
        if (i < nb) bsum[i] = s[threadIdx.x] + carry;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total_out = carry;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_final(const TI* in, int64_t n, const int64_t* boff, TO* out,
                                                             const int64_t* total) {
    __shared__ int64_t s[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t acc = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        v[k] = (i < n) ? (int64_t)in[i] : 0;
        acc += v[k];
    }
    s[threadIdx.x] = acc;
    block_exclusive_scan(s);
    int64_t run = s[threadIdx.x] + boff[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        if (i < n) out[i] = (TO)run;
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (TO)(*total);
}

// ---- incidence -----------------------------------------------------------------------------------
struct TermTable {
    const int32_t* stencil[8];
    int64_t off[9];     // global element offsets
    int32_t ns[8];
    int32_t n_terms;
};

__global__ void k_count(const int32_t* stencil, int64_t n, int ns, int32_t* deg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * ns) atomicAdd(deg + stencil[i], 1);
}

__global__ void k_incidence(const int32_t* stencil, int64_t n, int ns, int64_t elem_off, const int32_t* vptr,
                            int32_t* cursor, int32_t* inc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * ns) {
        const int32_t v = stencil[i];
        const int32_t pos = atomicAdd(cursor + v, 1);
        inc[vptr[v] + pos] = (int32_t)(elem_off + i / ns);
    }
}

// Rows of any length. Row v's candidates are v itself and, for each element incident to v, its stencil
// vertices in a slot of kMaxStencil entries (shorter stencils padded with INT32_MAX): 1 + kMaxStencil * deg(v)
// values, padded to the next power of two. One 64-lane workgroup per row sorts them with a bitonic network
// (in LDS when they fit kRowLds entries, else in the row's own range of a global scratch buffer), then
// keeps the first of each run of equal values. Pass 0 writes the row's distinct count, pass 1 its columns.
constexpr int kMaxStencil = 4;
constexpr int kRowLds = 2048;
constexpr int kRowThreads = 64;

__host__ __device__ inline int32_t pow2_at_least(int32_t x) {
    int32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// candidates of row v, padded to a power of two; entries of rows longer than kRowLds go to global scratch
__global__ void k_row_size(const int32_t* vptr, int64_t nv, int32_t* long_size, int32_t* flags) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int32_t deg = vptr[v + 1] - vptr[v];
    if (deg > (1 << 27)) {   // the padded candidate count would pass 2^30
        atomicOr(flags, 1);
        long_size[v] = 0;
        return;
    }
    const int32_t p = pow2_at_least(1 + kMaxStencil * deg);
    long_size[v] = p > kRowLds ? p : 0;
}

// One row's candidates, sorted and de-duplicated by the 64 lanes of the workgroup. `buf` (P entries) is
// either the workgroup's LDS buffer or the row's range of global scratch: the caller passes one or the
// other from separate branches, so each inlined copy addresses a single memory space (LDS or global) and
// no generic (flat) pointer is formed.
__device__ __forceinline__ void row_sort_body(int32_t* buf, const TermTable& tt, int32_t v, const int32_t* vptr,
                                              const int32_t* inc, int32_t* cnt, const int32_t* rowptr,
                                              int32_t* colidx, int pass) {
    const int lane = (int)threadIdx.x;
    const int32_t k0 = vptr[v], n = 1 + kMaxStencil * (vptr[v + 1] - k0);
    const int32_t P = pow2_at_least(n);
    for (int32_t i = lane; i < P; i += kRowThreads) {
        int32_t c = INT32_MAX;
        if (i == 0) {
            c = v;
        } else if (i < n) {
            const int32_t a = (i - 1) % kMaxStencil;
            const int64_t g = inc[k0 + (i - 1) / kMaxStencil];
            int t = 0;
            while (t + 1 < tt.n_terms && g >= tt.off[t + 1]) ++t;
            const int ns = tt.ns[t];
            if (a < ns) c = tt.stencil[t][(g - tt.off[t]) * ns + a];
        }
        buf[i] = c;
    }
    __syncthreads();
    // bitonic sort, ascending
    for (int32_t size = 2; size <= P; size <<= 1)
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t i = lane; i < P / 2; i += kRowThreads) {
                const int32_t lo = 2 * stride * (i / stride) + (i & (stride - 1)), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int32_t a = buf[lo], b = buf[hi];
                if ((a > b) == up) {
                    buf[lo] = b;
                    buf[hi] = a;
                }
            }
            __syncthreads();
        }
    // first of each run of equal values, padding excluded; lane order keeps the columns sorted
    int32_t done = 0;
    for (int32_t base = 0; base < P; base += kRowThreads) {
        const int32_t i = base + lane;
        int32_t c = INT32_MAX;
        bool keep = false;
        if (i < P) {
            c = buf[i];
            const int32_t prev = buf[i > 0 ? i - 1 : 0];
            keep = c != INT32_MAX && (i == 0 || prev != c);
        }
        const uint64_t m = __ballot(keep);
        if (pass == 1 && keep) colidx[rowptr[v] + done + __popcll(m & ((1ull << lane) - 1ull))] = c;
        done += __popcll(m);
    }
    if (pass == 0 && lane == 0) cnt[v] = done;
}

__global__ __launch_bounds__(kRowThreads) void k_row_sort(TermTable tt, const int32_t* vptr, const int32_t* inc,
                                                          const int64_t* long_off, int32_t* long_buf, int32_t* cnt,
                                                          const int32_t* rowptr, int32_t* colidx, int pass) {
    __shared__ int32_t sbuf[kRowLds];
    const int32_t v = (int32_t)blockIdx.x;
    const int32_t P = pow2_at_least(1 + kMaxStencil * (vptr[v + 1] - vptr[v]));
    if (P <= kRowLds) row_sort_body(sbuf, tt, v, vptr, inc, cnt, rowptr, colidx, pass);
    else row_sort_body(long_buf + long_off[v], tt, v, vptr, inc, cnt, rowptr, colidx, pass);
}

__global__ void k_i64_to_i32(const int64_t* in, int32_t* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)in[i];
}

template <typename TI, typename TO>
static hipError_t scan_exclusive(const TI* in, int64_t n, TO* out, int64_t* d_tmp /* >= nb + 1 */, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, (n + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL((k_scan_sums<TI>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, d_tmp);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(kScanThreads), 0, s, d_tmp, nb, d_tmp + nb);
    hipLaunchKernelGGL((k_scan_final<TI, TO>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, d_tmp, out,
                       d_tmp + nb);
    return hipGetLastError();
}

static unsigned blocks_for(int64_t n, int threads) { return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads); }

int build_pattern_device(int64_t nv, const std::vector<PatternTerm>& terms, int32_t** rowptr_out,
                         int32_t** colidx_out, int64_t* nnzb_out, std::vector<void*>& owned, hipStream_t s) {
    if (terms.size() > 8) return fail(MAD_E_UNSUPPORTED, "at most 8 terms");
    int64_t slots_total = 0, elems_total = 0;
    TermTable tt{};
    tt.n_terms = (int32_t)terms.size();
    for (size_t t = 0; t < terms.size(); ++t) {
        tt.stencil[t] = terms[t].stencil;
        tt.ns[t] = terms[t].ns;
        tt.off[t] = elems_total;
        elems_total += terms[t].n;
        slots_total += terms[t].n * terms[t].ns;
    }
    tt.off[terms.size()] = elems_total;
    if (slots_total > INT32_MAX || elems_total > INT32_MAX || nv >= INT32_MAX)
        return fail(MAD_E_OVERFLOW, "stencil incidence exceeds int32");

    std::vector<void*> tmp;
    auto alloc = [&](void** p, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
        if (e == hipSuccess) tmp.push_back(*p);
        return e;
    };
    auto cleanup = [&]() {
        for (void* p : tmp) (void)hipFree(p);
        tmp.clear();
    };
    int32_t *deg = nullptr, *vptr = nullptr, *cursor = nullptr, *inc = nullptr, *cnt = nullptr, *flags = nullptr;
    int64_t *scan_tmp = nullptr, *rowptr64 = nullptr;
    const int64_t nb = (std::max<int64_t>(nv, 1) + kScanChunk) / kScanChunk + 2;
    hipError_t e = hipSuccess;
    if ((e = alloc((void**)&deg, sizeof(int32_t) * nv)) != hipSuccess ||
        (e = alloc((void**)&vptr, sizeof(int32_t) * (nv + 1))) != hipSuccess ||
        (e = alloc((void**)&cursor, sizeof(int32_t) * nv)) != hipSuccess ||
        (e = alloc((void**)&inc, sizeof(int32_t) * slots_total)) != hipSuccess ||
        (e = alloc((void**)&cnt, sizeof(int32_t) * nv)) != hipSuccess ||
        (e = alloc((void**)&flags, sizeof(int32_t) * 4)) != hipSuccess ||
        (e = alloc((void**)&scan_tmp, sizeof(int64_t) * (nb + 1))) != hipSuccess ||
        (e = alloc((void**)&rowptr64, sizeof(int64_t) * (nv + 1))) != hipSuccess) {
        cleanup();
        return fail(MAD_E_OOM, std::string("pattern scratch: ") + hipGetErrorString(e));
    }
#define PT_TRY(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            cleanup();                                                              \
            return fail(MAD_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
        }                                                                           \
    } while (0)
    PT_TRY(launch_fill(deg, nv, 4, s));
    PT_TRY(launch_fill(cursor, nv, 4, s));
    PT_TRY(launch_fill(flags, 4, 4, s));
    for (const auto& t : terms) {
        if (t.n == 0) continue;
        hipLaunchKernelGGL(k_count, dim3(blocks_for(t.n * t.ns, 256)), dim3(256), 0, s, t.stencil, t.n, t.ns, deg);
    }
    PT_TRY(hipGetLastError());
    PT_TRY((scan_exclusive<int32_t, int32_t>(deg, nv, vptr, scan_tmp, s)));
    for (size_t t = 0; t < terms.size(); ++t) {
        if (terms[t].n == 0) continue;
        hipLaunchKernelGGL(k_incidence, dim3(blocks_for(terms[t].n * terms[t].ns, 256)), dim3(256), 0, s,
                           terms[t].stencil, terms[t].n, terms[t].ns, tt.off[t], vptr, cursor, inc);
    }
    PT_TRY(hipGetLastError());
    // global scratch for rows whose candidates exceed the LDS buffer (high-valence vertices)
    hipLaunchKernelGGL(k_row_size, dim3(blocks_for(nv, 256)), dim3(256), 0, s, vptr, nv, cnt, flags);
    PT_TRY(hipGetLastError());
    PT_TRY((scan_exclusive<int32_t, int64_t>(cnt, nv, rowptr64, scan_tmp, s)));
    int64_t long_total = 0;
    int32_t hflag = 0;
    PT_TRY(hipMemcpyAsync(&long_total, rowptr64 + nv, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PT_TRY(hipMemcpyAsync(&hflag, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PT_TRY(hipStreamSynchronize(s));
    if (hflag != 0) {
        cleanup();
        return fail(MAD_E_OVERFLOW, "a vertex lies in more than 2^27 element stencils");
    }
    int64_t* long_off = nullptr;
    int32_t* long_buf = nullptr;
    if (long_total > 0) {
        if ((e = alloc((void**)&long_off, sizeof(int64_t) * (nv + 1))) != hipSuccess ||
            (e = alloc((void**)&long_buf, sizeof(int32_t) * (size_t)long_total)) != hipSuccess) {
            cleanup();
            return fail(MAD_E_OOM, std::string("pattern scratch: ") + hipGetErrorString(e));
        }
        PT_TRY(hipMemcpyAsync(long_off, rowptr64, sizeof(int64_t) * (nv + 1), hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(k_row_sort, dim3((unsigned)nv), dim3(kRowThreads), 0, s, tt, vptr, inc,
                       (const int64_t*)long_off, long_buf, cnt, (const int32_t*)nullptr, (int32_t*)nullptr, 0);
    PT_TRY(hipGetLastError());
    PT_TRY((scan_exclusive<int32_t, int64_t>(cnt, nv, rowptr64, scan_tmp, s)));
    int64_t total = 0;
    PT_TRY(hipMemcpyAsync(&total, rowptr64 + nv, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PT_TRY(hipStreamSynchronize(s));
    if (total > INT32_MAX) {
        cleanup();
        return fail(MAD_E_OVERFLOW, "block count exceeds int32");
    }
    int32_t *rowptr = nullptr, *colidx = nullptr;
    e = hipMalloc((void**)&rowptr, sizeof(int32_t) * (nv + 1));
    if (e == hipSuccess) {
        owned.push_back(rowptr);
        e = hipMalloc((void**)&colidx, sizeof(int32_t) * std::max<int64_t>(total, 1));
        if (e == hipSuccess) owned.push_back(colidx);
    }
    if (e != hipSuccess) {
        cleanup();
        return fail(MAD_E_OOM, "pattern arrays");
    }
    hipLaunchKernelGGL(k_i64_to_i32, dim3(blocks_for(nv + 1, 256)), dim3(256), 0, s, rowptr64, rowptr, nv + 1);
    hipLaunchKernelGGL(k_row_sort, dim3((unsigned)nv), dim3(kRowThreads), 0, s, tt, vptr, inc,
                       (const int64_t*)long_off, long_buf, cnt, (const int32_t*)rowptr, colidx, 1);
    PT_TRY(hipGetLastError());
    PT_TRY(hipStreamSynchronize(s));
#undef PT_TRY
    cleanup();
    *rowptr_out = rowptr;
    *colidx_out = colidx;
    *nnzb_out = total;
    return MAD_OK;
}

// slot of block (s, t) for every element: binary search of column v_t in row v_s
__global__ void k_slots(const int32_t* stencil, int64_t n, int ns, const int32_t* rowptr, const int32_t* colidx,
                        int32_t* slots, int32_t* flags) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    for (int a = 0; a < ns; ++a) {
        const int32_t r = stencil[e * ns + a];
        for (int b = 0; b < ns; ++b) {
            const int32_t c = stencil[e * ns + b];
            int32_t lo = rowptr[r], hi = rowptr[r + 1] - 1, found = -1;
            while (lo <= hi) {
                const int32_t mid = lo + (hi - lo) / 2;
                const int32_t m = colidx[mid];
                if (m == c) {
                    found = mid;
                    break;
                }
                if (m < c) lo = mid + 1;
                else hi = mid - 1;
            }
            if (found < 0) {
                atomicOr(flags + 1, kFlagSlotMissing);
                found = rowptr[r];
            }
            slots[(int64_t)(a * ns + b) * n + e] = found;
        }
    }
}

hipError_t launch_slots(const int32_t* stencil, int64_t n, int ns, const int32_t* rowptr, const int32_t* colidx,
                        int32_t* slots, int32_t* flags, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_slots, dim3(blocks_for(n, 256)), dim3(256), 0, s, stencil, n, ns, rowptr, colidx, slots,
                       flags);
    return hipGetLastError();
}

// ---- dynamic sparsity: blocks of new interaction pairs (Sec. 6.3, CSR update of the appendix) --------
// The update follows the appendix's count / prefix-sum / copy / insert structure with one change: the
// new columns of a row are sorted and merged with the old ones instead of appended in atomic order, so
// every row stays sorted (the layout, the FP64 redo and the callers binary-search rows) and the result is
// unique, bit for bit, whatever order the atomics ran in.

__device__ __forceinline__ bool has_block(const int32_t* rp, const int32_t* ci, int32_t r, int32_t c) {
    int32_t lo = rp[r], hi = rp[r + 1] - 1;
    while (lo <= hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        const int32_t m = ci[mid];
        if (m == c) return true;
        if (m < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return false;
}

// pass 0: count each pair's missing blocks per row; pass 1: write them into the row's candidate segment
__global__ void k_pair_blocks(const int32_t* pairs, int64_t n, int64_t nv, const int32_t* rp, const int32_t* ci,
                              int32_t* cnt, const int32_t* coff, int32_t* fill, int32_t* stage, int32_t* flags,
                              int pass) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
    if (a < 0 || b < 0 || a >= nv || b >= nv) {
        if (pass == 0) atomicOr(flags, 1);
        return;
    }
    if (a == b) return;
    const int32_t rs[2] = {a, b}, cs[2] = {b, a};
    for (int k = 0; k < 2; ++k) {
        if (has_block(rp, ci, rs[k], cs[k])) continue;
        if (pass == 0) atomicAdd(cnt + rs[k], 1);
        else stage[coff[rs[k]] + atomicAdd(fill + rs[k], 1)] = cs[k];
    }
}

// one lane per row: sort the row's candidate columns, drop repeats; new count and total row count
__global__ void k_row_unique(int64_t nv, const int32_t* rp, const int32_t* coff, int32_t* stage, int32_t* nnew,
                             int32_t* rowcnt) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nv) return;
    int32_t* v = stage + coff[r];
    const int32_t m = coff[r + 1] - coff[r];
    for (int32_t i = 1; i < m; ++i) {
        const int32_t x = v[i];
        int32_t j = i - 1;
        while (j >= 0 && v[j] > x) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = x;
    }
    int32_t k = 0;
    for (int32_t i = 0; i < m; ++i)
        if (i == 0 || v[i] != v[i - 1]) v[k++] = v[i];
    nnew[r] = k;
    rowcnt[r] = rp[r + 1] - rp[r] + k;
}

// Merge the old and the new columns into the new rows; old block j -> map[j]; the new blocks' indices are
// listed at extra[noff[r] ...]. One wave per kMergeRows consecutive rows. A row without new blocks (almost
// every row) only shifts, by noff[r] (the new blocks of the rows before it): the wave's lanes copy all such
// entries of its rows together, each lane finding its entry's row by a binary search over the wave's row
// starts in LDS, so reads and writes are coalesced. A row with new blocks is merged by its own lane.
constexpr int kMergeRows = 64, kMergeWaves = 4;
__global__ __launch_bounds__(64 * kMergeWaves) void k_row_merge(int64_t nv, const int32_t* rp, const int32_t* ci,
                                                                 const int32_t* coff, const int32_t* stage,
                                                                 const int32_t* nnew, const int64_t* rp_new,
                                                                 const int32_t* noff, int32_t* ci_new, int32_t* map,
                                                                 int32_t* extra) {
    __shared__ int32_t s_rp[kMergeWaves][kMergeRows + 1];
    __shared__ int32_t s_shift[kMergeWaves][kMergeRows];   // noff[r], or -1 for a row with new blocks
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = ((int64_t)blockIdx.x * kMergeWaves + w) * kMergeRows;
    if (r0 >= nv) return;   // wave-uniform
    const int nrows = (int)(nv - r0 < kMergeRows ? nv - r0 : kMergeRows);
    const int64_t r = r0 + lane;
    if (lane < nrows) {
        s_rp[w][lane] = rp[r];
        s_shift[w][lane] = nnew[r] == 0 ? noff[r] : -1;
    }
    if (lane == 0) s_rp[w][nrows] = rp[r0 + nrows];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int32_t lo = s_rp[w][0], hi = s_rp[w][nrows];
    for (int32_t i = lo + lane; i < hi; i += 64) {
        int a = 0, b = nrows;   // the last row start <= i: s_rp[a] <= i < s_rp[a + 1]
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if (s_rp[w][m] <= i) a = m;
            else b = m;
        }
        const int32_t sh = s_shift[w][a];
        if (sh >= 0) {
            map[i] = i + sh;
            ci_new[i + sh] = ci[i];
        }
    }
    if (lane < nrows && s_shift[w][lane] < 0) {
        int32_t i = s_rp[w][lane];
        const int32_t ie = s_rp[w][lane + 1];
        const int32_t* nv_ = stage + coff[r];
        const int32_t ne = nnew[r];
        int32_t j = 0;
        int32_t o = (int32_t)rp_new[r];
        int32_t x = noff[r];
        while (i < ie || j < ne) {
            if (j >= ne || (i < ie && ci[i] < nv_[j])) {
                map[i] = o;
                ci_new[o++] = ci[i++];
            } else {
                extra[x++] = o;
                ci_new[o++] = nv_[j++];
            }
        }
    }
}

__global__ void k_remap(int32_t* a, int64_t n, const int32_t* map) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = map[a[i]];
}

int insert_pairs_device(mad_problem* p, const int32_t* pairs, int64_t n, int64_t* n_added, hipStream_t s) {
    const int64_t nv = p->mesh->nv;
    DynBuffers& B = p->dyn;
    auto T = [&](hipError_t e) { return e; };
    MAD_HIP_TRY(launch_fill(B.cnt, nv + 1, 4, s));
    MAD_HIP_TRY(launch_fill(B.fill, nv + 1, 4, s));
    MAD_HIP_TRY(launch_fill(B.flags, 4, 4, s));
    if (n > 0)
        hipLaunchKernelGGL(k_pair_blocks, dim3(blocks_for(n, 256)), dim3(256), 0, s, pairs, n, nv, p->d_rowptr,
                           p->d_colidx, B.cnt, (const int32_t*)nullptr, B.fill, (int32_t*)nullptr, B.flags, 0);
    MAD_HIP_TRY(T(hipGetLastError()));
    MAD_HIP_TRY((scan_exclusive<int32_t, int32_t>(B.cnt, nv, B.coff, B.scan_tmp, s)));
    if (n > 0)
        hipLaunchKernelGGL(k_pair_blocks, dim3(blocks_for(n, 256)), dim3(256), 0, s, pairs, n, nv, p->d_rowptr,
                           p->d_colidx, B.cnt, (const int32_t*)B.coff, B.fill, B.stage, B.flags, 1);
    hipLaunchKernelGGL(k_row_unique, dim3(blocks_for(nv, 256)), dim3(256), 0, s, nv, p->d_rowptr,
                       (const int32_t*)B.coff, B.stage, B.nnew, B.rowcnt);
    MAD_HIP_TRY(T(hipGetLastError()));
    MAD_HIP_TRY((scan_exclusive<int32_t, int64_t>(B.rowcnt, nv, B.rp64, B.scan_tmp, s)));
    MAD_HIP_TRY((scan_exclusive<int32_t, int32_t>(B.nnew, nv, B.noff, B.scan_tmp, s)));
    int64_t total = 0;
    int32_t added = 0, hflags[4] = {0, 0, 0, 0};
    MAD_HIP_TRY(hipMemcpyAsync(&total, B.rp64 + nv, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MAD_HIP_TRY(hipMemcpyAsync(&added, B.noff + nv, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MAD_HIP_TRY(hipMemcpyAsync(hflags, B.flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
    MAD_HIP_TRY(hipStreamSynchronize(s));
    if (hflags[0] != 0) return fail(MAD_E_INVALID_ARG, "a pair names a vertex out of range");
    if (total > p->nnzb_cap) return fail(MAD_E_CAPACITY, "the new blocks exceed the reserve");
    // write the inactive buffer, then make it the active one
    hipLaunchKernelGGL(k_i64_to_i32, dim3(blocks_for(nv + 1, 256)), dim3(256), 0, s, B.rp64, p->d_rowptr_b, nv + 1);
    hipLaunchKernelGGL(k_row_merge, dim3(blocks_for(nv, kMergeRows * kMergeWaves)), dim3(64 * kMergeWaves), 0, s, nv,
                       p->d_rowptr, p->d_colidx,
                       (const int32_t*)B.coff, (const int32_t*)B.stage, (const int32_t*)B.nnew,
                       (const int64_t*)B.rp64, (const int32_t*)B.noff, p->d_colidx_b, B.map,
                       p->d_extra_blocks + p->n_extra);
    MAD_HIP_TRY(T(hipGetLastError()));
    // every stored block index of the layout (and the earlier extra blocks) follows its block
    auto remap = [&](int32_t* a, int64_t m) -> hipError_t {
        if (!a || m <= 0) return hipSuccess;
        hipLaunchKernelGGL(k_remap, dim3(blocks_for(m, 256)), dim3(256), 0, s, a, m, (const int32_t*)B.map);
        return hipGetLastError();
    };
    MAD_HIP_TRY(remap(p->d_extra_blocks, p->n_extra));
    MAD_HIP_TRY(remap(p->d_lb_gidx, p->n_lb));
    MAD_HIP_TRY(remap(p->d_lb_gidxT, p->n_lb));
    MAD_HIP_TRY(remap(p->d_gb_gidx, p->n_gb));
    MAD_HIP_TRY(remap(p->d_gb_gidxT, p->n_gb));
    MAD_HIP_TRY(remap(p->d_orphan_block, p->n_orphan_block));
    for (auto& t : p->terms) MAD_HIP_TRY(remap(t.d_slots, t.d_slots ? t.n * t.ns * t.ns : 0));
    MAD_HIP_TRY(hipStreamSynchronize(s));
    std::swap(p->d_rowptr, p->d_rowptr_b);
    std::swap(p->d_colidx, p->d_colidx_b);
    p->nnzb = total;
    p->n_extra += added;
    p->host_pattern_stale = true;
    if (n_added) *n_added = added;
    return MAD_OK;
}

}  // namespace mad
