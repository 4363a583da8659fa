// Layout selection by timing (the batched scheduling of the teaser scene and
// the patch-size study of Sec. 7.1): candidate layouts -- scatter strategy,
// patch target and one-workgroup-per-patch versus a persistent grid -- are
// built in turn, each is timed on the caller's data, and the fastest is kept.
// Results are cached per process by a fingerprint of the problem.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <mutex>
#include <string>
#include <tuple>

#include "mad_internal.hpp"

namespace mad {

struct TuneChoice {
    int scatter, faces, persistent, wg_waves;
};

static std::mutex g_tune_mu;
static std::map<std::string, TuneChoice> g_tune_cache;
static bool g_tune_file_read = false;

// The cache file named by MAD_TUNE_CACHE: one line per fingerprint, "<fingerprint> <scatter> <patch target>
// <persistent> <wg_waves>", appended as choices are made; read once per process (the last line of a
// fingerprint wins). Missing or unreadable files are ignored. Called with g_tune_mu held.
static void tune_file_load() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char* path = std::getenv("MAD_TUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string key;
        TuneChoice c{};
        if (in >> key >> c.scatter >> c.faces >> c.persistent >> c.wg_waves &&
            (c.scatter == MAD_SCATTER_PATCH || c.scatter == MAD_SCATTER_ATOMIC || c.scatter == MAD_SCATTER_COLOR) &&
            c.faces >= 1 &&
            c.faces <= (1 << 20) && c.persistent >= 0 && c.persistent <= 2 && (c.wg_waves == 4 || c.wg_waves == 8))
            g_tune_cache[key] = c;
    }
}

static void tune_file_append(const std::string& key, const TuneChoice& c) {
    const char* path = std::getenv("MAD_TUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    if (f) f << key << ' ' << c.scatter << ' ' << c.faces << ' ' << c.persistent << ' ' << c.wg_waves << '\n';
}

// problem identity: device, sizes, connectivity hash, terms, precision and mode
static std::string fingerprint(const mad_problem* p, uint32_t mode) {
    const mad_mesh& m = *p->mesh;
    uint64_t h = 1469598103934665603ull;   // FNV-1a over the triangle list and component offsets
    for (int32_t v : m.tris) {
        h ^= (uint32_t)v;
        h *= 1099511628211ull;
    }
    for (int64_t v : m.comp_off) {
        h ^= (uint64_t)v;
        h *= 1099511628211ull;
    }
    hipDeviceProp_t prop{};
    (void)hipGetDeviceProperties(&prop, p->device);
    std::string k = std::string(prop.gcnArchName) + "/" + std::to_string(p->n_cu) + "/" + std::to_string(m.nv) + "/" +
                    std::to_string(m.nt) + "/" + std::to_string(h) + "/" + std::to_string(p->d) + "/" +
                    std::to_string(p->prec) + "/" + std::to_string(mode);
    for (const auto& t : p->terms) k += "/" + std::to_string(t.kind);
    return k;
}

static const char* scatter_name(int sc) {
    return sc == MAD_SCATTER_PATCH ? "patch" : sc == MAD_SCATTER_ATOMIC ? "atomic" : "color";
}

static int time_layout(mad_problem* p, const double* x, uint32_t mode, double* energy, void* grad, void* hess,
                       int reps, hipStream_t s, double* ms_out) {
    hipEvent_t a, b;
    MAD_HIP_TRY(hipEventCreate(&a));
    MAD_HIP_TRY(hipEventCreate(&b));
    int rc = eval_problem(p, x, mode, energy, grad, hess, s);   // warm-up
    std::vector<float> t;
    for (int r = 0; rc == MAD_OK && r < reps; ++r) {
        float ms = 0.f;
        if (hipEventRecord(a, s) != hipSuccess) rc = fail(MAD_E_HIP, "hipEventRecord");
        if (rc == MAD_OK) rc = eval_problem(p, x, mode, energy, grad, hess, s);
        if (rc == MAD_OK && hipEventRecord(b, s) != hipSuccess) rc = fail(MAD_E_HIP, "hipEventRecord");
        if (rc == MAD_OK && hipEventSynchronize(b) != hipSuccess) rc = fail(MAD_E_HIP, "hipEventSynchronize");
        if (rc == MAD_OK && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = fail(MAD_E_HIP, "hipEventElapsedTime");
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != MAD_OK) return rc;
    std::sort(t.begin(), t.end());
    *ms_out = t.empty() ? 0.0 : t[t.size() / 2];
    return MAD_OK;
}

}  // namespace mad

using namespace mad;

extern "C" {

int32_t mad_problem_layout(const mad_problem* p, int32_t* scatter, int32_t* patch_faces, int32_t* persistent,
                           int32_t* n_patches, int32_t* wg_waves) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (!p->finalized) return fail(MAD_E_STATE, "not finalized");
    if (scatter) *scatter = p->scatter;
    if (patch_faces) *patch_faces = p->opt.patch_faces;
    if (persistent) *persistent = p->persistent;
    if (n_patches) *n_patches = p->patches.n;
    if (wg_waves) *wg_waves = p->wg_waves;
    return MAD_OK;
}

int32_t mad_problem_set_layout(mad_problem* p, int32_t scatter, int32_t patch_faces, int32_t persistent,
                               int32_t wg_waves, void* stream) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (!p->finalized) return fail(MAD_E_STATE, "not finalized");
    if (scatter != MAD_SCATTER_AUTO && scatter != MAD_SCATTER_ATOMIC && scatter != MAD_SCATTER_PATCH &&
        scatter != MAD_SCATTER_COLOR)
        return fail(MAD_E_INVALID_ARG, "bad scatter mode");
    if (patch_faces < 1 || patch_faces > (1 << 20)) return fail(MAD_E_INVALID_ARG, "bad patch_faces");
    if (persistent < 0 || persistent > 2) return fail(MAD_E_INVALID_ARG, "persistent must be 0, 1 or 2");
    if (wg_waves != 0 && wg_waves != 4 && wg_waves != 8) return fail(MAD_E_INVALID_ARG, "wg_waves must be 0, 4 or 8");
    if (scatter != MAD_SCATTER_PATCH && scatter != MAD_SCATTER_AUTO && persistent)
        return fail(MAD_E_UNSUPPORTED, "persistent needs the patch scatter");
    const int sc = scatter == MAD_SCATTER_AUTO ? MAD_SCATTER_PATCH : scatter;
    const int rc = build_layout(p, patch_faces, sc, persistent, (hipStream_t)stream, wg_waves);
    if (rc != MAD_OK) p->finalized = false;   // half-built layout: the problem cannot be evaluated
    return rc;
}

int32_t mad_problem_autotune(mad_problem* p, const double* x, uint32_t mode, double* energy, void* grad, void* hess,
                             int32_t reps, int32_t flags, void* stream) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (!p->finalized) return fail(MAD_E_STATE, "autotune before finalize");
    if (!x) return fail(MAD_E_INVALID_ARG, "x is NULL");
    if (mode & ~15u) return fail(MAD_E_INVALID_ARG, "unknown mode bits");
    if ((mode & MAD_ENERGY) && !energy) return fail(MAD_E_INVALID_ARG, "energy output is NULL");
    if ((mode & MAD_GRAD) && !grad) return fail(MAD_E_INVALID_ARG, "gradient output is NULL");
    if ((mode & MAD_HESS) && !hess) return fail(MAD_E_INVALID_ARG, "Hessian output is NULL");
    if ((mode & MAD_SPD) && !(mode & MAD_HESS)) return fail(MAD_E_INVALID_ARG, "MAD_SPD needs MAD_HESS");
    if (reps < 1 || reps > 1000) return fail(MAD_E_INVALID_ARG, "reps must be in [1, 1000]");
    if (flags & ~MAD_TUNE_FORCE) return fail(MAD_E_INVALID_ARG, "unknown autotune flags");
    hipStream_t s = (hipStream_t)stream;
    const std::string key = fingerprint(p, mode);
    if (!(flags & MAD_TUNE_FORCE)) {
        TuneChoice c{};
        bool hit = false;
        {
            std::lock_guard<std::mutex> g(g_tune_mu);
            tune_file_load();
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                c = it->second;
                hit = true;
            }
        }
        if (hit) {
            p->tune_report = "{\"cached\": true, \"candidates\": []}";
            if (c.scatter == p->scatter && c.faces == p->opt.patch_faces && c.persistent == p->persistent &&
                c.wg_waves == p->wg_waves)
                return MAD_OK;
            return mad_problem_set_layout(p, c.scatter, c.faces, c.persistent, c.wg_waves, stream);
        }
    }
    const bool prof = p->profiling;
    p->profiling = false;
    static const int kFaces[] = {128, 256, 512, 1024};
    std::vector<TuneChoice> cands;
    for (int w : {4, 8}) {
        if (w == 8 && p->prec != MAD_F32) continue;
        for (int f : kFaces)
            for (int pers = 0; pers < 2; ++pers) cands.push_back({MAD_SCATTER_PATCH, f, pers, w});
    }
    cands.push_back({MAD_SCATTER_ATOMIC, 512, 0, 4});
    cands.push_back({MAD_SCATTER_COLOR, 512, 0, 4});
    std::string rep = "{\"cached\": false, \"candidates\": [";
    double best = 1e300;
    TuneChoice bc = {p->scatter, p->opt.patch_faces, p->persistent, p->wg_waves};
    int rc = MAD_OK;
    for (size_t i = 0; rc == MAD_OK && i < cands.size(); ++i) {
        const TuneChoice& c = cands[i];
        rc = build_layout(p, c.faces, c.scatter, c.persistent, s, c.wg_waves);
        double ms = 0.0;
        if (rc == MAD_OK) rc = time_layout(p, x, mode, energy, grad, hess, reps, s, &ms);
        if (rc != MAD_OK) break;
        char buf[288];
        std::snprintf(buf, sizeof(buf),
                      "%s{\"scatter\": \"%s\", \"patch_faces\": %d, \"effective_faces\": %d, \"persistent\": %d, "
                      "\"wg_waves\": %d, \"n_patches\": %d, \"ms\": %.6f}",
                      i ? ", " : "", scatter_name(c.scatter), c.faces, p->opt.patch_faces,
                      c.persistent, p->wg_waves, p->patches.n, ms);
        rep += buf;
        if (ms < best) {
            best = ms;
            bc = {c.scatter, p->opt.patch_faces, c.persistent, p->wg_waves};
        }
    }
    p->profiling = prof;
    if (rc != MAD_OK) {
        p->finalized = false;   // the layout may be half built
        return rc;
    }
    char tail[192];
    std::snprintf(tail, sizeof(tail),
                  "], \"chosen\": {\"scatter\": \"%s\", \"patch_faces\": %d, \"persistent\": %d, \"wg_waves\": %d}}",
                  scatter_name(bc.scatter), bc.faces, bc.persistent, bc.wg_waves);
    p->tune_report = rep + tail;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = bc;
        tune_file_append(key, bc);
    }
    rc = build_layout(p, bc.faces, bc.scatter, bc.persistent, s, bc.wg_waves);
    if (rc != MAD_OK) p->finalized = false;
    return rc;
}

int32_t mad_problem_tune_report(const mad_problem* p, char* buf, int64_t cap, int64_t* len) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (len) *len = (int64_t)p->tune_report.size();
    if (buf && cap > 0) {
        const size_t n = std::min<size_t>((size_t)cap - 1, p->tune_report.size());
        std::memcpy(buf, p->tune_report.data(), n);
        buf[n] = '\0';
    }
    return MAD_OK;
}

}  // extern "C"
