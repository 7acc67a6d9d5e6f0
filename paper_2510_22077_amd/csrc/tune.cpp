// Autotuner for the launch parameters of the hot kernels, measured on the problem at
// hand: the block count of the Krylov reductions, the block size of the stencil
// kernels, and where the batched triangular solves keep the subdomain solution (LDS
// or HBM).  Results can be cached in a text file keyed by device architecture,
// problem size and precision, one line per problem:
//   <arch> <N> <Np> <Nc> <precision> s<split primaries> <red_blocks> <stencil_block> <trsv_mode>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "internal.h"

namespace gp {
template <typename T>
void trsv_gather(gplmm_ctx* c, const int32_t* sub_ids_dev, int nsub, const T* vin, T* out_local);
template <typename T>
void trsv_split(gplmm_ctx* c, const T* vin, T* loc);
void dots2(gplmm_ctx* c, const double* V, int64_t ldv, int k, const double* y, int64_t n, double* a, double* b);
double update2(gplmm_ctx* c, double* V, int64_t ldv, int j, const double* t, const double* s, double sj,
               double ainv, double* w, int64_t n);
}

using namespace gp;

namespace {

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// median of `reps` timed runs of f (after one untimed run), in ms
template <typename F>
double time_ms(gplmm_ctx* c, F f, int reps = 5) {
    f();
    std::vector<float> t;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, c->stream);
        f();
        (void)hipEventRecord(e1, c->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        t.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

std::string key_of(const gplmm_ctx* c) {
    std::ostringstream k;
    k << arch_name() << " " << c->N << " " << c->Np << " " << c->Nc << " "
      << (c->opt.precision == GPLMM_FP32 ? "fp32" : "fp64") << " s" << c->splits.size();
    return k.str();
}

template <typename T>
double time_trsv(gplmm_ctx* c) {
    T* loc = (T*)c->d_local;
    const T* v = (const T*)c->d_pv;
    return time_ms(c, [&]() {
        trsv_gather<T>(c, c->d_sub_ids + c->Np, c->Nc, v, loc);
        if (c->splits.empty()) trsv_gather<T>(c, c->d_sub_ids, c->Np, v, loc);
        else trsv_split<T>(c, v, loc);
    });
}

template <typename T>
double time_xv(gplmm_ctx* c) {
    T* a = (T*)c->d_pv;
    T* b = a + c->N;
    T* y = b + c->N;
    return time_ms(c, [&]() { launch_xv<T>(c, b, y, a, c->stream); });
}

}  // namespace

extern "C" int gplmm_autotune(gplmm_ctx* c, const char* cache_path, gplmm_tuning* out) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    gplmm_tuning t;
    std::memset(&t, 0, sizeof(t));
    const std::string key = key_of(c);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            if (line.rfind(key + " ", 0) != 0) continue;
            std::istringstream ls(line.substr(key.size()));
            int rb = 0, sb = 0, tm = 0;
            if (ls >> rb >> sb >> tm && rb >= 64 && rb <= 2048 && (sb == 128 || sb == 256 || sb == 512) &&
                tm >= 0 && tm <= 2) {
                c->red_blocks = rb;
                c->stencil_block = sb;
                c->trsv_mode = tm;
                t.from_cache = 1;
            }
        }
    }
    if (!t.from_cache) {
        // Krylov reductions: one Arnoldi orthogonalisation step (both passes) against half a
        // restart cycle of basis vectors; the coefficients are zero, so the basis is unchanged
        const int k = std::max(1, std::min(c->opt.restart / 2, 64));
        std::vector<double> ha(k + 1), hb(k + 1), zc(k + 1, 0.0);
        double best = 1e300;
        int best_rb = c->red_blocks;
        for (int rb : {256, 512, 1024, 2048}) {
            c->red_blocks = rb;
            const double ms = time_ms(c, [&]() {
                dots2(c, c->d_V, c->N, k, c->d_V + (int64_t)k * c->N, c->N, ha.data(), hb.data());
                update2(c, c->d_V, c->N, k - 1, zc.data(), zc.data(), 0.0, 1.0, c->d_V + (int64_t)k * c->N, c->N);
            });
            if (ms < best) {
                best = ms;
                best_rb = rb;
            }
        }
        c->red_blocks = best_rb;
        t.t_reduction_ms = best;
        // stencil block size: the preconditioner's X v and the Newton J v
        best = 1e300;
        int best_sb = c->stencil_block;
        for (int sb : {128, 256, 512}) {
            c->stencil_block = sb;
            const double ms = (c->opt.precision == GPLMM_FP32 ? time_xv<float>(c) : time_xv<double>(c)) +
                              time_ms(c, [&]() { launch_jv(c, c->d_r, c->d_tmp, c->d_dx, c->stream); });
            if (ms < best) {
                best = ms;
                best_sb = sb;
            }
        }
        c->stencil_block = best_sb;
        t.t_stencil_ms = best;
        // triangular solves: solution in LDS or in HBM (needs the local factors)
        if (c->built) {
            best = 1e300;
            int best_tm = 0;
            for (int tm : {0, 1, 2}) {
                c->trsv_mode = tm;
                const double ms = c->opt.precision == GPLMM_FP32 ? time_trsv<float>(c) : time_trsv<double>(c);
                if (ms < best) {
                    best = ms;
                    best_tm = tm;
                }
            }
            c->trsv_mode = best_tm;
            t.t_trsv_ms = best;
        }
        GP_HIP(c, hipGetLastError());
        if (cache_path) {
            std::ofstream o(cache_path, std::ios::app);
            o << key << " " << c->red_blocks << " " << c->stencil_block << " " << c->trsv_mode << "\n";
        }
    }
    t.red_blocks = c->red_blocks;
    t.stencil_block = c->stencil_block;
    t.trsv_mode = c->trsv_mode;
    c->graph_valid = false;
    if (out) *out = t;
    return GPLMM_OK;
}

extern "C" int gplmm_set_tuning(gplmm_ctx* c, const gplmm_tuning* t) {
    if (!c || !t) return GPLMM_E_ARG;
    if (t->red_blocks < 64 || t->red_blocks > 2048 ||
        (t->stencil_block != 128 && t->stencil_block != 256 && t->stencil_block != 512) ||
        t->trsv_mode < 0 || t->trsv_mode > 2)
        return gp::fail(c, GPLMM_E_ARG, "tuning values out of range");
    c->red_blocks = t->red_blocks;
    c->stencil_block = t->stencil_block;
    c->trsv_mode = t->trsv_mode;
    c->graph_valid = false;   // the captured application holds the old launch shapes
    return GPLMM_OK;
}
