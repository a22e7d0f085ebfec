// Launch shapes of the bound kernels: get/set and the autotuner.
//
// The autotuner times every candidate (waves per block x grid size) of the
// GMM-GMM and GMM-vMF kernels on a seeded batch of random cubes of the
// problems currently set, with HIP events, and keeps the fastest of each.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gosma_impl.h"

extern "C" void gosma_drop_graph(gosma_ctx *ctx);   // bb.hip

namespace {

uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

uint64_t pack_key(int level, uint64_t x, uint64_t y, uint64_t z)
{
    return ((uint64_t)level << 57) | (x << 38) | (y << 19) | z;
}

// A random cell of the root box lo + [0, w] at a level in [lmin, lmax].
uint64_t random_key(uint64_t &s, int lmin, int lmax, uint64_t *idx, int *level)
{
    const int L = lmin + (int)(splitmix64(s) % (uint64_t)(lmax - lmin + 1));
    const uint64_t n = 1ull << L;
    for (int k = 0; k < 3; ++k) idx[k] = splitmix64(s) % n;
    *level = L;
    return pack_key(L, idx[0], idx[1], idx[2]);
}

bool valid_tile(const gosma_tile &t)
{
    return (t.waves == 1 || t.waves == 2 || t.waves == 4) && t.blocks >= 1;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

int fail(gosma_ctx *ctx, int code, const char *msg, hipError_t e = hipSuccess)
{
    ctx->err = std::string(msg) + (e ? std::string(": ") + hipGetErrorString(e) : std::string());
    return code;
}

}  // namespace

extern "C" {

int gosma_get_tiles(gosma_ctx *ctx, gosma_tiles *out)
{
    if (!ctx || !out) return GOSMA_E_INVAL;
    out->s11 = gosma_tile{ctx->tile11.waves, ctx->tile11.blocks};
    out->s12 = gosma_tile{ctx->tile12.waves, ctx->tile12.blocks};
    return GOSMA_OK;
}

int gosma_set_tiles(gosma_ctx *ctx, const gosma_tiles *tiles)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (!tiles || !valid_tile(tiles->s11) || !valid_tile(tiles->s12))
        return fail(ctx, GOSMA_E_INVAL, "tiles: waves must be 1, 2 or 4 and blocks >= 1");
    gosma_drop_graph(ctx);   // a captured iteration holds the old shapes
    ctx->tile11 = gosma::Tile{tiles->s11.waves, tiles->s11.blocks};
    ctx->tile12 = gosma::Tile{tiles->s12.waves, tiles->s12.blocks};
    for (int b = 0; b < gosma::kBuckets; ++b) {
        ctx->btile11[b] = ctx->tile11;
        ctx->btile12[b] = ctx->tile12;
    }
    return GOSMA_OK;
}

int gosma_get_bucket_tiles(gosma_ctx *ctx, int bucket, gosma_tiles *out, int *n_problems)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (!out || bucket < 0 || bucket >= gosma::kBuckets)
        return fail(ctx, GOSMA_E_INVAL, "bucket must be in [0, GOSMA_N_BUCKETS) and out not NULL");
    out->s11 = gosma_tile{ctx->btile11[bucket].waves, ctx->btile11[bucket].blocks};
    out->s12 = gosma_tile{ctx->btile12[bucket].waves, ctx->btile12[bucket].blocks};
    if (n_problems) *n_problems = ctx->bucket_nprob[bucket];
    return GOSMA_OK;
}

int gosma_autotune(gosma_ctx *ctx, int64_t n_cubes, uint64_t seed, double *rows, int64_t cap, int64_t *n_rows,
                   gosma_tiles *chosen)
{
    using namespace gosma;
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (ctx->n_problems < 1 || !ctx->has_domain) return fail(ctx, GOSMA_E_STATE, "autotune needs a problem set");
    if (n_cubes < 1 || n_cubes > (1 << 24)) return fail(ctx, GOSMA_E_INVAL, "autotune: 1 <= n_cubes <= 2^24");
    if (rows && cap < 0) return fail(ctx, GOSMA_E_INVAL, "autotune: cap must be >= 0");
    hipError_t e = hipSetDevice(ctx->device);
    if (e) return fail(ctx, GOSMA_E_HIP, "hipSetDevice", e);

    // problems drawn from: all of them (bucket -1), then each non-empty size bucket
    std::vector<int> groups{-1};
    for (int b = 0; b < kBuckets; ++b)
        if (ctx->bucket_nprob[b] > 0) groups.push_back(b);
    const int64_t n = n_cubes;
    DevBuf d_rk, d_tk, d_pid, d_s11u, d_s11l, d_ub, d_lb, d_fl, d_setup;
    if ((e = hipMalloc(&d_rk.p, 8 * n)) || (e = hipMalloc(&d_tk.p, 8 * n)) || (e = hipMalloc(&d_pid.p, 4 * n)) ||
        (e = hipMalloc(&d_s11u.p, 8 * n)) || (e = hipMalloc(&d_s11l.p, 8 * n)) || (e = hipMalloc(&d_ub.p, 8 * n)) ||
        (e = hipMalloc(&d_lb.p, 8 * n)) || (e = hipMalloc(&d_fl.p, n)) ||
        (e = hipMalloc(&d_setup.p, sizeof(CubeSetup) * n)))
        return fail(ctx, GOSMA_E_NOMEM, "autotune buffers", e);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if ((e = hipEventCreate(&ev0)) || (e = hipEventCreate(&ev1))) {
        if (ev0) (void)hipEventDestroy(ev0);
        return fail(ctx, GOSMA_E_HIP, "autotune events", e);
    }
    const DevMix mx = ctx->mix();
    const S11Out s11{(double *)d_s11u.p, (double *)d_s11l.p};
    BoundOut bo{(double *)d_ub.p, (double *)d_lb.p, nullptr, nullptr, (uint8_t *)d_fl.p, nullptr, nullptr, nullptr, 0, nullptr};
    const int waves_c[3] = {1, 2, 4};
    const int grid_c[5] = {2048, 4096, 8192, 16384, 32768};
    int64_t row = 0;
    uint64_t s = seed;
    Tile best_all[2] = {ctx->tile11, ctx->tile12};
    Tile best_b[kBuckets][2];
    for (int b = 0; b < kBuckets; ++b) {
        best_b[b][0] = ctx->btile11[b];
        best_b[b][1] = ctx->btile12[b];
    }
    std::vector<uint32_t> members;
    for (size_t gi = 0; gi < groups.size() && !e; ++gi) {
        const int grp = groups[gi];
        members.clear();
        for (int p = 0; p < ctx->n_problems; ++p)
            if (grp < 0 || ctx->h_prob[p].bucket == grp) members.push_back((uint32_t)p);
        const int gM = grp < 0 ? ctx->maxM : ctx->bucket_maxM[grp], gN = grp < 0 ? ctx->maxN : ctx->bucket_maxN[grp];
        // random cubes: problem uniform among the members, rotation cells that meet the radius-pi ball
        std::vector<uint64_t> rk(n), tk(n);
        std::vector<uint32_t> pid(n);
        for (int64_t c = 0; c < n; ++c) {
            const uint32_t p = members[splitmix64(s) % (uint64_t)members.size()];
            const ProbDesc &P = ctx->h_prob[p];
            uint64_t idx[3];
            int L = 0;
            uint64_t key = 0;
            for (int tries = 0; tries < 64; ++tries) {
                key = random_key(s, 2, 10, idx, &L);
                double nr2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double h = P.r_w[k] / (double)(1ull << L);
                    const double lo = P.r_lo[k] + (double)idx[k] * h, hi = lo + h;
                    const double nk = lo > 0.0 ? lo : (hi < 0.0 ? hi : 0.0);
                    nr2 += nk * nk;
                }
                if (nr2 <= M_PI * M_PI) break;
            }
            rk[c] = key;
            tk[c] = random_key(s, 1, 8, idx, &L);
            pid[c] = p;
        }
        if ((e = hipMemcpy(d_rk.p, rk.data(), 8 * n, hipMemcpyHostToDevice)) ||
            (e = hipMemcpy(d_tk.p, tk.data(), 8 * n, hipMemcpyHostToDevice)) ||
            (e = hipMemcpy(d_pid.p, pid.data(), 4 * n, hipMemcpyHostToDevice)))
            break;
        // for the search's shapes the GMM-GMM kernel is timed on an eighth as many
        // cells as cubes: the search evaluates it once per distinct translation
        // cell of an iteration (about one per four to eight children)
        const int64_t n11 = grp < 0 ? n : std::max<int64_t>(64, n / 8);
        auto run = [&](int kernel, Tile t) -> hipError_t {
            if (kernel == GOSMA_KERNEL_S11)
                return launch_s11(mx, (const uint64_t *)d_tk.p, (const uint32_t *)d_pid.p, n11, nullptr, s11, gM, t,
                                  nullptr);
            return launch_s12(mx, (const uint64_t *)d_rk.p, (const uint64_t *)d_tk.p, (const uint32_t *)d_pid.p,
                              nullptr, s11.ub, s11.lo, n, nullptr, 1, bo, 0.0, gM, gN, false, t, (CubeSetup *)d_setup.p,
                              nullptr);
        };
        Tile *best = grp < 0 ? best_all : best_b[grp];
        double best_ms[2] = {INFINITY, INFINITY};
        // S11 results of every cube feed the S12 launches; compute them once
        e = launch_s11(mx, (const uint64_t *)d_tk.p, (const uint32_t *)d_pid.p, n, nullptr, s11, gM, best[0], nullptr);
        for (int kernel = GOSMA_KERNEL_S11; kernel <= GOSMA_KERNEL_S12 && !e; ++kernel)
            for (int wi = 0; wi < 3 && !e; ++wi)
                for (int gj = 0; gj < 5 && !e; ++gj) {
                    const Tile t{waves_c[wi], grid_c[gj] / waves_c[wi]};
                    if ((e = run(kernel, t))) break;    // warm-up
                    if ((e = hipEventRecord(ev0, nullptr))) break;
                    for (int r = 0; r < 3 && !e; ++r) e = run(kernel, t);
                    if (e || (e = hipEventRecord(ev1, nullptr)) || (e = hipEventSynchronize(ev1))) break;
                    float ms = 0.0f;
                    if ((e = hipEventElapsedTime(&ms, ev0, ev1))) break;
                    const double per = ms / 3.0;
                    if (rows && row < cap) {
                        rows[5 * row + 0] = kernel;
                        rows[5 * row + 1] = t.waves;
                        rows[5 * row + 2] = t.blocks;
                        rows[5 * row + 3] = per;
                        rows[5 * row + 4] = grp;
                    }
                    ++row;
                    if (per < best_ms[kernel]) {
                        best_ms[kernel] = per;
                        best[kernel] = t;
                    }
                }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (!e) e = hipDeviceSynchronize();
    if (e) return fail(ctx, GOSMA_E_HIP, "autotune launches", e);
    gosma_drop_graph(ctx);
    ctx->tile11 = best_all[0];
    ctx->tile12 = best_all[1];
    for (int b = 0; b < kBuckets; ++b) {
        ctx->btile11[b] = best_b[b][0];
        ctx->btile12[b] = best_b[b][1];
    }
    if (n_rows) *n_rows = row;
    if (chosen) gosma_get_tiles(ctx, chosen);
    return GOSMA_OK;
}

}  // extern "C"
