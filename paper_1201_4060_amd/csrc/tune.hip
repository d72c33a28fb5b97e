// Autotuner of the evaluation knobs (binning tile, gather variant, item size, tiles per
// workgroup) and the table the evaluation and batch planner consult.
//
// Entries are keyed by (order, coefficient type, ncomp, density class), the
// density class being round(log2(P / (n0 n1 n2))): the best configuration of
// the gather depends on how many particles share a tile, not on n or P alone.
// bsi_tune times every candidate on uniform positions generated on the device
// and keeps the fastest; the table can be written to and read from a
// JSON-lines file.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"

namespace bsi {

namespace {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number `i` of the
// stream started at `seed`; uniform doubles from its top 53 bits.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_uniform_positions(uint64_t seed, long P, double L0, double L1, double L2, double* pos) {
    const long p = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (p >= P) return;
    const double L[3] = {L0, L1, L2};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        pos[3 * p + d] = L[d] * double(splitmix64(seed, uint64_t(3 * p + d)) >> 11) * 0x1.0p-53;
}

int density_class(const bsi_field* f, int64_t P) {
    const double cells = double(f->n[0]) * f->n[1] * f->n[2];
    const double r = std::log2(std::max<double>(double(P), 1.0) / cells);
    return int(std::lround(std::max(-40.0, std::min(10.0, r))));
}

bool tiled_supported_any(const bsi_field* f, int tile);

bsi_eval_config default_config(const bsi_field* f, int64_t P) {
    bsi_eval_config c{};
    c.block = 256;
    c.xcd_remap = 1;
    c.tiles_per_group = 2;
    const double dens = double(P) / (double(f->n[0]) * f->n[1] * f->n[2]);
    if (dens >= 1.0 / 64.0) {
        for (int T : {8, 4, 6, 12, 16})
            if (tiled_supported_any(f, T)) {
                c.sort_tile = T;
                c.variant = 0;
                return c;
            }
    }
    // below one particle per 8^3 cells the stencils of neighbouring particles
    // barely overlap; binning then still buys page locality on large grids,
    // which pays for its launches only from a few 10^4 particles on
    c.variant = 1;
    c.sort_tile = (dens >= 1.0 / 512.0 || P >= 32768) ? 8 : 0;
    return c;
}

// minimal reader of the flat JSON objects bsi_tune writes (integers and one
// number array)
bool json_int(const std::string& line, const char* key, long long* v) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = line.find(k);
    if (at == std::string::npos) return false;
    const char* s = line.c_str() + at + k.size();
    while (*s == ' ') ++s;
    char* end = nullptr;
    *v = std::strtoll(s, &end, 10);
    return end != s;
}

}  // namespace

size_t bin_bucket_count(const bsi_field* f, int tile);
bool tiled_supported(const bsi_field* f, int tile);

namespace {
bool tiled_supported_any(const bsi_field* f, int tile) { return tiled_supported(f, tile); }
}  // namespace

bsi_status lookup_config(bsi_ctx* ctx, const bsi_field* f, int64_t P, bsi_eval_config* out) {
    const int d = density_class(f, P);
    std::lock_guard<std::mutex> lk(ctx->mu);
    const auto key = std::make_tuple(f->N, int(f->desc.coef), f->C, d);
    auto it = ctx->tune_table.find(key);
    if (it != ctx->tune_table.end()) {
        *out = it->second;
        return BSI_OK;
    }
    int best = 3;  // accept neighbours up to two density classes away
    for (const auto& kv : ctx->tune_table) {
        if (std::get<0>(kv.first) != f->N || std::get<1>(kv.first) != int(f->desc.coef) ||
            std::get<2>(kv.first) != f->C)
            continue;
        const int dist = std::abs(std::get<3>(kv.first) - d);
        if (dist < best) {
            best = dist;
            *out = kv.second;
        }
    }
    if (best < 3) return BSI_OK;
    *out = default_config(f, P);
    return BSI_OK;
}

bsi_status eval_run(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                    const bsi_eval_config& cfg, hipStream_t s);

}  // namespace bsi

using namespace bsi;

extern "C" {

bsi_status bsi_tune(bsi_field* f, int64_t P, uint64_t seed, const char* db_path, bsi_eval_config* best,
                    double* best_us) {
    clear_error();
    BSI_CHECK(f != nullptr, BSI_E_INVAL, "field is NULL");
    BSI_CHECK(P > 0 && P < (int64_t(1) << 31), BSI_E_INVAL, "P must be in [1, 2^31)");
    bsi_ctx* ctx = f->ctx;
    BSI_HIP(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, nullptr);
    const size_t osz = f->desc.coef == BSI_F64 ? 8 : 4;
    double* pos = nullptr;
    void* u = nullptr;
    void* g = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bsi_status st = BSI_OK;
    auto fail = [&](bsi_status code, const std::string& msg) {
        if (st == BSI_OK) {
            set_error(msg);
            st = code;
        }
    };
    if (hipMalloc(&pos, 3 * size_t(P) * sizeof(double)) != hipSuccess ||
        hipMalloc(&u, size_t(P) * f->C * osz) != hipSuccess ||
        hipMalloc(&g, size_t(P) * f->C * 3 * osz) != hipSuccess) {
        (void)hipGetLastError();
        fail(BSI_E_NOMEM, "tuning buffers do not fit");
    }
    if (st == BSI_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
        (void)hipGetLastError();
        fail(BSI_E_DEVICE, "event creation failed");
    }
    const bool timing = ctx->timing;
    ctx->timing = false;
    bsi_eval_config best_cfg{};
    double best_t = 1e300;
    if (st == BSI_OK) {
        hipLaunchKernelGGL(k_uniform_positions, dim3(unsigned((P + 255) / 256)), dim3(256), 0, s, seed, long(P),
                           f->L[0], f->L[1], f->L[2], pos);
        std::vector<bsi_eval_config> cands;
        const int nmax = std::max(f->n[0], std::max(f->n[1], f->n[2]));
        const int tmin = (nmax + 255) / 256;
        // particles per 8^3 tile when spread evenly: four wavefronts per tile
        // are tried when a tile fills at least one of them
        const double per_tile8 = double(P) * 512.0 / (double(f->n[0]) * f->n[1] * f->n[2]);
        for (int T : {4, 6, 8, 12, 16}) {
            if (T < tmin || !tiled_supported(f, T)) continue;
            for (int ir : {2, 4, 8}) {
                for (int tb : {64, 256}) {
                    if (tb == 256 && (T != 8 || per_tile8 < 64.0)) continue;
                    bsi_eval_config c{};
                    c.sort_tile = T;
                    c.block = 256;
                    c.xcd_remap = 1;
                    c.variant = 0;
                    c.tiles_per_group = 2;
                    c.item_rounds = ir;
                    c.tile_block = T == 8 ? tb : 0;
                    cands.push_back(c);
                }
            }
        }
        for (int T : {0, 4, 8, 16, 32}) {
            if (T != 0 && T < tmin) continue;
            bsi_eval_config c{};
            c.sort_tile = T;
            c.block = 256;
            c.xcd_remap = 1;
            c.variant = 1;
            c.tiles_per_group = 1;
            cands.push_back(c);
        }
        for (const auto& c : cands) {
            if (eval_run(f, pos, P, u, g, c, s) != BSI_OK) {  // warm-up (also sizes the workspace)
                clear_error();
                continue;
            }
            float t[3];
            bool ok = true;
            for (int r = 0; r < 3 && ok; ++r) {
                ok = hipEventRecord(e0, s) == hipSuccess && eval_run(f, pos, P, u, g, c, s) == BSI_OK &&
                     hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&t[r], e0, e1) == hipSuccess;
            }
            if (!ok) {
                (void)hipGetLastError();
                fail(BSI_E_DEVICE, "timing of a tuning candidate failed");
                break;
            }
            std::sort(t, t + 3);
            const double us = 1000.0 * t[1];
            if (us < best_t) {
                best_t = us;
                best_cfg = c;
            }
        }
        if (st == BSI_OK && best_t >= 1e300) fail(BSI_E_UNSUPPORTED, "no candidate configuration ran");
    }
    ctx->timing = timing;
    if (hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        fail(BSI_E_DEVICE, "tuning run failed");
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (pos) (void)hipFree(pos);
    if (u) (void)hipFree(u);
    if (g) (void)hipFree(g);
    if (st != BSI_OK) return st;
    const int dcls = density_class(f, P);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->tune_table[std::make_tuple(f->N, int(f->desc.coef), f->C, dcls)] = best_cfg;
    }
    if (db_path) {
        FILE* fp = std::fopen(db_path, "a");
        BSI_CHECK(fp != nullptr, BSI_E_INVAL, std::string("cannot open tuning file ") + db_path);
        std::fprintf(fp,
                     "{\"order\":%d,\"coef\":%d,\"ncomp\":%d,\"density_class\":%d,\"n\":[%d,%d,%d],"
                     "\"P\":%lld,\"sort_tile\":%d,\"variant\":%d,\"tiles_per_group\":%d,\"block\":%d,"
                     "\"xcd_remap\":%d,\"tile_block\":%d,\"item_rounds\":%d,\"us\":%.3f}\n",
                     f->N, int(f->desc.coef), f->C, dcls, f->n[0], f->n[1], f->n[2], (long long)P,
                     best_cfg.sort_tile, best_cfg.variant, best_cfg.tiles_per_group, best_cfg.block,
                     best_cfg.xcd_remap, best_cfg.tile_block, best_cfg.item_rounds, best_t);
        std::fclose(fp);
    }
    if (best) *best = best_cfg;
    if (best_us) *best_us = best_t;
    return BSI_OK;
}

bsi_status bsi_ctx_load_tuning(bsi_ctx* ctx, const char* db_path) {
    clear_error();
    BSI_CHECK(ctx && db_path, BSI_E_INVAL, "NULL argument");
    std::ifstream in(db_path);
    BSI_CHECK(in.good(), BSI_E_INVAL, std::string("cannot open tuning file ") + db_path);
    std::string line;
    int lineno = 0;
    std::vector<std::pair<std::tuple<int, int, int, int>, bsi_eval_config>> rows;
    while (std::getline(in, line)) {
        ++lineno;
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        long long N, coef, C, d, T, var, tpg, blk, xcd;
        const bool ok = json_int(line, "order", &N) && json_int(line, "coef", &coef) &&
                        json_int(line, "ncomp", &C) && json_int(line, "density_class", &d) &&
                        json_int(line, "sort_tile", &T) && json_int(line, "variant", &var) &&
                        json_int(line, "tiles_per_group", &tpg) && json_int(line, "block", &blk) &&
                        json_int(line, "xcd_remap", &xcd);
        BSI_CHECK(ok, BSI_E_INVAL, std::string(db_path) + ":" + std::to_string(lineno) + ": malformed entry");
        long long tb = 0, ir = 0;  // absent in entries that predate the fields
        if (!json_int(line, "tile_block", &tb)) tb = 0;
        if (!json_int(line, "item_rounds", &ir)) ir = 0;
        BSI_CHECK(tb == 0 || tb == 64 || tb == 256, BSI_E_INVAL,
                  std::string(db_path) + ":" + std::to_string(lineno) + ": tile_block out of range");
        BSI_CHECK(ir >= 0 && ir <= 1024, BSI_E_INVAL,
                  std::string(db_path) + ":" + std::to_string(lineno) + ": item_rounds out of range");
        BSI_CHECK((N == 2 || N == 4 || N == 6) && coef >= 0 && coef <= 2 && (C == 1 || C == 3) && T >= 0 && T <= 1024 &&
                      (var == 0 || var == 1) && tpg >= 0 && tpg <= 64 && blk >= 64 && blk <= 256 &&
                      blk % 64 == 0,
                  BSI_E_INVAL, std::string(db_path) + ":" + std::to_string(lineno) + ": value out of range");
        bsi_eval_config c{};
        c.sort_tile = int(T);
        c.variant = int(var);
        c.tiles_per_group = int(tpg);
        c.block = int(blk);
        c.xcd_remap = int(xcd);
        c.tile_block = int(tb);
        c.item_rounds = int(ir);
        rows.push_back({std::make_tuple(int(N), int(coef), int(C), int(d)), c});
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto& r : rows) ctx->tune_table[r.first] = r.second;  // later lines win
    return BSI_OK;
}

bsi_status bsi_ctx_lookup_config(bsi_ctx* ctx, const bsi_field* f, int64_t P, bsi_eval_config* out) {
    clear_error();
    BSI_CHECK(ctx && f && out, BSI_E_INVAL, "NULL argument");
    BSI_CHECK(f->ctx == ctx, BSI_E_INVAL, "field belongs to another context");
    return lookup_config(ctx, f, P, out);
}

bsi_status bsi_fill_uniform_positions(bsi_ctx* ctx, uint64_t seed, int64_t P, const double* length,
                                      double* pos_dev, void* stream) {
    clear_error();
    BSI_CHECK(ctx && length && pos_dev, BSI_E_INVAL, "NULL argument");
    BSI_CHECK(P >= 0 && P < (int64_t(1) << 31), BSI_E_INVAL, "P must be in [0, 2^31)");
    if (P == 0) return BSI_OK;
    BSI_HIP(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_uniform_positions, dim3(unsigned((P + 255) / 256)), dim3(256), 0,
                       pick_stream(ctx, stream), seed, long(P), length[0], length[1], length[2], pos_dev);
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

}  // extern "C"
