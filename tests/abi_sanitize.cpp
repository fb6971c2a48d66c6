// Drives the host-side paths of libstagcg's C-ABI that run without a GPU (size and workspace queries, argument
// validation, the error strings, the tuning-table reader and writer), so that a build of the library with host
// -fsanitize=address,undefined checks the ABI glue (compiled and run by tests/test_sanitize_cpu.py). Exits
// non-zero when a call returns something other than documented.
#include <cstdio>
#include <cstring>
#include <string>

#include "../include/sp_api.h"

static int failures = 0;
#define CHECK(cond)                                                    \
    do {                                                               \
        if (!(cond)) {                                                 \
            std::printf("check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                \
        }                                                              \
    } while (0)

static sp_geom geom(int x, int y, int z, int t, int bc = 0) {
    sp_geom g;
    g.dims[0] = x; g.dims[1] = y; g.dims[2] = z; g.dims[3] = t;
    g.bc_t = bc;
    return g;
}

static void write_file(const char* path, const char* text) {
    FILE* f = std::fopen(path, "w");
    if (!f) return;
    std::fputs(text, f);
    std::fclose(f);
}

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    CHECK(sp_version() > 0);
    for (int c = -8; c <= 2; ++c) CHECK(sp_strerror(c) != nullptr && std::strlen(sp_strerror(c)) > 0);
    CHECK(sp_last_error() != nullptr);

    // sizes
    sp_geom g = geom(20, 20, 20, 64);
    CHECK(sp_gauge_bytes(&g, SP_F32, 12) == 8ull * 256000 * 48);
    CHECK(sp_gauge_bytes(&g, SP_I16, 12) == 8ull * 256000 * 24);
    CHECK(sp_gauge_bytes(&g, SP_F64, 12) == 0);
    CHECK(sp_gauge_bytes(&g, 9, 18) == 0);
    CHECK(sp_vec_bytes(&g, SP_F16) == 256000ull * 16);
    CHECK(sp_vec_bytes(&g, SP_I16) == 0);
    CHECK(sp_gauge_bytes(nullptr, SP_F32, 18) == 0);
    const sp_geom bad[] = {geom(3, 4, 4, 4), geom(4, 4, 4, 0), geom(4, -2, 4, 4), geom(4, 4, 4, 4, 2),
                           geom(512, 512, 512, 512)};
    for (const sp_geom& b : bad) {
        CHECK(sp_vec_bytes(&b, SP_F32) == 0);
        CHECK(sp_force_workspace_bytes(&b) == 0);
        CHECK(sp_hyp_workspace_bytes(&b) == 0);
        CHECK(sp_npr_path_bytes(&b) == 0);
    }
    CHECK(sp_force_workspace_bytes(&g) > 0);
    CHECK(sp_hyp_workspace_bytes(&g) > 0 && sp_npr_path_bytes(&g) == 32000ull * 256 * 144);

    // workspace layout over one and many systems (the pointers are never dereferenced by the query)
    sp_gauge U;
    U.f64 = (const void*)0x1000;
    U.lo = (const void*)0x2000;
    U.lo_prec = SP_F32;
    U.recon = 12;
    sp_cg_params prm;
    std::memset(&prm, 0, sizeof prm);
    prm.tol = 1e-8;
    prm.max_iter = 100;
    prm.inner = SP_F32;
    prm.delta = 0.1;
    sp_system sys[9];
    sp_geom gs[3] = {geom(8, 8, 8, 8), geom(12, 12, 12, 24), geom(4, 4, 4, 4, 1)};
    for (int i = 0; i < 9; ++i) {
        sys[i].g = &gs[i % 3];
        sys[i].U = &U;
        sys[i].mass = 0.1;
        sys[i].b_e = nullptr;
        sys[i].x_e = nullptr;
    }
    const size_t w1 = sp_cg_workspace_bytes(1, sys, &prm);
    const size_t w9 = sp_cg_workspace_bytes(9, sys, &prm);
    CHECK(w1 > 0 && w9 > w1);
    CHECK(sp_cg_workspace_bytes(0, sys, &prm) == 0);
    CHECK(sp_cg_workspace_bytes(1, sys, nullptr) == 0);
    sp_cg_params bad_inner = prm;
    bad_inner.inner = SP_I16;  // a link storage, not an iteration precision
    CHECK(sp_cg_workspace_bytes(1, sys, &bad_inner) == 0);
    CHECK(sp_full_workspace_bytes(&gs[0], &U, &prm) > 0);

    // solves refused before any device work
    sp_cg_stats st;
    double* fake = (double*)0x3000;
    CHECK(sp_cg_solve(&gs[0], &U, 0.1, fake, fake, nullptr, &st, (void*)0x4000, w1, nullptr) == SP_ERR_INVALID_ARG);
    sp_cg_params neg = prm;
    neg.tol = -1;
    CHECK(sp_cg_solve(&gs[0], &U, 0.1, fake, fake, &neg, &st, (void*)0x4000, w1, nullptr) == SP_ERR_INVALID_ARG);
    neg = prm;
    neg.max_iter = 0;
    CHECK(sp_cg_solve(&gs[0], &U, 0.1, fake, fake, &neg, &st, (void*)0x4000, w1, nullptr) == SP_ERR_INVALID_ARG);
    CHECK(sp_cg_solve(&gs[0], &U, 0.1, fake, fake, &prm, &st, nullptr, w1, nullptr) == SP_ERR_WORKSPACE);
    CHECK(sp_cg_solve(&gs[0], &U, 0.1, fake, fake, &prm, &st, (void*)0x4000, w1 - 1, nullptr) == SP_ERR_WORKSPACE);
    CHECK(sp_cg_solve(&gs[0], &U, 0.1, nullptr, fake, &prm, &st, (void*)0x4000, w1, nullptr) == SP_ERR_INVALID_ARG);
    sp_gauge U16 = U;
    U16.lo_prec = SP_F16;
    sp_cg_params bf = prm;
    bf.inner = SP_BF16;  // FP16 links cannot serve BF16 vectors
    CHECK(sp_cg_solve(&gs[0], &U16, 0.1, fake, fake, &bf, &st, (void*)0x4000, w1, nullptr) == SP_ERR_UNSUPPORTED);
    CHECK(sp_cg_solve_batched(0, sys, &prm, nullptr, (void*)0x4000, w9, nullptr) == SP_ERR_INVALID_ARG);
    CHECK(sp_full_solve(&gs[0], &U, 0.0, fake, fake, &prm, &st, (void*)0x4000, 1ull << 30, nullptr) ==
          SP_ERR_INVALID_ARG);
    CHECK(std::strlen(sp_last_error()) > 0);

    // the allocation-free gradient refuses a lattice beyond its fixed array before anything is enqueued
    sp_geom big = geom(28, 28, 28, 96);
    CHECK(sp_cg_force_noalloc(&big, &U, 0.1, fake, fake, fake, nullptr, nullptr, nullptr) == SP_ERR_WORKSPACE);
    CHECK(sp_cg_force_noalloc(&gs[0], nullptr, 0.1, fake, fake, fake, nullptr, nullptr, nullptr) == SP_ERR_INVALID_ARG);

    // shards and the probe's sizes
    sp_shard sh;
    sh.local = geom(20, 20, 20, 8, 1);
    sh.t0 = 24;
    sh.T = 64;
    CHECK(sp_shard_face_bytes(&sh, SP_F32) == 4000ull * 24);
    CHECK(sp_shard_vec_bytes(&sh, SP_F16) == (32000ull + 8000) * 16);
    CHECK(sp_shard_ghost_bytes(&sh, SP_I16, 12) == 8000ull * 24);
    sh.t0 = 25;
    CHECK(sp_shard_face_bytes(&sh, SP_F32) == 0);
    sh.t0 = 60;
    CHECK(sp_shard_vec_bytes(&sh, SP_F32) == 0);
    CHECK(sp_face_pack(nullptr, SP_F32, fake, 0, fake, nullptr) == SP_ERR_INVALID_ARG);
    CHECK(sp_stream_out_bytes(1 << 20, 4) == ((1u << 20) / 1024) * 4);
    CHECK(sp_stream_out_bytes(1 << 20, 3) == 0);
    CHECK(sp_stream_probe(5, 1, fake, fake, nullptr, 16, nullptr) == SP_ERR_INVALID_ARG);

    // the tuning table: a round trip, then malformed files that must leave the table unchanged
    const std::string good = dir + "/good.json", out = dir + "/out.json", badf = dir + "/bad.json";
    write_file(good.c_str(), "{\n  \"8x8x8x8/l1/r12/v1\": {\"nt\": 128, \"remap\": 1, \"stream\": 1},\n"
                             "  \"8x8x8x8/l1/r12/v1/n4\": {\"nt\": 64, \"remap\": 0}\n}\n");
    CHECK(sp_tune_load(good.c_str()) == SP_OK);
    CHECK(sp_tune_save(out.c_str()) == SP_OK);
    const char* malformed[] = {
        "{\n  \"6x6x6x6/l1/r12/v1\": {\"nt\": 128, \"remap\": 1",  // cut off
        "{\"6x6x6x6/l1/r12/v1\": {\"nt\": 96, \"remap\": 1}}",       // bad block size
        "{\"6x6x6x6/l1/r12/v1\": {\"nt\": 64, \"remap\": 1, \"strm\": 1}}",
        "{\"6x6x6x6/l1/r12/v1\": {\"nt\": 64}}",
        "{\"6x6x6x6",
        "\"",
    };
    for (const char* m : malformed) {
        write_file(badf.c_str(), m);
        CHECK(sp_tune_load(badf.c_str()) == SP_ERR_INVALID_ARG);
    }
    std::string longkey = "{\"";
    longkey.append(100000, 'k');
    longkey += "\": {\"nt\": 64, \"remap\": 0, \"stream\": 0}}";
    write_file(badf.c_str(), longkey.c_str());
    CHECK(sp_tune_load(badf.c_str()) == SP_OK);
    CHECK(sp_tune_load((dir + "/missing.json").c_str()) == SP_ERR_INVALID_ARG);
    CHECK(sp_tune_load(nullptr) == SP_ERR_INVALID_ARG);
    sp_release_cache();

    std::printf(failures ? "FAILED (%d)\n" : "ALL OK\n", failures);
    return failures ? 1 : 0;
}
