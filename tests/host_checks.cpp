// host_checks.cpp -- unit checks of libfsb's pure host code, built with g++
// and the address and undefined-behaviour sanitizers (no GPU, no HIP call
// beyond error names): configuration and column checks, workspace layouts,
// the mapping of failed persistent launches, the batch's school and tuning
// checks, tile and chunk tables, and the autotuner's cache lines.  Prints
// "host checks ok" and exits 0, or names the first failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "fsb.h"
#include "fsb_host.hpp"
#include "fsb_internal.hpp"
#include "fsb_plan.hpp"

using namespace fsb;

static int failures = 0;

#define CHECK(cond)                                                               \
    do {                                                                          \
        if (!(cond)) {                                                            \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

static fsb_config base_config() {
    fsb_config c{};
    c.n_fish = 1000;
    c.seed = 7;
    c.pond_half = 100.0f;
    c.swim_step = 0.1f;
    c.w_init_lo = 1.0f;
    c.w_init_hi = 2.0f;
    c.w_min = 1.0f;
    c.w_max = 4.0f;
    c.reduce_mode = FSB_REDUCE_COMPENSATED;
    c.history_len = 4;
    c.swim_rule = 0;
    return c;
}

static void config_checks() {
    fsb_config c = base_config();
    CHECK(check_config(&c, true) == FSB_OK);
    CHECK(check_config(nullptr, true) == FSB_ERR_INVALID_ARG);
    c.n_fish = 0;
    CHECK(check_config(&c, true) == FSB_ERR_INVALID_ARG);
    CHECK(check_config(&c, false) == FSB_OK);
    c = base_config();
    c.pond_half = 0x1p64f;
    CHECK(check_config(&c, true) == FSB_ERR_INVALID_ARG);
    c = base_config();
    c.swim_step = 0x1p-110f;
    CHECK(check_config(&c, true) == FSB_ERR_INVALID_ARG);
    c = base_config();
    c.w_min = 5.0f;
    CHECK(check_config(&c, true) == FSB_ERR_INVALID_ARG);
    c = base_config();
    c.history_len = kMaxHistory + 1;
    CHECK(check_config(&c, true) == FSB_ERR_INVALID_ARG);
    c = base_config();
    c.swim_rule = FSB_SWIM_WEIGHTED;
    c.w_min = 0.0f;
    CHECK(check_config(&c, true) == FSB_ERR_INVALID_ARG);
    CHECK(!last_error().empty());
}

static void column_checks() {
    static float buf[5][64] __attribute__((aligned(16)));
    fsb_state st{buf[0], buf[1], buf[2], buf[3], buf[4]};
    CHECK(check_columns(st, 64) == FSB_OK);
    fsb_state overlap{buf[0], buf[0] + 32, buf[2], buf[3], buf[4]};
    CHECK(check_columns(overlap, 64) == FSB_ERR_INVALID_ARG);
    CHECK(check_columns(overlap, 32) == FSB_OK);  // adjacent halves do not overlap
    fsb_state misaligned{buf[0] + 1, buf[1], buf[2], buf[3], buf[4]};
    CHECK(check_columns(misaligned, 8) == FSB_ERR_INVALID_ARG);
    fsb_state null_col{buf[0], nullptr, buf[2], buf[3], buf[4]};
    CHECK(check_columns(null_col, 8) == FSB_ERR_INVALID_ARG);
    alignas(256) static unsigned char ws[512];
    CHECK(check_workspace(ws, sizeof(ws), 512) == FSB_OK);
    CHECK(check_workspace(ws, sizeof(ws), 513) == FSB_ERR_INVALID_ARG);
    CHECK(check_workspace(ws + 16, 256, 256) == FSB_ERR_INVALID_ARG);
    CHECK(check_workspace(nullptr, 256, 256) == FSB_ERR_INVALID_ARG);
}

static void layout_checks() {
    for (uint32_t h : {0u, 1u, 7u, 1000u}) {
        const Layout L = school_layout(h);
        CHECK(L.hist >= L.ctrl + sizeof(Ctrl));
        CHECK(L.blockmax >= L.hist + (size_t)h * sizeof(fsb_record));
        CHECK(L.partials >= L.blockmax + kMaxGrid * 4);
        CHECK(L.sync >= L.partials + 2 * 3 * (size_t)kMaxGrid * 8);
        CHECK(L.deep >= L.sync + kSyncWords * 4);
        CHECK(L.total >= L.deep + (size_t)kDeepSlots * 3 * kMaxBarrierBlocks * 8);
        CHECK(L.total % kAlign == 0 && L.hist % kAlign == 0 && L.deep % kAlign == 0);
    }
    CHECK(kStaticLayout.total <= kStaticScratchBytes);
    for (bool deep : {false, true}) {
        const BatchLayout B = batch_layout(4096, 600000, 500, deep);
        CHECK(B.tile_begin >= B.sync + kSyncWords * 4);
        CHECK(B.tiles >= B.tile_begin + 4097 * 4);
        CHECK(B.tile_part >= B.tiles + 600000 * sizeof(Tile));
        CHECK(B.school_max >= B.tile_part + (deep ? 16 : 2) * 3 * 600000ull * 8);
        CHECK(B.rec >= B.school_naive + 2 * 4096 * 4 * 4);
        CHECK(B.chunks >= B.rec + 500ull * 4096 * sizeof(fsb_record));
        CHECK(B.total >= B.queue + 2 * kLineWords * 4 && B.total % kAlign == 0);
    }
}

static void launch_error_checks() {
    CHECK(persistent_launch_fail(hipErrorIllegalState, "launch") == FSB_ERR_UNSUPPORTED);
    CHECK(last_error().find("another process") != std::string::npos);
    CHECK(persistent_launch_fail(hipErrorCooperativeLaunchTooLarge, "launch") ==
          FSB_ERR_UNSUPPORTED);
    CHECK(last_error().find("co-resident") != std::string::npos);
    CHECK(persistent_launch_fail(hipErrorLaunchFailure, "launch") == FSB_ERR_HIP);
    CHECK(last_error().find("launch") == 0);
}

static void school_list_checks() {
    uint64_t cap = 0, total = 0;
    const uint64_t starts[3] = {0, 1000, 3000}, sizes[3] = {1000, 2000, 5};
    CHECK(check_schools(3, starts, sizes, &cap, &total) == FSB_OK);
    CHECK(total == 3005 && cap == tiles_for(1000, 4) + tiles_for(2000, 4) + tiles_for(5, 4));
    const uint64_t overlap[2] = {0, 4}, sz8[2] = {8, 4};
    CHECK(check_schools(2, overlap, sz8, &cap, &total) == FSB_ERR_INVALID_ARG);
    const uint64_t odd[2] = {0, 10};
    CHECK(check_schools(2, odd, sz8, &cap, &total) == FSB_ERR_INVALID_ARG);
    const uint64_t huge[2] = {0, (1ull << 63) + 4}, sz1[2] = {4, 4};
    CHECK(check_schools(2, huge, sz1, &cap, &total) == FSB_ERR_INVALID_ARG);
    const uint64_t wrap[2] = {0, kMaxStart}, szw[2] = {4, kMaxSchoolFish};
    CHECK(check_schools(2, wrap, szw, &cap, &total) == FSB_OK);
    const uint64_t empty[1] = {0}, sz0[1] = {0};
    CHECK(check_schools(1, empty, sz0, &cap, &total) == FSB_ERR_INVALID_ARG);
    CHECK(check_schools(0, starts, sizes, &cap, &total) == FSB_ERR_INVALID_ARG);
    CHECK(check_schools(3, nullptr, sizes, &cap, &total) == FSB_ERR_INVALID_ARG);
}

static void tuning_checks() {
    fsb_tuning t{256, 8, 100, 0, 0, FSB_SCHED_STATIC, 0};
    CHECK(check_tuning(&t) == FSB_OK);
    t.block_size = 512;
    CHECK(check_tuning(&t) == FSB_ERR_INVALID_ARG);
    t = {1024, 8, 100, 0, FSB_RUN_FUSED_DEEP, FSB_SCHED_STATIC, 0};
    CHECK(check_tuning(&t) == FSB_ERR_INVALID_ARG);
    t = {256, 8, 100, 0, 0, FSB_SCHED_DYNAMIC, 0};
    CHECK(check_tuning(&t) == FSB_ERR_INVALID_ARG);
    t = {256, 12, 100, 0, 0, FSB_SCHED_STATIC, 0};
    CHECK(check_tuning(&t) == FSB_ERR_INVALID_ARG);
    t = {256, 8, 0, 0, 0, FSB_SCHED_STATIC, 0};
    CHECK(check_tuning(&t) == FSB_ERR_INVALID_ARG);
}

static void tile_table_checks() {
    const uint32_t n = 6;
    const uint64_t size[n] = {1, 5, 256, 257, 1024 * 16 + 3, 70001};
    uint64_t start[n], seed[n];
    uint64_t at = 8;
    for (uint32_t s = 0; s < n; ++s) {
        start[s] = at;
        seed[s] = 0x123456789ull * (s + 1);
        at += (size[s] + 63) / 64 * 64 + 4;  // gaps between schools
    }
    for (uint32_t fpl : {4u, 8u, 16u}) {
        std::vector<Tile> tiles;
        std::vector<uint32_t> begin;
        build_tile_table(n, start, size, seed, fpl, tiles, begin);
        CHECK(begin.size() == n + 1 && begin[0] == 0 && begin[n] == tiles.size());
        const uint32_t cap = 64 * fpl;
        for (uint32_t s = 0; s < n; ++s) {
            CHECK(begin[s + 1] - begin[s] == tiles_for(size[s], fpl));
            uint64_t covered = 0;
            for (uint32_t i = begin[s]; i < begin[s + 1]; ++i) {
                const Tile& t = tiles[i];
                CHECK(t.school == s && t.n_fish >= 1 && t.n_fish <= cap);
                CHECK(4ull * t.group0 == covered);  // consecutive, no gap, no overlap
                CHECK(t.col4 == start[s] / 4 + t.group0);
                CHECK(t.k0 == (uint32_t)seed[s] && t.k1 == (uint32_t)(seed[s] >> 32));
                covered += t.n_fish;
            }
            CHECK(covered == size[s]);  // never past the school's last fish
        }
    }
}

static void chunk_checks() {
    for (uint64_t n_tiles : {1ull, 7ull, 1000ull, 65536ull})
        for (uint32_t sched : {(uint32_t)FSB_SCHED_DYNAMIC, (uint32_t)FSB_SCHED_GUIDED})
            for (uint32_t chunk : {1u, 4u, 64u})
                for (uint32_t waves : {1u, 3u, 1024u}) {
                    std::vector<uint32_t> st;
                    build_chunk_starts(n_tiles, sched, chunk, waves, st);
                    CHECK(st.size() >= 2 && st.front() == 0 && st.back() == n_tiles);
                    for (size_t i = 1; i < st.size(); ++i) {
                        const uint64_t len = st[i] - st[i - 1];
                        CHECK(len >= 1);
                        if (i + 1 < st.size()) CHECK(len >= chunk);  // only the last may be short
                        if (sched == FSB_SCHED_DYNAMIC && i + 1 < st.size()) CHECK(len == chunk);
                        if (sched == FSB_SCHED_GUIDED) {
                            const uint64_t left = n_tiles - st[i - 1];
                            const uint64_t share = (left + waves - 1) / waves;
                            const uint64_t want = share > chunk ? share : chunk;
                            CHECK(len == (want < left ? want : left));
                        }
                    }
                }
}

static void cache_line_checks() {
    const fsb_tuning t{256, 16, 1000, 0, FSB_RUN_FUSED_DEEP, FSB_SCHED_DYNAMIC, 4};
    const std::string key = "gfx950|4096|606898723|0123456789abcdef|0";
    const std::string line = format_cache_line(key, t);
    fsb_tuning got{};
    CHECK(parse_cache_line(line.c_str(), key, &got));
    CHECK(std::memcmp(&got, &t, sizeof(t)) == 0);
    CHECK(!parse_cache_line(line.c_str(), key + "x", &got));  // another key
    CHECK(!parse_cache_line("gfx950|1 256 8", "gfx950|1", &got));  // truncated
    CHECK(!parse_cache_line("", key, &got));
    const std::string bad = key + " 1024 16 1000 0 5 1 4\n";  // deep needs 256 threads
    CHECK(!parse_cache_line(bad.c_str(), key, &got));
    std::string long_key(400, 'k');  // longer than the key buffer: read up to its size
    const std::string long_line = long_key + " 256 8 100 0 0 0 0\n";
    CHECK(!parse_cache_line(long_line.c_str(), long_key, &got));
    CHECK(!parse_cache_line("k 4294967295 8 100 0 0 0 0", "k", &got));
}

int main() {
    config_checks();
    column_checks();
    layout_checks();
    launch_error_checks();
    school_list_checks();
    tuning_checks();
    tile_table_checks();
    chunk_checks();
    cache_line_checks();
    if (failures) {
        std::fprintf(stderr, "%d host checks failed\n", failures);
        return 1;
    }
    std::printf("host checks ok\n");
    return 0;
}
