// fsb_plan.hpp -- host-only planning of a batch of schools: argument checks
// of the school list and of a launch shape, the tile table, the chunk table
// of the work-queue schedules, and the lines of the autotuner's cache file.
// Pure host arithmetic with no HIP call, so it is also built on its own with
// the address and undefined-behaviour sanitizers (tests/host_checks.cpp).
#pragma once

#include <cinttypes>
#include <cstdio>
#include <string>
#include <vector>

#include "fsb.h"
#include "fsb_host.hpp"
#include "fsb_internal.hpp"

namespace fsb {

// Largest start of a school in the packed columns: keeps start + size far
// from wrapping a 64-bit index.
constexpr uint64_t kMaxStart = 1ull << 62;
constexpr uint64_t kMaxSchoolFish = 1ull << 34;

// Tiles of a school of `fish` fish at `fpl` fish per lane (64 lanes per tile).
inline uint64_t tiles_for(uint64_t fish, uint32_t fpl) {
    const uint64_t groups = (fish + 3) / 4;
    const uint64_t per_tile = 64ull * (fpl / 4);
    return (groups + per_tile - 1) / per_tile;
}

inline bool valid_fpl(uint32_t fpl) { return fpl == 4 || fpl == 8 || fpl == 16; }
inline bool valid_block(uint32_t b) { return b == 256 || b == 1024; }

// The school list: n in [1, 2^24]; every school non-empty and at most 2^34
// fish, starting at a multiple of 4 no later than 2^62, increasing and not
// overlapping; at most 2^40 fish in all and fewer than 2^32 tiles at four
// fish per lane (the most tiles any shape makes).  Writes that tile count
// (the tile tables' capacity) and the total fish.
inline int check_schools(uint32_t n, const uint64_t* starts, const uint64_t* sizes, uint64_t* cap,
                         uint64_t* total) {
    if (n == 0 || n > (1u << 24)) return fail(FSB_ERR_INVALID_ARG, "n_schools must be in [1, 2^24]");
    if (!starts || !sizes) return fail(FSB_ERR_INVALID_ARG, "starts/sizes are NULL");
    uint64_t c = 0, tot = 0, end = 0;
    for (uint32_t s = 0; s < n; ++s) {
        if (sizes[s] == 0) return fail(FSB_ERR_INVALID_ARG, "school " + std::to_string(s) + " is empty");
        if (sizes[s] > kMaxSchoolFish)
            return fail(FSB_ERR_INVALID_ARG, "school " + std::to_string(s) + " exceeds 2^34 fish");
        if (starts[s] > kMaxStart)
            return fail(FSB_ERR_INVALID_ARG, "school " + std::to_string(s) + " starts beyond 2^62");
        if (starts[s] % 4) return fail(FSB_ERR_INVALID_ARG, "starts must be multiples of 4");
        if (starts[s] < end)
            return fail(FSB_ERR_INVALID_ARG, "schools must be increasing and not overlap");
        end = starts[s] + sizes[s];
        c += tiles_for(sizes[s], 4);
        tot += sizes[s];
    }
    if (tot > kMaxFish) return fail(FSB_ERR_INVALID_ARG, "more than 2^40 fish in the batch");
    if (c >= (1ull << 32)) return fail(FSB_ERR_INVALID_ARG, "too many tiles");
    *cap = c;
    *total = tot;
    return FSB_OK;
}

inline int check_tuning(const fsb_tuning* t) {
    if (!valid_block(t->block_size)) return fail(FSB_ERR_INVALID_ARG, "block_size must be 256 or 1024");
    if (!valid_fpl(t->fish_per_thread))
        return fail(FSB_ERR_INVALID_ARG, "fish_per_thread must be 4, 8 or 16");
    if (t->steps_per_launch == 0) return fail(FSB_ERR_INVALID_ARG, "steps_per_launch must be >= 1");
    if (t->variant != 0 && t->variant != FSB_RUN_FUSED_PREV && t->variant != FSB_RUN_FUSED_LEAN &&
        t->variant != FSB_RUN_FUSED_DEEP)
        return fail(FSB_ERR_INVALID_ARG,
                    "variant must be 0, FSB_RUN_FUSED_PREV, FSB_RUN_FUSED_LEAN or FSB_RUN_FUSED_DEEP");
    if (t->variant == FSB_RUN_FUSED_DEEP && t->block_size != 256)
        return fail(FSB_ERR_INVALID_ARG, "the deep variant runs 256-thread blocks");
    if (t->schedule != FSB_SCHED_STATIC && t->schedule != FSB_SCHED_DYNAMIC &&
        t->schedule != FSB_SCHED_GUIDED)
        return fail(FSB_ERR_INVALID_ARG, "schedule must be FSB_SCHED_STATIC, _DYNAMIC or _GUIDED");
    if (t->schedule != FSB_SCHED_STATIC && t->chunk_tiles == 0)
        return fail(FSB_ERR_INVALID_ARG, "chunk_tiles must be >= 1 for a dynamic or guided schedule");
    return FSB_OK;
}

// Tile table of checked schools at `fpl` fish per lane: the tiles of school s
// are tiles[begin[s] .. begin[s+1]), in order; each covers up to 64 x fpl
// consecutive fish of its school and never straddles two schools.
inline void build_tile_table(uint32_t n, const uint64_t* start, const uint64_t* size,
                             const uint64_t* seed, uint32_t fpl, std::vector<Tile>& tiles,
                             std::vector<uint32_t>& begin) {
    tiles.clear();
    begin.assign(n + 1, 0u);
    const uint32_t per_tile = 64u * (fpl / 4);  // groups of four fish per tile
    for (uint32_t s = 0; s < n; ++s) {
        begin[s] = (uint32_t)tiles.size();
        const uint64_t groups = (size[s] + 3) / 4;
        for (uint64_t g0 = 0; g0 < groups; g0 += per_tile) {
            const uint64_t fish_left = size[s] - 4 * g0;
            const uint64_t cap = 4ull * per_tile;
            Tile t{};
            t.col4 = start[s] / 4 + g0;
            t.school = s;
            t.group0 = (uint32_t)g0;
            t.n_fish = (uint32_t)(fish_left < cap ? fish_left : cap);
            t.k0 = (uint32_t)seed[s];
            t.k1 = (uint32_t)(seed[s] >> 32);
            tiles.push_back(t);
        }
    }
    begin[n] = (uint32_t)tiles.size();
}

// Chunk starts of the dynamic and guided schedules over n_tiles tiles for a
// grid of `waves` wavefronts: chunks of chunk_tiles consecutive tiles (guided:
// the chunk starting at tile p spans max(chunk_tiles, ceil((n_tiles - p) /
// waves)) tiles), then n_tiles as the end.  chunk_tiles >= 1, waves >= 1.
inline void build_chunk_starts(uint64_t n_tiles, uint32_t schedule, uint32_t chunk_tiles,
                               uint32_t waves, std::vector<uint32_t>& start) {
    start.clear();
    for (uint64_t p = 0; p < n_tiles;) {
        start.push_back((uint32_t)p);
        uint64_t len = chunk_tiles;
        if (schedule == FSB_SCHED_GUIDED) {
            const uint64_t share = (n_tiles - p + waves - 1) / waves;
            if (share > len) len = share;
        }
        p = p + len < n_tiles ? p + len : n_tiles;
    }
    start.push_back((uint32_t)n_tiles);
}

// One line of the autotuner's cache file: the key (no blanks), then the seven
// fields of fsb_tuning.
inline std::string format_cache_line(const std::string& key, const fsb_tuning& t) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s %u %u %u %u %u %u %u\n", key.c_str(), t.block_size,
                  t.fish_per_thread, t.steps_per_launch, t.blocks_per_cu, t.variant, t.schedule,
                  t.chunk_tiles);
    return buf;
}

// A cache line's tuning if its key is `key` and the tuning is valid; false
// for any other line (another key, missing or malformed fields, an invalid
// tuning), which is then ignored.
inline bool parse_cache_line(const char* line, const std::string& key, fsb_tuning* out) {
    char k[300];
    fsb_tuning t{};
    if (std::sscanf(line, "%299s %u %u %u %u %u %u %u", k, &t.block_size, &t.fish_per_thread,
                    &t.steps_per_launch, &t.blocks_per_cu, &t.variant, &t.schedule,
                    &t.chunk_tiles) != 8)
        return false;
    if (key != k) return false;
    const std::string saved = last_error();
    const bool ok = check_tuning(&t) == FSB_OK;
    last_error() = saved;  // a rejected line is not the caller's error
    if (ok) *out = t;
    return ok;
}

}  // namespace fsb
