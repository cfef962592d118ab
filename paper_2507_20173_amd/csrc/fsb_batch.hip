// fsb_batch.hip -- many independent schools of uneven size advanced together
// by one persistent launch of several iterations.
//
// Work is cut into tiles: a tile is one wavefront's share of one school
// (64 lanes x fish_per_lane fish, the last tile of a school ragged).  The
// static schedule deals chunks of consecutive tiles to the wavefronts round
// robin, the same way in every sweep (one chunk per wavefront when the chunk
// size is n_tiles / W).  The dynamic and guided schedules cut the tile list
// into chunks (fixed-size, or shrinking with the tiles left) that wavefronts
// take from a per-sweep atomic counter, one atomic per chunk.  No result
// depends on which wavefront runs a tile.  Per iteration every tile
//   - reads its school's M_s (slot s % 3 of the per-school max ring),
//   - feeds, accumulates compensated lane sums, swims the next iteration,
//   - reduces over the wave (butterflies, no LDS): lane 0 stores the tile's
//     binary64 partials; the max of a run of consecutive tiles of one school
//     is folded into the school's next slot with one device-scope atomic max
//     when the run ends, and M of a school is loaded once per run.
// The grid barrier (shared with the single-school persistent kernel) then
// separates iterations.  After it, one wavefront per school folds that
// school's tile partials in tile order (deterministic) into the school's
// record and clears the used max slot.  Same 32 B/fish per iteration as the
// single-school persistent kernel; schools differ only in key and range.
// The first iteration index is read from a device counter that each launch
// advances, so one captured launch can be replayed as a graph.
#include <cstdlib>
#include <cstring>

#include "fsb_sweep.hpp"

namespace fsb {

// ---------------------------------------------------------------------------
// Tile schedule of one sweep, for one wavefront (all of its lanes call these
// together; every value here is uniform across the wavefront).
// ---------------------------------------------------------------------------
struct Walk {
    uint32_t tl;     // current tile; n_tiles once this wavefront's share is done
    uint32_t end;    // end of the current chunk
    uint32_t chunk;  // static schedule: index of the current chunk
};

__device__ __forceinline__ uint32_t grab_chunk(const BatchArgs& a, uint32_t* queue,
                                               uint32_t lane, uint32_t& end) {
    uint32_t c = 0;
    if (lane == 0) c = __hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c = uniform(c);
    if (c >= a.n_chunks) {
        end = 0;
        return a.n_tiles;
    }
    end = a.chunk_start[c + 1];
    return a.chunk_start[c];
}

__device__ __forceinline__ void static_chunk_at(const BatchArgs& a, Walk& w) {
    const uint64_t b = (uint64_t)w.chunk * a.static_chunk;
    if (b >= a.n_tiles) {
        w.tl = a.n_tiles;
        w.end = 0;
        return;
    }
    const uint64_t e = b + a.static_chunk;
    w.tl = (uint32_t)b;
    w.end = e < a.n_tiles ? (uint32_t)e : a.n_tiles;
}

__device__ __forceinline__ Walk first_tile(const BatchArgs& a, uint32_t* queue, uint32_t lane,
                                           uint32_t wave) {
    Walk w{a.n_tiles, 0u, wave};
    if (a.n_chunks) w.tl = grab_chunk(a, queue, lane, w.end);
    else static_chunk_at(a, w);
    return w;
}

__device__ __forceinline__ void next_tile(const BatchArgs& a, uint32_t* queue, uint32_t lane,
                                          uint32_t n_waves, Walk& w) {
    if (w.tl + 1 < w.end) {
        ++w.tl;
        return;
    }
    if (a.n_chunks) {
        w.tl = grab_chunk(a, queue, lane, w.end);
        return;
    }
    w.chunk += n_waves;
    static_chunk_at(a, w);
}

// Counter of sweep phase p (0 = prologue, k + 1 = sweep k of the launch).
__device__ __forceinline__ uint32_t* queue_of(const BatchArgs& a, uint32_t p) {
    return a.queue + (p & 1u) * kLineWords;
}

// ---------------------------------------------------------------------------
// Initial state of every school (not persistent).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void batch_init_fish(const BatchArgs& a, uint32_t k0, uint32_t k1,
                                                uint64_t i, float& x, float& y, float& w,
                                                float& c) {
    const Words p = pair_words(i >> 1, 0, kDomainInit, k0, k1);
    const Words q = pair_words(i >> 1, 1, kDomainInit, k0, k1);
    const bool odd = i & 1;
    x = a.H * signed_unit(odd ? p.r2 : p.r0);
    y = a.H * signed_unit(odd ? p.r3 : p.r1);
    const float span = a.whi - a.wlo;
    w = a.wlo + span * unit(odd ? q.r2 : q.r0);
    c = distance(x, y);
}

__global__ __launch_bounds__(256) void batch_init_kernel(BatchArgs a) {
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t wave = uniform(blockIdx.x * (256 / kWave) + threadIdx.x / kWave);
    const uint32_t n_waves = gridDim.x * (256 / kWave);
    for (uint32_t tl = wave; tl < a.n_tiles; tl += n_waves) {
        const Tile T = a.tiles[tl];
        const uint64_t base = 4 * T.col4;  // packed index of the tile's first fish
        for (uint32_t f = lane; f < T.n_fish; f += kWave) {
            const uint64_t i = 4ull * T.group0 + f;  // fish index within the school
            float x, y, w, c;
            batch_init_fish(a, T.k0, T.k1, i, x, y, w, c);
            a.x[base + f] = x;
            a.y[base + f] = y;
            a.w[base + f] = w;
            a.prev[base + f] = c;
            a.cur[base + f] = c;
        }
    }
}

// Clears the barrier words, the per-school max ring and the naive sums
// before a persistent launch (a kernel, so it can live in a graph).
__global__ void batch_reset_kernel(BatchArgs a) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nth = gridDim.x * blockDim.x;
    for (uint32_t i = tid; i < kSyncWords; i += nth) a.sync[i] = 0u;
    for (uint32_t i = tid; i < a.max_slots * a.n_schools; i += nth) a.school_max[i] = 0u;
    for (uint32_t i = tid; i < 8 * a.n_schools; i += nth) a.school_naive[i] = 0.0f;
    for (uint32_t i = tid; i < a.n_schools; i += nth) a.school_flag[i] = 0u;
    if (tid < 2) a.queue[tid * kLineWords] = 0u;
    if (tid < 2) a.ctrl->redo[tid] = 0u;
}

// ---------------------------------------------------------------------------
// Record of iteration s for every school: one wavefront per school folds the
// school's tile partials (lanes stride over tiles in order, then a butterfly).
// ---------------------------------------------------------------------------
template <bool kNaive>
__device__ void combine_schools(const BatchArgs& a, uint32_t s, uint32_t wave, uint32_t n_waves,
                                uint32_t lane) {
    const uint32_t S = a.n_schools;
    for (uint32_t c = wave; c < S; c += n_waves) {
        double acc[3] = {0.0, 0.0, 0.0};
        if constexpr (!kNaive) {
            const uint32_t tb = a.tile_begin[c], te = a.tile_begin[c + 1];
            const double* part = a.tile_part + (size_t)(s & 1u) * 3 * a.tile_cap;
            // Lane l adds tiles tb + l, tb + l + 64, ... in that order.  Up to
            // kBatchLoads of them are loaded before any is added, so a large
            // school's fold waits on memory once per batch, not once per tile.
            constexpr uint32_t kBatchLoads = 8;
            uint32_t i = tb + lane;
            for (; i + (kBatchLoads - 1) * kWave < te; i += kBatchLoads * kWave) {
                double v[3][kBatchLoads];
#pragma unroll
                for (uint32_t j = 0; j < kBatchLoads; ++j)
#pragma unroll
                    for (int k = 0; k < 3; ++k) v[k][j] = part[(size_t)k * a.tile_cap + i + j * kWave];
#pragma unroll
                for (uint32_t j = 0; j < kBatchLoads; ++j)
#pragma unroll
                    for (int k = 0; k < 3; ++k) acc[k] += v[k][j];
            }
            for (; i < te; i += kWave)
                for (int k = 0; k < 3; ++k) acc[k] += part[(size_t)k * a.tile_cap + i];
            for (int k = 0; k < 3; ++k) acc[k] = wave_sum_f64(acc[k]);
        }
        if (lane == 0) {
            uint32_t* slot = a.school_max + (size_t)(s % 3u) * S + c;
            fsb_record r;
            if constexpr (kNaive) {
                float* ns = a.school_naive + ((size_t)(s & 1u) * S + c) * 4;
                for (int k = 0; k < 3; ++k) {
                    acc[k] = (double)ns[k];
                    ns[k] = 0.0f;
                }
            }
            r.sum_w = acc[0];
            r.sum_wx = acc[1];
            r.sum_wy = acc[2];
            r.max_delta = __uint_as_float(ld_agent(slot));
            r.step_lo = s;
            a.rec[(size_t)(s % a.hist_len) * S + c] = r;
            st_agent(slot, 0u);
        }
    }
}

// Wave-wide sums of one tile -> its partial (lane 0 stores).
template <bool kNaive>
__device__ __forceinline__ void tile_sums(const BatchArgs& a, LaneSums<kNaive>& ls, uint32_t s,
                                          uint32_t tl, uint32_t school, uint32_t lane) {
    if constexpr (kNaive) {
        float v[3];
        for (int k = 0; k < 3; ++k) v[k] = wave_sum_f32(ls.f[k]);
        if (lane == 0) {
            float* ns = a.school_naive + ((size_t)(s & 1u) * a.n_schools + school) * 4;
            for (int k = 0; k < 3; ++k) atomicAdd(ns + k, v[k]);
        }
    } else {
        double v[3];
        for (int k = 0; k < 3; ++k) v[k] = csum_value(wave_csum(ls.c[k]));
        if (lane == 0) {
            double* part = a.tile_part + (size_t)(s & 1u) * 3 * a.tile_cap;
            for (int k = 0; k < 3; ++k) part[(size_t)k * a.tile_cap + tl] = v[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent batched kernel.  GPL = groups of four fish per lane per tile.
// Within a sweep a wavefront walks its tiles with the next tile's record and
// its school's max fetched while the current tile streams.
// ---------------------------------------------------------------------------

// Prologue work of one tile.  32-byte variant: swim t0 from (x, y), keep
// (x, y, prev).  Lean variant: a look-ahead swim of t0 for the max only,
// nothing stored.
template <int GPL, bool kNT, bool kLean>
__device__ __forceinline__ uint32_t tile_prologue(const BatchArgs& a, const Tile& T, uint32_t t0,
                                                  uint32_t lane) {
    const float H = a.H, Sw = a.S;
    const SwimRule rule{a.rule, a.wmin};
    uint32_t best = 0u;
#pragma unroll
    for (int q = 0; q < GPL; ++q) {
        const uint32_t j = lane + q * kWave;  // group within the tile
        if (4 * j >= T.n_fish) break;
        const uint64_t g = (uint64_t)T.group0 + j;
        const uint64_t c4 = T.col4 + j;
        if (4 * j + 4 <= T.n_fish) {
            float4 X = ldv<kNT>(a.x, c4), Y = ldv<kNT>(a.y, c4);
            float4 C;
#pragma unroll
            for (int f = 0; f < 4; ++f) lane_of(C, f) = distance(lane_of(X, f), lane_of(Y, f));
            float4 Wt = swim_weights<kNT>(rule, a.w, c4);
            float dx[4], dy[4];
            group_draws(Sw, T.k0, T.k1, g, t0, dx, dy);
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const float nc = swim(rule, lane_of(X, f), lane_of(Y, f), dx[f], dy[f], H,
                                      lane_of(C, f), lane_of(Wt, f));
                best = max(best, mag_bits(lane_of(C, f) - nc));
            }
            if constexpr (!kLean) {
                stv<kNT>(a.x, c4, X);
                stv<kNT>(a.y, c4, Y);
                stv<kNT>(a.prev, c4, C);
            }
        } else {
            for (uint32_t f = 0; 4 * j + f < T.n_fish; ++f) {
                const uint64_t o = 4 * c4 + f;
                float dx, dy;
                fish_draw(Sw, T.k0, T.k1, 4 * g + f, t0, dx, dy);
                float x = a.x[o], y = a.y[o];
                const float c = distance(x, y);
                const float wt = (rule.flags & kSwimWeighted) ? a.w[o] : 1.0f;
                const float nc = swim(rule, x, y, dx, dy, H, c, wt);
                best = max(best, mag_bits(c - nc));
                if constexpr (!kLean) {
                    a.x[o] = x;
                    a.y[o] = y;
                    a.prev[o] = c;
                }
            }
        }
    }
    return best;
}

template <int BLOCK, int GPL, bool kNaive, bool kNT, bool kLean>
__global__ __launch_bounds__(BLOCK) void batch_kernel(BatchArgs a) {
    constexpr uint32_t WPB = BLOCK / kWave;
    __shared__ uint32_t M_sh;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t wave = uniform(blockIdx.x * WPB + threadIdx.x / kWave);
    const uint32_t n_waves = gridDim.x * WPB;
    const uint32_t S = a.n_schools;
    const float H = a.H, Sw = a.S, wmin = a.wmin, wmax = a.wmax;
    const SwimRule rule{a.rule, a.wmin};
    const Barrier bar{a.sync, a.ctrl, a.spin_limit};
    uint32_t phase = 0;
    const uint32_t t0 = uniform(ld_agent(a.step));

    {
        uint32_t* next_max = a.school_max + (size_t)(t0 % 3u) * S;
        uint32_t* const queue = queue_of(a, 0);
        uint32_t best = 0u, run_school = 0u;
        for (Walk w = first_tile(a, queue, lane, wave); w.tl < a.n_tiles;
             next_tile(a, queue, lane, n_waves, w)) {
            const Tile T = a.tiles[w.tl];
            if (T.school != run_school) {  // a run of one school's tiles ends
                best = wave_max_u32(best);
                if (lane == 0 && best) max_agent(next_max + run_school, best);
                best = 0u;
                run_school = T.school;
            }
            best = max(best, tile_prologue<GPL, kNT, kLean>(a, T, t0, lane));
        }
        best = wave_max_u32(best);
        if (lane == 0 && best) max_agent(next_max + run_school, best);
    }
    if (!barrier_max(bar, 0u, phase, &M_sh)) return;

    for (uint32_t k = 0; k < a.steps; ++k) {
        const uint32_t s = t0 + k;
        const bool last = k + 1 == a.steps;
        if (k > 0) combine_schools<kNaive>(a, s - 1u, wave, n_waves, lane);
        // this sweep takes phase k + 1's counter; phase k + 2's (last used
        // by phase k, which every wavefront has left) is cleared for it
        uint32_t* const queue = queue_of(a, k + 1u);
        if (a.n_chunks && blockIdx.x == 0 && threadIdx.x == 0) st_agent(queue_of(a, k), 0u);
        const uint32_t* cur_max = a.school_max + (size_t)(s % 3u) * S;
        uint32_t* next_max = a.school_max + (size_t)((s + 1u) % 3u) * S;
        // M of a school is final once the barrier is passed and nobody writes
        // its slot during this sweep, so a plain load is coherent here; it is
        // loaded once per run of consecutive tiles of one school.
        Walk w = first_tile(a, queue, lane, wave);
        Tile T{};
        uint32_t Mb = 0u;
        if (w.tl < a.n_tiles) {
            T = a.tiles[w.tl];
            Mb = cur_max[T.school];
        }
        uint32_t best = 0u;  // lane max over the current run of one school's tiles
        while (w.tl < a.n_tiles) {
            Walk wn = w;
            next_tile(a, queue, lane, n_waves, wn);
            const uint32_t nx = wn.tl;
            Tile Tn{};
            if (nx < a.n_tiles) Tn = a.tiles[nx];
            float4 X[GPL], Y[GPL], W[GPL], P[GPL];
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                const uint32_t j = lane + q * kWave;
                if (4 * j + 4 <= T.n_fish) {
                    X[q] = ldv<kNT>(a.x, T.col4 + j);
                    Y[q] = ldv<kNT>(a.y, T.col4 + j);
                    W[q] = ldv<kNT>(a.w, T.col4 + j);
                    if constexpr (!kLean) P[q] = ldv<kNT>(a.prev, T.col4 + j);
                }
            }
            const bool run_ends = nx >= a.n_tiles || Tn.school != T.school;
            const uint32_t Mn = nx >= a.n_tiles ? 0u : run_ends ? cur_max[Tn.school] : Mb;
            const float M = __uint_as_float(Mb);
            LaneSums<kNaive> ls;
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                const uint32_t j = lane + q * kWave;
                if (4 * j >= T.n_fish) break;
                const uint64_t g = (uint64_t)T.group0 + j;
                const uint64_t c4 = T.col4 + j;
                if (4 * j + 4 <= T.n_fish) {
                    float4 C;
                    float dx[4], dy[4];
                    if constexpr (kLean) {
                        // redo swim s from the stored pre-swim position
                        group_draws(Sw, T.k0, T.k1, g, s, dx, dy);
#pragma unroll
                        for (int f = 0; f < 4; ++f) {
                            lane_of(P[q], f) = distance(lane_of(X[q], f), lane_of(Y[q], f));
                            lane_of(C, f) = swim(rule, lane_of(X[q], f), lane_of(Y[q], f), dx[f],
                                                 dy[f], H, lane_of(P[q], f), lane_of(W[q], f));
                        }
                    } else {
#pragma unroll
                        for (int f = 0; f < 4; ++f)
                            lane_of(C, f) = distance(lane_of(X[q], f), lane_of(Y[q], f));
                    }
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        const float diff = lane_of(P[q], f) - lane_of(C, f);
                        lane_of(W[q], f) = feed(lane_of(W[q], f), diff, M, wmin, wmax);
                    }
                    ls.add4(W[q], X[q], Y[q]);
                    stv<kNT>(a.w, c4, W[q]);
                    if constexpr (kLean) {
                        stv<kNT>(a.x, c4, X[q]);
                        stv<kNT>(a.y, c4, Y[q]);
                    }
                    if (last) {
                        if constexpr (kLean) stv<kNT>(a.prev, c4, P[q]);
                        stv<kNT>(a.cur, c4, C);
                    } else {
                        group_draws(Sw, T.k0, T.k1, g, s + 1u, dx, dy);
                        float4 nx = X[q], ny = Y[q];
#pragma unroll
                        for (int f = 0; f < 4; ++f) {
                            const float nc = swim(rule, lane_of(nx, f), lane_of(ny, f), dx[f],
                                                  dy[f], H, lane_of(C, f), lane_of(W[q], f));
                            best = max(best, mag_bits(lane_of(C, f) - nc));
                        }
                        if constexpr (!kLean) {
                            stv<kNT>(a.x, c4, nx);
                            stv<kNT>(a.y, c4, ny);
                            stv<kNT>(a.prev, c4, C);
                        }
                    }
                } else {
                    for (uint32_t f = 0; 4 * j + f < T.n_fish; ++f) {
                        const uint64_t o = 4 * c4 + f;
                        float x = a.x[o], y = a.y[o];
                        const float w0 = a.w[o];
                        float pv, c;
                        float dx, dy;
                        if constexpr (kLean) {
                            fish_draw(Sw, T.k0, T.k1, 4 * g + f, s, dx, dy);
                            pv = distance(x, y);
                            c = swim(rule, x, y, dx, dy, H, pv, w0);
                            a.x[o] = x;
                            a.y[o] = y;
                        } else {
                            pv = a.prev[o];
                            c = distance(x, y);
                        }
                        const float nw = feed(w0, pv - c, M, wmin, wmax);
                        a.w[o] = nw;
                        ls.add(nw, x, y);
                        if (last) {
                            if constexpr (kLean) a.prev[o] = pv;
                            a.cur[o] = c;
                        } else {
                            fish_draw(Sw, T.k0, T.k1, 4 * g + f, s + 1u, dx, dy);
                            const float nc = swim(rule, x, y, dx, dy, H, c, nw);
                            best = max(best, mag_bits(c - nc));
                            if constexpr (!kLean) {
                                a.x[o] = x;
                                a.y[o] = y;
                                a.prev[o] = c;
                            }
                        }
                    }
                }
            }
            tile_sums<kNaive>(a, ls, s, w.tl, T.school, lane);
            if (!last && run_ends) {
                best = wave_max_u32(best);
                if (lane == 0 && best) max_agent(next_max + T.school, best);
                best = 0u;
            }
            T = Tn;
            Mb = Mn;
            w = wn;
        }
        if (!barrier_max(bar, 0u, phase, &M_sh)) return;
    }
    combine_schools<kNaive>(a, t0 + a.steps - 1u, wave, n_waves, lane);
    if (blockIdx.x == 0 && threadIdx.x == 0) st_agent(a.step, t0 + a.steps);
}

// ---------------------------------------------------------------------------
// Deep batched kernel: KD iterations per grid barrier, as the single-school
// deep kernel (positions do not depend on weights, so a superstep replays its
// swims with the published maxima and swims the next superstep ahead for its
// maxima; x, y, w and the objective cur are read and written once per
// superstep, cur formed from the positions only in a launch's first).  Per school the
// maxima of iteration t live in slot t mod 3 KD of the max ring (written by
// the previous superstep's look-ahead, read by this one, cleared by the next
// one's combine), the tile partials of iteration t in slot t mod 2 KD.
// Compensated sums only; 256-thread blocks.  Registers are capped at 168 per
// lane so that three waves share each SIMD (its 512 registers per lane / 3):
// at 169 the occupancy drops to two waves and an iteration takes ~18% longer.
// ---------------------------------------------------------------------------
template <int KD>
__device__ void combine_schools_deep(const BatchArgs& a, uint32_t t0, uint32_t count,
                                     uint32_t wave, uint32_t n_waves, uint32_t lane) {
    const uint32_t S = a.n_schools;
    for (uint32_t c = wave; c < S; c += n_waves) {
        const uint32_t tb = a.tile_begin[c], te = a.tile_begin[c + 1];
        for (uint32_t j = 0; j < count; ++j) {
            const uint32_t t = t0 + j;
            const double* part = a.tile_part + (size_t)(t % (2 * KD)) * 3 * a.tile_cap;
            double acc[3] = {0.0, 0.0, 0.0};
            for (uint32_t i = tb + lane; i < te; i += kWave)
                for (int k = 0; k < 3; ++k) acc[k] += part[(size_t)k * a.tile_cap + i];
            for (int k = 0; k < 3; ++k) acc[k] = wave_sum_f64(acc[k]);
            if (lane == 0) {
                uint32_t* slot = a.school_max + (size_t)(t % (3 * KD)) * S + c;
                fsb_record r;
                r.sum_w = acc[0];
                r.sum_wx = acc[1];
                r.sum_wy = acc[2];
                r.max_delta = __uint_as_float(ld_agent(slot));
                r.step_lo = t;
                a.rec[(size_t)(t % a.hist_len) * S + c] = r;
                st_agent(slot, 0u);
            }
        }
    }
}

// The wave's maxima of kd iterations t .. t + kd - 1 for one school, into
// the ring (one device-scope atomic max per iteration, lane 0).
template <int KD>
__device__ __forceinline__ void flush_maxima(const BatchArgs& a, uint32_t (&best)[KD],
                                             uint32_t t, uint32_t kd, uint32_t school,
                                             uint32_t lane) {
#pragma unroll
    for (int j = 0; j < KD; ++j) {
        if ((uint32_t)j >= kd) break;
        const uint32_t m = wave_max_u32(best[j]);
        if (lane == 0 && m)
            max_agent(a.school_max + (size_t)((t + j) % (3 * KD)) * a.n_schools + school, m);
        best[j] = 0u;
    }
}

template <int BLOCK, int GPL, bool kNT, int KD, uint32_t kRule>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3)))
void batch_deep_kernel(BatchArgs a) {
    static_assert((kRule & kSwimWeighted) == 0, "the deep kernel never runs the weighted rule");
    constexpr uint32_t WPB = BLOCK / kWave;
    __shared__ uint32_t M_sh;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t wave = uniform(blockIdx.x * WPB + threadIdx.x / kWave);
    const uint32_t n_waves = gridDim.x * WPB;
    const float H = a.H, Sw = a.S, wmin = a.wmin, wmax = a.wmax;
    const SwimRule rule{kRule, a.wmin};  // compile-time flags: no run-time rule tests
    const Barrier bar{a.sync, a.ctrl, a.spin_limit};
    uint32_t phase = 0;
    const uint32_t t0 = uniform(ld_agent(a.step));

    // Prologue: the first superstep's maxima, from the stored positions.
    {
        const uint32_t kd0 = min((uint32_t)KD, a.steps);
        uint32_t* const queue = queue_of(a, 0);
        uint32_t best[KD];
#pragma unroll
        for (int j = 0; j < KD; ++j) best[j] = 0u;
        uint32_t run_school = 0u;
        for (Walk w = first_tile(a, queue, lane, wave); w.tl < a.n_tiles;
             next_tile(a, queue, lane, n_waves, w)) {
            const Tile T = a.tiles[w.tl];
            if (T.school != run_school) {
                flush_maxima<KD>(a, best, t0, kd0, run_school, lane);
                run_school = T.school;
            }
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                const uint32_t jg = lane + q * kWave;  // group within the tile
                if (4 * jg >= T.n_fish) break;
                const uint64_t g = (uint64_t)T.group0 + jg;
                const uint64_t c4 = T.col4 + jg;
                const uint32_t nf = min(4u, T.n_fish - 4 * jg);
                float4 X, Y, C;
                if (nf == 4) {
                    X = ldv<kNT>(a.x, c4);
                    Y = ldv<kNT>(a.y, c4);
                } else {  // the school's ragged last group: only its own fish are read
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        lane_of(X, f) = (uint32_t)f < nf ? a.x[4 * c4 + f] : 0.0f;
                        lane_of(Y, f) = (uint32_t)f < nf ? a.y[4 * c4 + f] : 0.0f;
                    }
                }
#pragma unroll
                for (int f = 0; f < 4; ++f) lane_of(C, f) = distance(lane_of(X, f), lane_of(Y, f));
#pragma unroll
                for (int j = 0; j < KD; ++j) {
                    if ((uint32_t)j >= kd0) break;
                    float dx[4], dy[4];
                    group_draws(Sw, T.k0, T.k1, g, t0 + j, dx, dy);
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        const float nc = swim(rule, lane_of(X, f), lane_of(Y, f), dx[f], dy[f], H,
                                              lane_of(C, f), 1.0f);
                        if ((uint32_t)f < nf) best[j] = max(best[j], mag_bits(lane_of(C, f) - nc));
                        lane_of(C, f) = nc;
                    }
                }
            }
        }
        flush_maxima<KD>(a, best, t0, kd0, run_school, lane);
    }
    if (!barrier_max(bar, 0u, phase, &M_sh)) return;

    // A sweep replays a superstep and swims the next one ahead.  Under the
    // plain swim the look-ahead of a large school forms a fish's objectives
    // only when its move can reach a guess just below the school's current
    // maxima (look_skip_limit); the guess is checked after the barrier, and
    // a school whose next maxima fall below it is swept once more, with no
    // replay and an exact look-ahead, before the next superstep.
    uint32_t kd_prev = 0;
    uint32_t sweep = 0;       // sweep phase (0 = prologue)
    bool redo_sweep = false;  // this sweep only redoes flagged schools' look-ahead
    for (uint32_t k0 = 0; k0 < a.steps;) {
        const uint32_t s0 = t0 + k0;
        const uint32_t kd = min((uint32_t)KD, a.steps - k0);
        const uint32_t kd_next = min((uint32_t)KD, a.steps - k0 - kd);
        const bool last = kd_next == 0;
        ++sweep;
        if (k0 > 0 && !redo_sweep)
            combine_schools_deep<KD>(a, s0 - kd_prev, kd_prev, wave, n_waves, lane);
        kd_prev = kd;
        // this sweep takes phase `sweep`'s counter; the other one (last used by
        // the previous phase, which every wavefront has left) is cleared for
        // the next phase
        uint32_t* const queue = queue_of(a, sweep);
        if (a.n_chunks && blockIdx.x == 0 && threadIdx.x == 0) st_agent(queue_of(a, sweep + 1u), 0u);
        // the redo word of this phase's parity: last read after the check two
        // phases ago, which every block has left
        uint32_t* const redo = &a.ctrl->redo[sweep & 1u];
        if (blockIdx.x == 0 && threadIdx.x == 0) st_agent(redo, 0u);
        bool filt = false;
        float skip_limit = 0.0f;
        uint32_t best[KD];
#pragma unroll
        for (int j = 0; j < KD; ++j) best[j] = 0u;
        float M[KD];
#pragma unroll
        for (int j = 0; j < KD; ++j) M[j] = 0.0f;
        uint32_t run_school = 0xffffffffu;
        for (Walk w = first_tile(a, queue, lane, wave); w.tl < a.n_tiles;
             next_tile(a, queue, lane, n_waves, w)) {
            const Tile T = a.tiles[w.tl];
            if (redo_sweep && !uniform(ld_agent(a.school_flag + T.school))) continue;
            if (T.school != run_school) {
                if (run_school != 0xffffffffu && !last)
                    flush_maxima<KD>(a, best, s0 + kd, kd_next, run_school, lane);
                run_school = T.school;
                // final since the barrier, and nobody writes these slots this sweep
#pragma unroll
                for (int j = 0; j < KD; ++j)
                    if ((uint32_t)j < kd)
                        M[j] = __uint_as_float(uniform(
                            a.school_max[(size_t)((s0 + j) % (3 * KD)) * a.n_schools + T.school]));
                if constexpr (kRule == 0) {
                    filt = !redo_sweep && a.look_theta > 0.0f && !last &&
                           a.tile_begin[T.school + 1] - a.tile_begin[T.school] >= a.look_min_tiles;
                    if (filt) {
                        float m_min = M[0];
#pragma unroll
                        for (int j = 1; j < KD; ++j)
                            if ((uint32_t)j < kd) m_min = fminf(m_min, M[j]);
                        skip_limit = look_skip_limit(a.look_theta * m_min, H, Sw);
                    }
                }
            }
            LaneSumsF64 ls[KD];
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                const uint32_t jg = lane + q * kWave;
                if (4 * jg >= T.n_fish) break;
                const uint64_t g = (uint64_t)T.group0 + jg;
                const uint64_t c4 = T.col4 + jg;
                const uint32_t nf = min(4u, T.n_fish - 4 * jg);
                float4 X, Y, W, C, P;
                if (nf == 4) {
                    X = ldv<kNT>(a.x, c4);
                    Y = ldv<kNT>(a.y, c4);
                    W = ldv<kNT>(a.w, c4);
                } else {  // every index below is a constant once the loops unroll, so the
                          // float4 state stays in registers (a run-time lane index would
                          // move it to memory for the whole loop)
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        lane_of(X, f) = (uint32_t)f < nf ? a.x[4 * c4 + f] : 0.0f;
                        lane_of(Y, f) = (uint32_t)f < nf ? a.y[4 * c4 + f] : 0.0f;
                        lane_of(W, f) = (uint32_t)f < nf ? a.w[4 * c4 + f] : 0.0f;
                    }
                }
                if (k0 == 0 && !redo_sweep) {
#pragma unroll
                    for (int f = 0; f < 4; ++f)
                        lane_of(C, f) = distance(lane_of(X, f), lane_of(Y, f));
                } else if (nf == 4) {  // stored by this launch's previous sweep (below)
                    C = ldv<kNT>(a.cur, c4);
                } else {
#pragma unroll
                    for (int f = 0; f < 4; ++f)
                        lane_of(C, f) = (uint32_t)f < nf ? a.cur[4 * c4 + f] : 0.0f;
                }
#pragma unroll
                for (int j = 0; j < KD; ++j) {
                    if ((uint32_t)j >= kd || redo_sweep) break;  // a redo sweep replays nothing
                    float dx[4], dy[4];
                    group_draws(Sw, T.k0, T.k1, g, s0 + j, dx, dy);
                    P = C;
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        lane_of(C, f) = swim(rule, lane_of(X, f), lane_of(Y, f), dx[f], dy[f], H,
                                             lane_of(P, f), 1.0f);
                        lane_of(W, f) = feed(lane_of(W, f), lane_of(P, f) - lane_of(C, f), M[j],
                                             wmin, wmax);
                    }
                    if (nf == 4) {
                        ls[j].add4(W, X, Y);
                    } else {
#pragma unroll
                        for (int f = 0; f < 4; ++f)
                            if ((uint32_t)f < nf) ls[j].add(lane_of(W, f), lane_of(X, f), lane_of(Y, f));
                    }
                }
                if (redo_sweep) {
                    // the columns stay as stored
                } else if (nf == 4) {
                    stv<kNT>(a.x, c4, X);
                    stv<kNT>(a.y, c4, Y);
                    stv<kNT>(a.w, c4, W);
                    stv<kNT>(a.cur, c4, C);
                    if (last) stv<kNT>(a.prev, c4, P);
                } else {
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        if ((uint32_t)f >= nf) break;
                        a.x[4 * c4 + f] = lane_of(X, f);
                        a.y[4 * c4 + f] = lane_of(Y, f);
                        a.w[4 * c4 + f] = lane_of(W, f);
                        a.cur[4 * c4 + f] = lane_of(C, f);
                        if (last) a.prev[4 * c4 + f] = lane_of(P, f);
                    }
                }
                if (!last && filt) {
                    // the plain swim's operations; C[f] is the objective of the
                    // current position only while fresh[f] holds
                    bool fresh[4] = {true, true, true, true};
#pragma unroll
                    for (int j = 0; j < KD; ++j) {
                        if ((uint32_t)j >= kd_next) break;
                        float dx[4], dy[4];
                        group_draws(Sw, T.k0, T.k1, g, s0 + kd + j, dx, dy);
#pragma unroll
                        for (int f = 0; f < 4; ++f) {
                            const float ox = lane_of(X, f), oy = lane_of(Y, f);
                            lane_of(X, f) = clamp_to(ox + dx[f], -H, H);
                            lane_of(Y, f) = clamp_to(oy + dy[f], -H, H);
                            if ((uint32_t)f < nf &&
                                __builtin_fmaf(dx[f], dx[f], dy[f] * dy[f]) >= skip_limit) {
                                float oc = lane_of(C, f);
                                if (!fresh[f]) oc = distance(ox, oy);
                                const float nc = distance(lane_of(X, f), lane_of(Y, f));
                                best[j] = max(best[j], mag_bits(oc - nc));
                                lane_of(C, f) = nc;
                                fresh[f] = true;
                            } else {
                                fresh[f] = false;
                            }
                        }
                    }
                } else if (!last) {
#pragma unroll
                    for (int j = 0; j < KD; ++j) {
                        if ((uint32_t)j >= kd_next) break;
                        float dx[4], dy[4];
                        group_draws(Sw, T.k0, T.k1, g, s0 + kd + j, dx, dy);
#pragma unroll
                        for (int f = 0; f < 4; ++f) {
                            const float nc = swim(rule, lane_of(X, f), lane_of(Y, f), dx[f], dy[f],
                                                  H, lane_of(C, f), 1.0f);
                            if ((uint32_t)f < nf)
                                best[j] = max(best[j], mag_bits(lane_of(C, f) - nc));
                            lane_of(C, f) = nc;
                        }
                    }
                }
            }
            // the tile's partials of each iteration (lane 0 stores): a
            // binary64 butterfly over the wave, whose six roundings are far
            // below the lanes' own binary32 error; a tile is one wave's work,
            // so this runs KD x 3 times per tile and costs a third of what a
            // TwoSum butterfly does
#pragma unroll
            for (int j = 0; j < KD; ++j) {
                if ((uint32_t)j >= kd || redo_sweep) break;
                double v[3];
                for (int k = 0; k < 3; ++k) v[k] = wave_sum_f64(ls[j].v[k]);
                if (lane == 0) {
                    double* part = a.tile_part + (size_t)((s0 + j) % (2 * KD)) * 3 * a.tile_cap;
                    for (int k = 0; k < 3; ++k) part[(size_t)k * a.tile_cap + w.tl] = v[k];
                }
            }
        }
        if (run_school != 0xffffffffu && !last)
            flush_maxima<KD>(a, best, s0 + kd, kd_next, run_school, lane);
        if (!barrier_max(bar, 0u, phase, &M_sh)) return;
        bool again = false;
        if (kRule == 0 && !redo_sweep && a.look_theta > 0.0f && !last) {
            // Every skipped |diff| is below the school's guess, so a published
            // maximum of at least the guess is exact.  One wavefront per
            // skipping school checks the next maxima against the guess, formed
            // from the same words as in the sweep; a school with one below it
            // is flagged.  After one more barrier, if any school is flagged,
            // the next sweep redoes those schools' look-ahead exactly (their
            // atomic maxima then reach the exact values: the skipping sweep's
            // are never above them).
            const size_t S = a.n_schools;
            for (uint32_t c = wave; c < a.n_schools; c += n_waves) {
                if (a.tile_begin[c + 1] - a.tile_begin[c] < a.look_min_tiles) continue;
                if (lane == 0) {
                    const uint32_t* mx = a.school_max + c;
                    float m_min = __uint_as_float(ld_agent(mx + (size_t)(s0 % (3 * KD)) * S));
                    for (uint32_t j = 1; j < kd; ++j)
                        m_min = fminf(m_min, __uint_as_float(
                                                 ld_agent(mx + (size_t)((s0 + j) % (3 * KD)) * S)));
                    const float guess = a.look_theta * m_min;
                    uint32_t fail = 0u;
                    for (uint32_t j = 0; j < kd_next; ++j)
                        fail |= __uint_as_float(
                                    ld_agent(mx + (size_t)((s0 + kd + j) % (3 * KD)) * S)) < guess;
                    st_agent(a.school_flag + c, fail);
                    if (fail) st_agent(redo, 1u);
                }
            }
            if (!barrier_max(bar, 0u, phase, &M_sh)) return;
            again = ld_agent(redo) != 0u;  // the same superstep's look-ahead again
        }
        redo_sweep = again;
        if (!again) {
            if (last) combine_schools_deep<KD>(a, s0, kd, wave, n_waves, lane);
            k0 += KD;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st_agent(a.step, t0 + a.steps);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
float batch_look_theta() {
    static const float theta = [] {
        const char* v = std::getenv("FSB_LOOKAHEAD_FILTER");
        if (v && std::strcmp(v, "off") == 0) return 0.0f;
        if (v && std::strcmp(v, "redo") == 0) return 2.0f;
        return kBatchLookTheta;
    }();
    return theta;
}

hipError_t launch_batch_init(const BatchArgs& a, uint32_t /*block*/, hipStream_t stream) {
    uint64_t waves = a.n_tiles;
    uint64_t blocks = (waves + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(batch_init_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t stream) {
    uint64_t work = (uint64_t)(a.max_slots > 8 ? a.max_slots : 8) * a.n_schools;
    if (work < kSyncWords) work = kSyncWords;
    uint64_t blocks = (work + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(batch_reset_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <int BLOCK, int GPL, bool kNaive>
const void* batch_fn8(uint32_t nt, uint32_t lean) {
    if (nt) return lean ? reinterpret_cast<const void*>(batch_kernel<BLOCK, GPL, kNaive, true, true>)
                        : reinterpret_cast<const void*>(batch_kernel<BLOCK, GPL, kNaive, true, false>);
    return lean ? reinterpret_cast<const void*>(batch_kernel<BLOCK, GPL, kNaive, false, true>)
                : reinterpret_cast<const void*>(batch_kernel<BLOCK, GPL, kNaive, false, false>);
}

template <int BLOCK, int GPL>
const void* batch_fn4(uint32_t naive, uint32_t nt, uint32_t lean) {
    return naive ? batch_fn8<BLOCK, GPL, true>(nt, lean) : batch_fn8<BLOCK, GPL, false>(nt, lean);
}

template <int BLOCK>
const void* batch_fn2(uint32_t fpl, uint32_t naive, uint32_t nt, uint32_t lean) {
    switch (fpl) {
        case 4: return batch_fn4<BLOCK, 1>(naive, nt, lean);
        case 8: return batch_fn4<BLOCK, 2>(naive, nt, lean);
        case 16: return batch_fn4<BLOCK, 4>(naive, nt, lean);
        default: return nullptr;
    }
}

template <bool kNT, uint32_t kRule>
const void* batch_deep_fn(uint32_t fpl) {
    switch (fpl) {
        case 4: return reinterpret_cast<const void*>(batch_deep_kernel<256, 1, kNT, kBatchDepth, kRule>);
        case 8: return reinterpret_cast<const void*>(batch_deep_kernel<256, 2, kNT, kBatchDepth, kRule>);
        case 16: return reinterpret_cast<const void*>(batch_deep_kernel<256, 4, kNT, kBatchDepth, kRule>);
        default: return nullptr;
    }
}

// The kernel of a shape and variant (null if there is none: the deep variant
// runs 256-thread blocks, compensated sums only, and the plain or greedy rule).
const void* batch_fn(uint32_t block, uint32_t fpl, uint32_t naive, uint32_t nt, uint32_t variant,
                     uint32_t rule) {
    if (variant == kBatchDeep) {
        if (block != 256 || naive || (rule & kSwimWeighted)) return nullptr;
        if (rule & kSwimGreedy)
            return nt ? batch_deep_fn<true, kSwimGreedy>(fpl) : batch_deep_fn<false, kSwimGreedy>(fpl);
        return nt ? batch_deep_fn<true, 0u>(fpl) : batch_deep_fn<false, 0u>(fpl);
    }
    const uint32_t lean = variant == kBatchLean;
    switch (block) {
        case 256: return batch_fn2<256>(fpl, naive, nt, lean);
        case 1024: return batch_fn2<1024>(fpl, naive, nt, lean);
        default: return nullptr;
    }
}

hipError_t batch_resident_grid(uint32_t block, uint32_t fish_per_lane, uint32_t naive,
                               uint32_t variant, uint32_t* out_grid) {
    *out_grid = 0;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int per_cu = 1 << 30;
    for (uint32_t nt = 0; nt < 2; ++nt)  // both cache policies and both rules must fit
        for (uint32_t rule : {0u, kSwimGreedy}) {
            const void* fn = batch_fn(block, fish_per_lane, naive, nt, variant, rule);
            if (!fn) return hipErrorInvalidValue;
            int b = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, (int)block, 0);
            if (e != hipSuccess) return e;
            per_cu = b < per_cu ? b : per_cu;
        }
    uint64_t g = (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 0);
    if (g > kMaxBarrierBlocks) g = kMaxBarrierBlocks;
    *out_grid = (uint32_t)g;
    return hipSuccess;
}

hipError_t launch_batch(const BatchArgs& a, uint32_t block, uint32_t fish_per_lane,
                        uint32_t naive, uint32_t streaming, uint32_t variant, uint32_t grid,
                        hipStream_t stream) {
    const void* fn = batch_fn(block, fish_per_lane, naive, streaming, variant, a.rule);
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = launch_batch_reset(a, stream);
    if (e != hipSuccess) return e;
    BatchArgs aa = a;
    void* args[] = {&aa};
    return launch_persistent(fn, dim3(grid), dim3(block), args, stream);
}

}  // namespace fsb
