// libkdt: kinetic Delaunay triangulation of moving lattice points on MI355X.
//
// Kernels (one 64-lane wavefront per block of the partition, Sec. IV):
//   k_build_blocks  every block's DT* from scratch, the threads of a
//                workgroup inserting in parallel (kdt_pbuild.hpp); the
//                starting state of Fig. 4 (k_build_listed: the blocks the
//                rebuild branch left for after a step)
//   k_step       one time step: for each block, its moves in order, each a
//                walk to the target, Delete, Insert (Fig. 4)
//   k_run_fused  all steps of a move stream; blocks are independent, so each
//                wavefront runs its block's steps back to back
//   k_qcount / k_qwrite   compaction of the real triangles (query)
// plus the host implementation of include/kdt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/kdt.h"
#include "kdt_device.hpp"
#include "kdt_mlp.hpp"
#include "kdt_pbuild.hpp"

using namespace kdt;

namespace {

constexpr int KDT_COORD_LIMIT = 1 << 24;

// ------------------------------------------------------------------ device

// Kernel arguments are read through the scalar cache in 64-byte lines; the
// fields a move reads sit in the first line and, with the step kernels' own
// arguments, the third, so that the second (build, global mode, selection
// inputs) is not fetched on the way to a move.
struct DevState {
    Tri* tri;
    int2* xy;
    int* vtri;
    const long long* pt_off;
    const long long* tri_off;
    const int4* frame;
    int* status;
    int policy;    // repair-or-rebuild selection: KDT_POLICY_*
    int step_lds;  // dynamic LDS the step kernels run with: blocks whose build fits it are rebuilt there
    int* sticky;
    const int* order;  // per-block insertion order (Hilbert order at init)
    int* owner;        // one int per triangle slot: cavity claims of the parallel build
    int* own2;         // one int per triangle slot: boundary claims of the parallel build
    int* rb_list;      // blocks to rebuild after this step: [0] count, [1] finished builders, [2..] blocks
    const float* mlp_w;  // MLP parameters (policy MLP)
    long long log_cap;   // steps the log holds (ring)
    float tau;           // threshold rule: rebuild iff sum of d / spacing > tau
    float dlim;          // d of the latest d-calculation (0: none yet): feature 15, the d-limit rule
    int n_blocks;
    int repair;    // repair variant: KDT_REPAIR_*
    int prefetch;  // rings around the movers' stars warmed in cache before a block's moves (0: none)
    int pad_;
    BlockStats* stats;
    float* log;  // per step and block: LOG_FIELDS floats, or null
    // the branch of every block for this step chosen before the step kernels
    // (k_choose; its features logged there), or null: chosen by the block
    const int8_t* choice;
};
static_assert(offsetof(DevState, step_lds) < 64 && offsetof(DevState, stats) >= 128, "move fields off their lines");

__device__ __forceinline__ BlockView view_of(const DevState& s, int b) {
    BlockView B;
    const long long p0 = s.pt_off[b], p1 = s.pt_off[b + 1];
    B.tri = s.tri + s.tri_off[b];
    B.xy = s.xy + p0;
    B.vtri = s.vtri + p0;
    B.n = (int)(p1 - p0);
    B.ntri = 2 * B.n - 2;
    return B;
}

// What a block's step reads first -- its status, move range, point range,
// record offset and frame -- requested in one round trip.
struct BlockHead {
    int status, m0, m1;
    long long p0, p1, toff;
    int4 fr;
};
__device__ __forceinline__ BlockHead load_head(const DevState& s, int b, const int* off) {
    BlockHead h;
    h.status = s.status[b];
    h.m0 = off[b];
    h.m1 = off[b + 1];
    h.p0 = s.pt_off[b];
    h.p1 = s.pt_off[b + 1];
    h.toff = s.tri_off[b];
    h.fr = s.frame[b];
    return h;
}
// Nothing to do: a failed block, or a move range that starts past its end
// (no moves, as the loop would find).  The other fields are tested too,
// against what never holds (a block's points lie inside its frame), so that
// the compiler keeps every load of the head ahead of this branch.
__device__ __forceinline__ bool head_skip(const BlockHead& h) {
    // (bitwise: a chain of || would wait for each load at its own branch)
    return ((h.status != 0) | (h.m0 > h.m1) | (h.p0 > h.p1) | (h.toff < 0) | (h.fr.x > h.fr.z) |
            (h.fr.y > h.fr.w)) != 0;
}

__device__ __forceinline__ void fail_block(const DevState& s, int b, int code) {
    if (threadIdx.x == 0) {
        s.status[b] = code;
        atomicAdd(reinterpret_cast<unsigned long long*>(&s.stats[b].errors), 1ull);
        atomicMin(s.sticky, code);
    }
}

constexpr int PB_THREADS = 128;
constexpr int PB_LDS_BYTES = 128 * 1024;  // dynamic LDS asked for by the block build
__host__ __device__ constexpr size_t pb_fixed_lds() {
    return (sizeof(int) * (4 + PB_DEFER + (size_t)PB_THREADS * ATT_B_INTS) + 15) & ~(size_t)15;
}
// LDS a block of n points needs to be built in LDS: records, both claim
// arrays and incident triangles (after the fixed part).
__host__ __device__ constexpr size_t pb_block_lds(long long n) {
    return (size_t)(2 * n - 2) * (sizeof(Tri) + 2 * sizeof(int)) + sizeof(int) * (size_t)n;
}

// Build block b's DT* with the PB_THREADS threads of a workgroup: in
// `lds_bytes` of dynamic LDS when its working state fits there (written
// back at the end), else in place.  flagged: a block the rebuild branch
// left for after the step (its cost goes into the step log).
__device__ __forceinline__ void build_block(const DevState& s, int b, bool flagged, long long step, int lds_bytes,
                                            char* dyn) {
    const long long c0 = wall_clock64();
    BlockView G = view_of(s, b);
    int* lds = reinterpret_cast<int*>(dyn);
    PBMem M;
    M.att = lds + 4 + PB_DEFER;
    if (pb_fixed_lds() + pb_block_lds(G.n) <= (size_t)lds_bytes) {
        M.tri = reinterpret_cast<Tri*>(dyn + pb_fixed_lds());
        M.cown = reinterpret_cast<int*>(M.tri + G.ntri);
        M.bown = M.cown + G.ntri;
        M.vtri = M.bown + G.ntri;
    } else {
        M.tri = G.tri;
        M.vtri = G.vtri;
        M.cown = s.owner + s.tri_off[b];
        M.bown = s.own2 + s.tri_off[b];
    }
    const int rc = pbuild_block(G, s.order + s.pt_off[b], M, lds);
    if (rc != ST_OK) fail_block(s, b, rc);
    if (flagged && threadIdx.x == 0) {
        // the branch's cost in the step log includes the build
        if (s.log && s.log_cap > 0)
            s.log[((step % s.log_cap) * (long long)s.n_blocks + b) * LOG_FIELDS + 17] += (float)(wall_clock64() - c0);
    }
}

// Every block's DT* from scratch (the starting state), one workgroup each.
__global__ void __launch_bounds__(PB_THREADS) k_build_blocks(DevState s, int lds_bytes) {
    extern __shared__ __align__(16) char dyn[];
    build_block(s, blockIdx.x, false, 0, lds_bytes, dyn);
}

// The blocks the rebuild branch of this step listed (too large to build in
// the step kernel): a fixed grid (a few workgroups per compute unit) strides
// over the list; the last workgroup to finish empties it for the next step.
__global__ void __launch_bounds__(PB_THREADS) k_build_listed(DevState s, long long step, int lds_bytes) {
    extern __shared__ __align__(16) char dyn[];
    const int cnt = s.rb_list[0];
    if (cnt == 0) return;  // nothing listed: nothing to empty either
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
        build_block(s, s.rb_list[2 + i], true, step, lds_bytes, dyn);
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&s.rb_list[1], 1) == (int)gridDim.x - 1) {
            s.rb_list[0] = 0;
            s.rb_list[1] = 0;
        }
    }
}

// One move of one block (Fig. 4): Delete p, Insert it at the target.
//  1. gather p's star; if the target q lies in the star's closed region the
//     only points it can meet are the link vertices, else walk to q;
//  2. blocked (no change) if q is outside the frame or held by a point;
//  3. retriangulate the hole, insert q seeded by a triangle it destroys;
//  4. write the changes back.
// Returns ST_OK (applied or blocked; *applied tells which) or an error, in
// which case memory is unchanged.
// In MV_PLAN mode nothing is written back: the move's records stay in the
// table, *applied is 2 and *plan tells what the move read (the k star slots,
// the table's used entries, the walk path in S.wpath); the caller empties
// the table.  Counters are kept only when st is given.
constexpr int MV_APPLY = 0;
constexpr int MV_PLAN = 1;
struct MovePlan {
    int k, used, npath;  // star slots, table entries, walk slots read
    int nvt_del, nvt;    // incident-triangle updates: the deletion's, then the insertion's
    int2 q;              // the new position
    int fast;            // 1: star-only path
};

template <class WL>
__device__ __forceinline__ int apply_move(BlockView& B, WL& S, const kdt_move_t mv, const int4 fr,
                          BlockStats* st, int* applied, int mode = MV_APPLY, MovePlan* plan = nullptr,
                          bool flip = false) {
    const int lane = lane_id();
    *applied = 0;
    const int p = mv.point, dir = mv.dir, dist = mv.dist;
    if (p < 0 || p >= B.n || dir < 0 || dir > 3 || dist < 1) return ST_ARG;
    const int2 o = B.xy[p];
    const int t0 = B.vtri[p];  // read beside the position: one round trip
    long long qx = o.x, qy = o.y;
    if (dir == 0) qx += dist;
    else if (dir == 1) qx -= dist;
    else if (dir == 2) qy += dist;
    else qy -= dist;
    if (qx < fr.x || qx >= fr.z || qy < fr.y || qy >= fr.w) {
        if (lane == 0 && st) st->blocked += 1;
        return ST_OK;
    }
    const int2 q = make_int2((int)qx, (int)qy);
    const long long c0 = wall_clock64();
    int npath = 0;
    int* path = mode == MV_PLAN ? S.wpath : nullptr;
    int used = 0, nvt = 0;
    const int k = gather_star(B, S, p, t0, &used, st);
    if (k < 0) return k;
    const long long c1 = wall_clock64();
    bool in_star, on_vertex;
    locate_in_star(S, k, o, q, &in_star, &on_vertex);
    if (flip && in_star && !on_vertex) {
        // move-and-flip when q lies inside the kernel of p's star
        int nf = 0;
        const int r = move_and_flip(B, S, k, p, q, &used, &nvt, &nf);
        if (r < 0) return r;  // memory unchanged
        if (r == 1) {
            if (mode == MV_PLAN) {
                if (lane == 0 && st) {  // the plan's counters (kept if it commits)
                    st->flipped += 1;
                    st->flips += nf;
                }
                *plan = MovePlan{k, used, npath, nvt, nvt, q, 0};
                *applied = 2;
                return ST_OK;
            }
            int ndirty = 0;
            for (int base = 0; base < used; base += WAVE)
                ndirty += __popcll(ballot(base + lane < used && (S.tflag[S.tused[base + lane]] & F_DIRTY)));
            commit(B, S, used, nvt, nvt);
            if (lane == 0) B.xy[p] = q;
            const long long c4 = wall_clock64();
            if (lane == 0 && st) {
                const long long dt = c4 - c0;
                st->hist[dt <= 1 ? 0 : min(15, 63 - __clzll(dt))] += 1;
                st->t_star += c1 - c0;
                st->t_hole += c4 - c1;
                st->applied += 1;
                st->flipped += 1;
                st->flips += nf;
                st->tri_touched += used - k;  // records read beyond the star's ring
                // records read and written, incident-triangle updates, move record, position
                st->alg_bytes += 64LL * (used - k) + 64LL * ndirty + 4LL * nvt + 32;
            }
            *applied = 1;
            return ST_OK;
        }
    }
    int hops = 0, tq = -1, kr = k;
    bool in_ring = false;
    if (!in_star) {
        // q in a (closed, real) triangle around the star: no walk
        bool hit = false, occ = false;
        if (lane < k) {
            const Tri t = S.trec[S.out_ent[lane]];
            if (t.v.z != GHOST) {
                const int2 a = cget(t, 0), b = cget(t, 1), c = cget(t, 2);
                hit = orient(a, b, q) >= 0 && orient(b, c, q) >= 0 && orient(c, a, q) >= 0;
                occ = hit && (same(a, q) || same(b, q) || same(c, q));
            }
        }
        const uint64_t hm = ballot(hit);
        if (hm) {
            in_ring = true;
            on_vertex = ballot(occ) != 0;
            tq = S.outref[first_lane(hm)] >> 2;
        } else {
            // walk from the triangle beyond the link edge that the ray from
            // p toward q crosses (any triangle would do; this one is nearest)
            bool sec = false;
            if (lane < k) {
                const int nx = lane + 1 < k ? lane + 1 : 0;
                sec = S.link[lane] != GHOST && S.link[nx] != GHOST && orient(o, S.lxy[lane], q) >= 0 &&
                      orient(o, S.lxy[nx], q) < 0;
            }
            const uint64_t sm = ballot(sec);
            const int start = sm ? (S.outref[first_lane(sm)] >> 2) : S.star_slot[0];
            int hit2;
            tq = walk<false>(B, &S, start, q, &hit2, &hops, path, &npath);
            if (tq < 0) return ST_INTERNAL;
            on_vertex = hit2 >= 0;
        }
    }
    if (on_vertex) {
        table_clear(S);
        if (lane == 0 && st) {
            st->blocked += 1;
            st->walk_sum += hops;
        }
        return ST_OK;
    }
    const long long c2 = wall_clock64();
    // fast path: q inside the star and no triangle around the star
    // destroyed by q -- the star region alone changes -- or q inside the
    // region grown by the destroyed triangles around the star
    bool fast = (in_star || in_ring) && k + 1 <= EMK;
    if (fast) {
        const uint64_t cm = ballot(lane < k && conflicts(S.trec[S.out_ent[lane]], q, p));
        if (cm) {
            kr = grow_region(B, S, k, q, p, cm, &used, !in_star);
            fast = kr > 0;
        } else {
            fast = in_star;  // q in a triangle around the star destroys it
        }
    }
    int rc;
    if (fast) {
        // applied moves write the region straight to memory; a plan keeps it
        // in the table
        rc = fill_star(B, S, kr, p, q, true, &used, &nvt, st, mode == MV_APPLY);
        if (rc != ST_OK) return rc;
        if (mode == MV_PLAN) {
            *plan = MovePlan{k, used, npath, nvt, nvt, q, 1};
            *applied = 2;
            return ST_OK;
        }
        table_drop(S, used);
        if (lane == 0) B.xy[p] = q;
        const long long c4 = wall_clock64();
        if (lane == 0 && st) {
            const long long dt = c4 - c0;
            st->hist[dt <= 1 ? 0 : min(15, 63 - __clzll(dt))] += 1;
            st->t_star += c1 - c0;
            st->t_locate += c2 - c1;
            st->t_hole += c4 - c2;
            st->applied += 1;
            st->fast += 1;
            st->alg_bytes += 16 + 8 + 8;
        }
        *applied = 1;
        return ST_OK;
    }
    rc = fill_star(B, S, k, p, q, false, &used, &nvt, st);
    if (rc != ST_OK) return rc;
    const long long c3 = wall_clock64();
    // where the cavity of q in DT*(S - p) starts: the triangle the walk
    // found (outside the star, so untouched by the deletion), else every
    // hole or surrounding triangle q destroys, else the end of a walk from
    // the hole
    int seed = tq, nseed = 0;
    if (in_star) {
        nseed = seed_cavity(S, k, q, p);
        if (nseed == 0) {
            int hit2;
            seed = walk<true>(B, &S, S.star_slot[0], q, &hit2, &hops, path, &npath);
            if (seed < 0 || hit2 >= 0) return ST_INTERNAL;
        }
    }
    const int nvt_del = nvt;
    rc = insert_vertex(B, S, p, q, seed, nseed, S.star_slot[k - 2], S.star_slot[k - 1], &used, &nvt, st);
    if (rc != ST_OK) return rc;
    if (mode == MV_PLAN) {
        *plan = MovePlan{k, used, npath, nvt_del, nvt, q, 0};
        *applied = 2;
        return ST_OK;
    }
    commit(B, S, used, nvt_del, nvt);
    if (lane == 0) B.xy[p] = q;
    const long long c4 = wall_clock64();
    if (lane == 0 && st) {
        const long long dt = c4 - c0;
        st->hist[dt <= 1 ? 0 : min(15, 63 - __clzll(dt))] += 1;
        st->t_star += c1 - c0;
        st->t_locate += c2 - c1;
        st->t_hole += c3 - c2;
        st->t_insert += c4 - c3;
        st->applied += 1;
        st->walk_sum += hops;
        st->tri_touched += hops;
        // move record, own position, walk records, new position
        st->alg_bytes += 16 + 8 + 64LL * hops + 8;
    }
    *applied = 1;
    return ST_OK;
}

// Position hash of the rebuild branch's dry run, in the wavefront's repair
// scratch (unused on that branch): open addressing on 64-bit cell keys, with
// 0 an empty entry and 1 a vacated cell.  Probes go 64 entries at a time.
constexpr int PH_CAP = 2048;
constexpr unsigned long long PH_EMPTY = 0ull, PH_GONE = 1ull;
__device__ __forceinline__ unsigned long long ph_key(int2 p) {
    return ((((unsigned long long)(unsigned)p.x) << 24) | (unsigned)p.y) + 2ull;
}
__device__ __forceinline__ int ph_home(unsigned long long k) {
    return (int)((k * 0x9E3779B97F4A7C15ull) >> 53) & (PH_CAP - 1);
}
// Entry that holds key k, or -1.  Whole wavefront.
__device__ int ph_find(const unsigned long long* T, unsigned long long k) {
    const int h0 = ph_home(k);
    for (int base = 0; base < PH_CAP; base += WAVE) {
        const int h = (h0 + base + lane_id()) & (PH_CAP - 1);
        const unsigned long long v = T[h];
        const uint64_t hit = ballot(v == k);
        if (hit) return __shfl(h, first_lane(hit));
        if (ballot(v == PH_EMPTY)) return -1;  // entries never become empty again
    }
    return -1;
}
// Insert key k (not present).  Whole wavefront.
__device__ void ph_insert(unsigned long long* T, unsigned long long k) {
    const int h0 = ph_home(k);
    for (int base = 0; base < PH_CAP; base += WAVE) {
        const int h = (h0 + base + lane_id()) & (PH_CAP - 1);
        const unsigned long long v = T[h];
        const uint64_t fr = ballot(v == PH_EMPTY || v == PH_GONE);
        if (fr) {
            if (lane_id() == first_lane(fr)) T[h] = k;
            wsync();
            return;
        }
    }
}
// The n distinct positions, inserted by all lanes at once.
__device__ void ph_build(unsigned long long* T, const int2* xy, int n) {
    for (int h = lane_id(); h < PH_CAP; h += WAVE) T[h] = PH_EMPTY;
    wsync();
    for (int i = lane_id(); i < n; i += WAVE) {
        const unsigned long long k = ph_key(xy[i]);
        int h = ph_home(k);
        for (int t = 0; t < PH_CAP; ++t) {
            if (atomicCAS(&T[h], PH_EMPTY, k) == PH_EMPTY) break;
            h = (h + 1) & (PH_CAP - 1);
        }
    }
    wsync();
}

// Rebuild branch: the block's moves are first checked against the move rule
// (a dry run over the positions: the moved points and their new places are
// kept in LDS, occupancy comes from a position hash when the block is small
// enough, else from a walk in the block's current triangulation, untouched
// until the rebuild); then the new positions are written and the block's
// DT* is rebuilt from scratch.
// The build: here, by this one wavefront, with the block's working state in
// the kernel's dynamic LDS `dynx` when it fits (s.step_lds bytes); else left
// to k_build_listed (defer: the block is listed) or done here in place.
__device__ __forceinline__ int dry_run_and_rebuild(const DevState& s, WaveLDS& S, int b, const kdt_move_t* mv, int m0,
                                   int m1, int8_t* applied, BlockStats* st, bool defer, char* dynx) {
    BlockView B = view_of(s, b);
    const int4 fr = s.frame[b];
    const int lane = lane_id();
    const bool hashed = B.n + (m1 - m0) <= PH_CAP / 2;
    static_assert(sizeof(unsigned long long) * PH_CAP <= DRY_V_OFF, "position hash overlaps the moved points");
    unsigned long long* T = reinterpret_cast<unsigned long long*>(&S);
    int* dry_v = dry_v_of(S);
    int2* dry_q = dry_q_of(S);
    if (hashed) ph_build(T, B.xy, B.n);
    int nmoved = 0;  // wave-uniform; dry_v / dry_q: moved points and their new places
    for (int c0 = m0; c0 < m1; c0 += WAVE) {
        // the chunk's moves and their points' places at the start of the step, one per lane
        kdt_move_t r;
        r.point = 0; r.dir = 0; r.dist = 1; r.pad = 0;
        int2 o0 = make_int2(0, 0);
        bool bad = false;
        if (c0 + lane < m1) {
            r = mv[c0 + lane];
            bad = r.point < 0 || r.point >= B.n || r.dir < 0 || r.dir > 3 || r.dist < 1;
            if (!bad) o0 = B.xy[r.point];
        }
        if (ballot(bad)) return ST_ARG;
        const int cn = min(WAVE, m1 - c0);
        for (int j = 0; j < cn; ++j) {
            const int m = c0 + j;
            const int p = __shfl(r.point, j), dir = __shfl(r.dir, j), dist = __shfl(r.dist, j);
            int2 o = make_int2(__shfl(o0.x, j), __shfl(o0.y, j));
            int prev = -1;  // p's entry in the moved list
            for (int i = lane; i < nmoved; i += WAVE)
                if (dry_v[i] == p) prev = i;
            const uint64_t mp = ballot(prev >= 0);
            prev = mp ? __shfl(prev, first_lane(mp)) : -1;
            if (prev >= 0) o = dry_q[prev];
            long long qx = o.x, qy = o.y;
            if (dir == 0) qx += dist;
            else if (dir == 1) qx -= dist;
            else if (dir == 2) qy += dist;
            else qy -= dist;
            bool ok = qx >= fr.x && qx < fr.z && qy >= fr.y && qy < fr.w;
            const int2 q = make_int2((int)qx, (int)qy);
            if (ok && hashed) {
                ok = ph_find(T, ph_key(q)) < 0;
            } else if (ok) {
                bool held = false;
                for (int i = lane; i < nmoved; i += WAVE) held |= same(dry_q[i], q);
                ok = !ballot(held);
                if (ok) {
                    // a point of the old triangulation at q that has not moved away
                    int hit, hops = 0;
                    const int tq = walk<false>(B, &S, B.vtri[p], q, &hit, &hops);
                    if (tq < 0) return ST_INTERNAL;
                    if (hit >= 0) {
                        bool gone = false;
                        for (int i = lane; i < nmoved; i += WAVE) gone |= dry_v[i] == hit;
                        ok = ballot(gone) != 0;
                    }
                }
            }
            if (ok) {
                const int slot = prev >= 0 ? prev : nmoved;
                if (slot >= DRYMAX) return ST_CAPACITY;
                if (hashed) {
                    const int e = ph_find(T, ph_key(o));
                    if (e < 0) return ST_INTERNAL;
                    if (lane == 0) T[e] = PH_GONE;
                    wsync();
                    ph_insert(T, ph_key(q));
                }
                if (lane == 0) {
                    dry_v[slot] = p;
                    dry_q[slot] = q;
                    st->applied += 1;
                }
                if (prev < 0) ++nmoved;
                wsync();
            } else if (lane == 0) {
                st->blocked += 1;
            }
            if (applied && lane == 0) applied[m] = ok ? 1 : 0;
        }
    }
    for (int i = lane; i < nmoved; i += WAVE) B.xy[dry_v[i]] = dry_q[i];
    gsync();
    if (lane == 0) {
        st->rebuilt += 1;
        st->alg_bytes += 64LL * B.ntri + 12LL * B.n;  // records written, positions read, vtri written
        st->tri_touched += B.ntri;
    }
    const bool in_lds = pb_block_lds(B.n) <= (size_t)s.step_lds;
    if (defer && !in_lds) {
        if (lane == 0) s.rb_list[2 + atomicAdd(&s.rb_list[0], 1)] = b;
        table_clear(S);
        return ST_OK;
    }
    // the attempts overlay the wavefront's repair scratch, unused here
    static_assert(PB_LDS_OFF >= (int)sizeof(int) * WAVE * ATT_B_INTS, "attempts overlap the build's counters");
    PBMem M;
    M.att = reinterpret_cast<int*>(&S);
    if (in_lds) {
        M.tri = reinterpret_cast<Tri*>(dynx);
        M.cown = reinterpret_cast<int*>(M.tri + B.ntri);
        M.bown = M.cown + B.ntri;
        M.vtri = M.bown + B.ntri;
    } else {
        M.tri = B.tri;
        M.vtri = B.vtri;
        M.cown = s.owner + s.tri_off[b];
        M.bown = s.own2 + s.tri_off[b];
    }
    const int rc = pbuild_block(B, s.order + s.pt_off[b], M, pb_lds_of(S));
    table_clear(S);
    return rc;
}

// The branch the policy takes for this block and step: 0 repair, 1 rebuild.
__device__ __forceinline__ int choose_branch(const DevState& s, const float* f) {
    if (s.policy == KDT_POLICY_REBUILD) return 1;
    if (s.policy == KDT_POLICY_THRESHOLD) return f[3] > s.tau ? 1 : 0;
    // the paper's limited distance (Sec. III): a block whose move goes
    // farther than tau * d is rebuilt
    if (s.policy == KDT_POLICY_DLIMIT) return f[15] > s.tau ? 1 : 0;
    if (s.policy != KDT_POLICY_MLP || !s.mlp_w) return 0;
    // 16 -> 32 -> 32 -> 2: hidden unit j on lane j, inputs broadcast
    const int lane = lane_id();
    const float* W = s.mlp_w;
    float h1 = 0.f;
    if (lane < MLP_H) {
        float a = W[MLP_B1 + lane];
        for (int i = 0; i < MLP_IN; ++i) a += W[MLP_W1 + lane * MLP_IN + i] * f[i];
        h1 = a > 0.f ? a : 0.f;
    }
    float a2 = lane < MLP_H ? W[MLP_B2 + lane] : 0.f;
    for (int i = 0; i < MLP_H; ++i) {
        const float hi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, h1), i));
        if (lane < MLP_H) a2 += W[MLP_W2 + lane * MLP_H + i] * hi;
    }
    const float h2 = lane < MLP_H && a2 > 0.f ? a2 : 0.f;
    float o = lane < MLP_OUT ? W[MLP_B3 + lane] : 0.f;
    for (int i = 0; i < MLP_H; ++i) {
        const float hi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, h2), i));
        if (lane < MLP_OUT) o += W[MLP_W3 + lane * MLP_H + i] * hi;
    }
    const float o0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, o), 0));
    const float o1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, o), 1));
    return o1 < o0 ? 1 : 0;
}

// The block's 16 features for this step (whole wavefront; every lane gets
// them), from its size, frame and the distances of moves m0 .. m1-1:
//   0 log2 n          1 k (moves)        2 log2(1+k)        3 sum d/s
//   4 log2(1+sum d/s) 5 max d/s          6 log2(1+max d/s)  7 mean d/s
//   8 #(d > s)        9 #(d > 4s)       10 100 k/n         11 sum (d/s)^2 / k
//  12 log2(1+sum d/s) * log2(1+k)       13 log2 s          14 log2(1+k) / log2 n
//  15 max distance / d, d of the latest d-calculation (0 if none)
//                                        (s = sqrt(frame area / n), d = distance)
__device__ __forceinline__ void block_features(int n, int4 fr, const kdt_move_t* mv, int m0, int m1, float dlim,
                                               float* f) {
    const int lane = lane_id();
    const int k = m1 - m0;
    const float area = (float)(fr.z - fr.x) * (float)(fr.w - fr.y);
    const float sp = sqrtf(area / (float)n);
    float sum = 0.f, mx = 0.f, sq = 0.f, c1 = 0.f, c4 = 0.f;
    for (int m = m0 + lane; m < m1; m += WAVE) {
        const float r = (float)mv[m].dist / sp;
        sum += r;
        mx = fmaxf(mx, r);
        sq += r * r;
        c1 += r > 1.f ? 1.f : 0.f;
        c4 += r > 4.f ? 1.f : 0.f;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sum += __shfl_xor(sum, off);
        mx = fmaxf(mx, __shfl_xor(mx, off));
        sq += __shfl_xor(sq, off);
        c1 += __shfl_xor(c1, off);
        c4 += __shfl_xor(c4, off);
    }
    const float ln = log2f((float)n), lk = log2f(1.f + (float)k);
    f[0] = ln; f[1] = (float)k; f[2] = lk; f[3] = sum; f[4] = log2f(1.f + sum);
    f[5] = mx; f[6] = log2f(1.f + mx); f[7] = sum / (float)k; f[8] = c1; f[9] = c4;
    f[10] = 100.f * (float)k / (float)n; f[11] = sq / (float)k; f[12] = f[4] * lk;
    f[13] = log2f(sp); f[14] = lk / ln; f[15] = dlim > 0.f ? mx * sp / dlim : 0.f;
}

// Warms the caches with what the block's moves of the step read first: lane
// i walks the star of mover i as the step starts (both ways round at once,
// one pair of records per round trip) and touches the triangle beyond each
// link edge (depth 1) and, at depth 2, the triangles beyond those, the
// mover's position and its move record; the values are dropped.  The
// moves, one after another, then find more of their records in cache
// instead of memory.  Read only, with every index checked against the
// block, so a stale or corrupt record only ends the lane's walk.
__device__ __forceinline__ int touch_ring(const BlockView& B, int ring, int depth) {
    if (bad_slot(B, ring)) return 0;
    if (depth < 2) return B.tri[ring].v.x;
    const int4 n = B.tri[ring].n;
    int acc = n.x;
    for (int e = 0; e < 3; ++e) {
        const int r2 = vget(n, e) >> 2;
        if (!bad_slot(B, r2)) acc ^= B.tri[r2].v.x;
    }
    return acc;
}

__device__ __forceinline__ void prefetch_stars(const BlockView& B, const kdt_move_t* __restrict__ mv, int m0,
                                               int m1, int depth) {
    const int lane = lane_id();
    int acc = 0;
    const int m = m0 + lane;
    const int p = m < m1 ? mv[m].point : -1;
    if ((unsigned)p < (unsigned)B.n) {
        const int t0 = B.vtri[p];
        acc ^= B.xy[p].x;
        if (!bad_slot(B, t0)) {
            const int4 v0 = B.tri[t0].v, n0 = B.tri[t0].n;
            const int pi = v0.x == p ? 0 : (v0.y == p ? 1 : (v0.z == p ? 2 : -1));
            if (pi >= 0) {
                int ccw = vget(n0, (pi + 1) % 3), cw = vget(n0, (pi + 2) % 3);
                int ring = vget(n0, pi) >> 2;
                int last_ccw = t0, last_cw = t0;
                for (int it = 0; it < KMAX / 2; ++it) {
                    const int cs = ccw >> 2, ws = cw >> 2;
                    if (cs == last_cw || bad_slot(B, cs) || bad_slot(B, ws)) break;
                    const int4 vc = B.tri[cs].v, nc = B.tri[cs].n, vw = B.tri[ws].v, nw = B.tri[ws].n;
                    acc ^= touch_ring(B, ring, depth);  // the previous round's ring record, in flight with these
                    const int pc = ((ccw & 3) + 1) % 3, pw = ((cw & 3) + 2) % 3;
                    if (vget(vc, pc) != p || vget(vw, pw) != p) break;
                    ring = vget(nc, pc) >> 2;
                    const int ring_w = vget(nw, pw) >> 2;
                    if (ws == cs) break;
                    acc ^= touch_ring(B, ring_w, depth);
                    last_ccw = cs;
                    last_cw = ws;
                    ccw = vget(nc, (pc + 1) % 3);
                    cw = vget(nw, (pw + 2) % 3);
                    if ((cw >> 2) == last_ccw) break;
                }
            }
        }
    }
    asm volatile("" ::"v"(acc));
}

__device__ __forceinline__ int run_block_moves(const DevState& s, WaveLDS& S, int b, const kdt_move_t* mv,
                                const BlockHead& h, int8_t* applied, long long step, bool defer, char* dynx) {
    BlockView B;
    B.tri = s.tri + h.toff;
    B.xy = s.xy + h.p0;
    B.vtri = s.vtri + h.p0;
    B.n = (int)(h.p1 - h.p0);
    B.ntri = 2 * B.n - 2;
    const int4 fr = h.fr;
    const int m0 = h.m0, m1 = h.m1;
    const int lane = lane_id();
    // counters start at zero in LDS and are added to the block's totals at
    // the end (no load of the totals on the way in)
    constexpr int NF = sizeof(BlockStats) / sizeof(long long);
    if (lane < NF) reinterpret_cast<long long*>(&S.st)[lane] = 0;
    wsync();
    const int k = m1 - m0;
    const bool pre = s.choice != nullptr && k > 0;  // chosen (and its features logged) by k_choose
    const bool need_f = k > 0 && !pre && (s.policy != KDT_POLICY_REPAIR || s.log);
    float f[MLP_IN];
    int branch = pre ? s.choice[b] : 0;
    if (need_f) {
        block_features(B.n, fr, mv, m0, m1, s.dlim, f);
        branch = choose_branch(s, f);
    }
    if (k > DRYMAX) branch = 0;  // more moves than the dry run holds: repair
    const long long c0 = wall_clock64();
    int rc = ST_OK;
    if (branch == 0) {
        if (k > 1 && s.prefetch) prefetch_stars(B, mv, m0, m1, s.prefetch);
        for (int m = m0; m < m1; ++m) {
            int app = 0;
            if (m > m0) gsync();  // the previous move's stores are visible
            rc = apply_move(B, S, mv[m], fr, &S.st, &app, MV_APPLY, nullptr, s.repair == KDT_REPAIR_FLIP);
            if (rc == ST_CAPACITY) {
                // beyond the move path's fixed capacities (a star of more than
                // KMAX triangles, a table or a cavity larger than its LDS
                // arrays): the move changed nothing, and the block takes the
                // rebuild branch for its remaining moves of the step, building
                // here (the same DT* from the same positions); the log marks
                // the block-step as neither branch's clean cost
                table_clear(S);
                rc = dry_run_and_rebuild(s, S, b, mv, m, m1, applied, &S.st, false, dynx);
                branch = 2;
                break;
            }
            if (applied && lane == 0) applied[m] = (int8_t)app;
            if (rc != ST_OK) break;
        }
    } else {
        rc = dry_run_and_rebuild(s, S, b, mv, m0, m1, applied, &S.st, defer, dynx);
    }
    const long long c1 = wall_clock64();
    // a failed move or dry run may leave the table (or the rebuild branch's
    // arrays laid over it) in any state: the next block this wavefront takes
    // (persistent launch) must find it empty
    if (rc != ST_OK) table_clear(S);
    wsync();
    if ((need_f || pre) && s.log && s.log_cap > 0 && lane < LOG_FIELDS && !(pre && lane < MLP_IN)) {
        const long long nb = (long long)(s.n_blocks);
        float* rec = s.log + ((step % s.log_cap) * nb + b) * LOG_FIELDS;
        float v = 0.f;
        if (lane < MLP_IN) {
            for (int i = 0; i < MLP_IN; ++i) v = lane == i ? f[i] : v;
        } else if (lane == 16) {
            v = (float)branch;
        } else if (lane == 17) {
            v = (float)(c1 - c0);
        } else if (lane == 18) {
            v = (float)k;
        } else if (lane == 19) {
            v = defer && pb_block_lds(B.n) > (size_t)s.step_lds ? 1.f : 0.f;
        }
        rec[lane] = v;
    }
    if (lane < NF) {
        const long long v = reinterpret_cast<const long long*>(&S.st)[lane];
        if (v) atomicAdd(reinterpret_cast<unsigned long long*>(&s.stats[b]) + lane, (unsigned long long)v);
    }
    if (rc != ST_OK) fail_block(s, b, rc);
    return rc;
}

// The blocks of a step by their number of moves, most first (a counting
// sort; blocks with equal counts in any order, which changes nothing: the
// blocks are independent), for the per-step launches: the blocks that set
// the step's length start first instead of wherever their index puts them.
// order[B] = the number of blocks with at least `cut` moves (the heavy
// class of the split launch: the first order[B] entries), order[B + 1] the
// number with at least `cut2` <= cut (heavy and middle classes).
constexpr int ORD_BUCKETS = DRYMAX + 2;  // k = 0 .. DRYMAX, and more
__device__ __forceinline__ int ord_count(const int* base, int B, int cut) {
    return cut <= 0 ? B : (cut > DRYMAX + 1 ? 0 : base[DRYMAX + 2 - cut]);
}
// One workgroup per step of a chunk (blockIdx.x): the move counts of a
// stream are known ahead, so the orders of several steps are taken in one
// launch, step s's at order + s * (B + 2).
constexpr int ORDER_STEPS = 64;  // steps whose orders one launch takes
__global__ void __launch_bounds__(1024) k_order(const int* __restrict__ step_off, int B, int cut, int cut2,
                                                int* order) {
    __shared__ int cnt[ORD_BUCKETS];
    __shared__ int base[ORD_BUCKETS];
    const int* off = step_off + (long long)blockIdx.x * (B + 1);
    order += (long long)blockIdx.x * (B + 2);
    const int tid = threadIdx.x;
    for (int i = tid; i < ORD_BUCKETS; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    for (int b = tid; b < B; b += blockDim.x) {
        const int k = min(max(off[b + 1] - off[b], 0), DRYMAX + 1);
        atomicAdd(&cnt[DRYMAX + 1 - k], 1);
    }
    __syncthreads();
    if (tid < WAVE) {  // exclusive prefix over the buckets, one wavefront
        int run = 0;
        for (int c0 = 0; c0 < ORD_BUCKETS; c0 += WAVE) {
            const int i = c0 + tid;
            const int v = i < ORD_BUCKETS ? cnt[i] : 0;
            int x = v;
            for (int d = 1; d < WAVE; d <<= 1) {
                const int y = __shfl_up(x, d);
                if (tid >= d) x += y;
            }
            if (i < ORD_BUCKETS) base[i] = run + x - v;
            run += __shfl(x, WAVE - 1);
        }
    }
    __syncthreads();
    if (tid == 0) {
        order[B] = ord_count(base, B, cut);
        order[B + 1] = ord_count(base, B, cut2);
    }
    __syncthreads();
    for (int b = tid; b < B; b += blockDim.x) {
        const int k = min(max(off[b + 1] - off[b], 0), DRYMAX + 1);
        order[atomicAdd(&base[DRYMAX + 1 - k], 1)] = b;
    }
}

// The block a per-step workgroup takes: its index (no order), or its rank
// in the step's order over all blocks (part 0), over the heavy class (part
// 1: ranks below order[B]), the middle class (part 3: ranks order[B] ..
// order[B + 1]) or the light class (part 2: the ranks from order[B + 1]);
// -1: none.
constexpr int PART_ALL = 0, PART_HEAVY = 1, PART_LIGHT = 2, PART_MID = 3;
__device__ __forceinline__ int pick_block(int B, const int* __restrict__ order, int part) {
    const int g = blockIdx.x;
    if (!order) return g < B ? g : -1;
    const int lo = part == PART_LIGHT ? order[B + 1] : (part == PART_MID ? order[B] : 0);
    const int hi = part == PART_HEAVY ? order[B] : (part == PART_MID ? order[B + 1] : B);
    const int r = lo + g;
    return r < hi ? order[r] : -1;
}

// The branch of every block with moves, before the step kernels, for the
// steps blockIdx.y of a chunk starting at step `step` (one wavefront per
// block and step, all at once): the features read only the block's size,
// frame and the step's move distances, so the choices of several steps can
// be taken ahead, off the steps' critical path.  With a log, the chunk is
// one step and the features are logged here.  A failed block, or one
// without moves, repairs (nothing to do).
constexpr int CHOOSE_STEPS = 64;  // steps whose choices one launch takes
__global__ void __launch_bounds__(WAVE) k_choose(DevState s, const kdt_move_t* __restrict__ mv,
                                                 const int* __restrict__ step_off, long long step,
                                                 int8_t* choice) {
    const int b = blockIdx.x;
    const int lane = lane_id();
    const int* off = step_off + (long long)blockIdx.y * (s.n_blocks + 1);
    choice += (long long)blockIdx.y * s.n_blocks;
    step += blockIdx.y;
    const int m0 = off[b], m1 = off[b + 1];
    int branch = 0;
    if (m1 > m0 && s.status[b] == 0) {
        float f[MLP_IN];
        block_features((int)(s.pt_off[b + 1] - s.pt_off[b]), s.frame[b], mv, m0, m1, s.dlim, f);
        branch = choose_branch(s, f);
        if (s.log && s.log_cap > 0 && lane < MLP_IN) {
            float v = 0.f;
            for (int i = 0; i < MLP_IN; ++i) v = lane == i ? f[i] : v;
            s.log[((step % s.log_cap) * (long long)s.n_blocks + b) * LOG_FIELDS + lane] = v;
        }
    }
    if (lane == 0) choice[b] = (int8_t)branch;
}

__global__ void __launch_bounds__(WAVE) k_step(DevState s, const kdt_move_t* __restrict__ mv,
                                               const int* __restrict__ off, int8_t* applied, long long step,
                                               const int* __restrict__ order = nullptr, int part = PART_ALL) {
    __shared__ WaveLDS S;
    extern __shared__ __align__(16) char dynx[];
    const int b = pick_block(s.n_blocks, order, part);
    if (b < 0) return;
    const BlockHead h = load_head(s, b, off);
    if (head_skip(h)) return;
    scratch_init(S);
    run_block_moves(s, S, b, mv, h, applied, step, true, dynx);
}

__global__ void __launch_bounds__(WAVE) k_run_fused(DevState s, const kdt_move_t* __restrict__ mv,
                                                    const int* __restrict__ off, int n_steps, int n_blocks,
                                                    int8_t* applied, long long step0) {
    __shared__ WaveLDS S;
    extern __shared__ __align__(16) char dynx[];
    const int b = blockIdx.x;
    // the status changes from here on only by this wavefront
    BlockHead h = load_head(s, b, off);
    if (h.status != 0) return;
    scratch_init(S);
    for (int t = 0; t < n_steps; ++t) {
        const int* o = off + (long long)t * (n_blocks + 1);
        h.m0 = o[b];
        h.m1 = o[b + 1];
        if (head_skip(h)) continue;
        if (run_block_moves(s, S, b, mv, h, applied, step0 + t, false, dynx) != ST_OK) return;
        gsync();
    }
}

// One time step on a fixed grid of G workgroups (a few per compute unit)
// that share the blocks in the given order -- largest expected cost first --
// without a queue: in round r workgroup w takes rank r*G + w, or r*G + G-1-w
// in odd rounds (each workgroup's blocks alternate between the large and the
// small end of every round, so the totals even out).  A shared counter would
// serialise one atomic per block.
__global__ void __launch_bounds__(WAVE) k_step_persist(DevState s, const kdt_move_t* __restrict__ mv,
                                                       const int* __restrict__ off,
                                                       const int* __restrict__ order, int n_blocks,
                                                       int8_t* applied, long long step) {
    __shared__ WaveLDS S;
    extern __shared__ __align__(16) char dynx[];
    scratch_init(S);
    const int G = gridDim.x, w = blockIdx.x;
    for (int r = 0; r * G < n_blocks; ++r) {
        const int qi = r * G + ((r & 1) ? G - 1 - w : w);
        if (qi >= n_blocks) continue;
        const int b = order[qi];
        const BlockHead h = load_head(s, b, off);
        if (head_skip(h)) continue;
        run_block_moves(s, S, b, mv, h, applied, step, true, dynx);
        gsync();
    }
}

// ------------------------------------------------------------------ global mode
// One triangulation over every point (the whole set is block 0 of the
// state), changed by many wavefronts at once.  A time step:
//   1. k_g_prep, k_g_classify: every move's source and target cell go into a
//      hash of the step's cells.  A move whose cells are named by no other
//      move of the step commutes with all of them: its target is held at its
//      turn in list order exactly when it is held at the start of the step.
//      The other ("interacting") moves wait for the ordered pass.  This holds
//      when every point moves at most once in the step (a second move of a
//      point starts at a cell no start-of-step position names): a step that
//      moves a point twice goes wholly to the ordered pass;
//   2. rounds of k_g_plan / k_g_commit (deterministic reservations): a
//      wavefront plans its move without writing (apply_move, MV_PLAN) and
//      claims every triangle slot the plan read with an atomic maximum of
//      its stamp (round, priority).  After the kernel boundary a wavefront
//      that holds all its claims plans again -- nothing it read has changed,
//      since every writer holds the claims of all it reads and writes -- and
//      commits; the others try again in the next round;
//   3. k_g_serial: the interacting moves and those still pending after the
//      last round, in list order, by one wavefront.
// The result is the sequential rule of the oracle: moves in list order,
// each blocked when its target cell is outside the domain or held.

constexpr int G_ROUNDS = 3;           // reservation rounds per step
constexpr int RSMAX = 384;            // slots a planned move may read
constexpr int PRECMAX = 96;           // records a planned move may write
constexpr int PVTMAX = 128;           // incident-triangle updates of a planned move
constexpr int G_SERIAL_LDS = 2048;    // ordered-pass entries sorted in LDS
constexpr int MS_PEND = 0, MS_DONE = 1, MS_SERIAL = 2;
constexpr int GB_CHUNK = 1 << 17;     // points the grid-wide builder plans at once
constexpr int GB_BIG = 1 << 14;       // cavity capacity of a deferred point's attempt
constexpr int GB_DEFER = 1 << 16;     // deferred points of one build
constexpr int GB_ROUNDS = 64;         // rounds of one chunk before its points are deferred
// g.ctr entries
constexpr int GC_STAMP = 0, GC_REPEAT = 1, GC_SERIAL = 2, GC_USED = 3, GC_PEND = 4, GC_DEFER = 5,
              GC_KIDX = 6, GC_N = 16;

struct GlobalDev {
    unsigned long long* claim;  // per triangle slot: stamp of the highest claim so far
    int* mstate;                // per move of the step: MS_*
    int* rs;                    // per move: the RSMAX slots its plan read
    int* rsn;                   // per move: slots in rs (0: no plan this round)
    int* pslot;                 // per move: the PRECMAX slots its plan writes
    Tri* prec;                  // ... and the records written there
    int2* pvt;                  // per move: PVTMAX incident-triangle updates (point, slot)
    int4* phdr;                 // per move: records, deletion's updates, all updates, star-only
    int2* pq;                   // per move: the new position
    unsigned long long* hkey;   // cell hash: cell key + 1, or 0 when empty
    int* hcnt;                  // moves naming the cell
    int hmask;
    int* ctr;                   // GC_* counters
    int* serial;                // ordered-pass list (move indices, any order)
    const int2* split;          // kd split keys in heap order (root 1)
    int depth;
    // quad-tree cells instead of kd cells (qt = 1): node {x0, y0, log2 side,
    // first of its 4 children or -1}, and for every leaf the node across each
    // side (equal or larger), in move-direction order +x, -x, +y, -y (-1 at
    // the border of the root square)
    int qt;
    int4* qn;
    int4* ql;
    int* qcnt;       // points per node (re-partition)
    int* qlev;       // first node of every level (re-partition, breadth first)
    int qcap;        // nodes the arrays hold
    long long qthr;  // threshold
    int* powner;                // kd cell holding each point
    unsigned long long* gstats; // KDT_GSTAT_* counters
    unsigned long long* part;   // per commit workgroup: applied, star-only, algorithmic bytes, transfers
};
constexpr int G_PART_MAX = 8192;  // commit workgroups the partial counters hold

struct GBuild {
    const int* ord;  // every point, Hilbert order
    int* att;        // GB_CHUNK interleaved attempts
    int* pend;       // per chunk entry: still to insert
    int2* plan;      // per chunk entry: (cavity, boundary) sizes of this round's plan
    int* deferred;   // deferred indices into ord
    int* big;        // the attempt of a deferred point
};

__device__ __forceinline__ void fail_global(const DevState& s, int code) {
    s.status[0] = code;
    atomicMin(s.sticky, code);
}

__device__ __forceinline__ void claim_max(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long claim_get(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Later rounds stamp higher; within a round the smaller priority wins.
__device__ __forceinline__ unsigned long long stamp_of(int round, int prio) {
    return ((unsigned long long)(unsigned)round << 32) | (0xffffffffu - (unsigned)prio);
}

__device__ __forceinline__ unsigned long long cell_key(int2 p) {
    return (((unsigned long long)(unsigned)p.x << 24) | (unsigned)p.y) + 1ull;
}
// A point's key in the same hash (above every cell key): counts the moves
// of the step that move it.
__device__ __forceinline__ unsigned long long point_key(int p) { return (1ull << 56) + (unsigned)p + 1ull; }
__device__ __forceinline__ int cell_slot(unsigned long long k, int mask) {
    return (int)((k * 0x9E3779B97F4A7C15ull) >> 40) & mask;
}
// The table holds at least 8 entries per move, so a free entry is found.
__device__ __forceinline__ void cell_add(const GlobalDev& g, unsigned long long k) {
    int h = cell_slot(k, g.hmask);
    for (int i = 0; i <= g.hmask; ++i) {
        const unsigned long long prev = atomicCAS(&g.hkey[h], 0ull, k);
        if (prev == 0ull || prev == k) {
            atomicAdd(&g.hcnt[h], 1);
            return;
        }
        h = (h + 1) & g.hmask;
    }
}
__device__ __forceinline__ int cell_count(const GlobalDev& g, unsigned long long k) {
    int h = cell_slot(k, g.hmask);
    for (int i = 0; i <= g.hmask; ++i) {
        const unsigned long long cur = g.hkey[h];
        if (cur == k) return g.hcnt[h];
        if (cur == 0ull) return 0;
        h = (h + 1) & g.hmask;
    }
    return 0;
}

__device__ __forceinline__ bool move_target(int2 o, int dir, int dist, int4 fr, int2* q) {
    long long qx = o.x, qy = o.y;
    if (dir == 0) qx += dist;
    else if (dir == 1) qx -= dist;
    else if (dir == 2) qy += dist;
    else qy -= dist;
    const bool in = qx >= fr.x && qx < fr.z && qy >= fr.y && qy < fr.w;
    *q = in ? make_int2((int)qx, (int)qy) : o;
    return in;
}

// kd cell of a position: from the root, right iff its key -- (x, y) at even
// levels, (y, x) at odd ones -- is not below the node's split key.
__device__ __forceinline__ int kd_cell_of(const int2* split, int depth, int2 p) {
    int k = 1;
    for (int l = 0; l < depth; ++l) {
        const int2 sk = split[k];
        const int a = (l & 1) ? p.y : p.x, b = (l & 1) ? p.x : p.y;
        k = 2 * k + ((a > sk.x || (a == sk.x && b >= sk.y)) ? 1 : 0);
    }
    return k - (1 << depth);
}

// The kd cell of position q for a point that was in cell `old`: kept when
// q passes every comparison on the path to `old` (lane l checks level l, one
// round of loads), else found by descending.  Whole wavefront.
__device__ __forceinline__ int owner_after_move(const GlobalDev& g, int old, int2 q) {
    const int lane = lane_id(), D = g.depth;
    bool ok = true;
    if (lane < D) {
        const int k = ((1 << D) + old) >> (D - lane);  // the path's node at level `lane`
        const bool right = (old >> (D - 1 - lane)) & 1;
        const int2 sk = g.split[k];
        const int a = (lane & 1) ? q.y : q.x, b = (lane & 1) ? q.x : q.y;
        ok = (a > sk.x || (a == sk.x && b >= sk.y)) == right;
    }
    if (!ballot(!ok)) return old;
    return kd_cell_of(g.split, D, q);
}

// ---- quad-tree cells (Sec. III "Data structure", Fig. 3)
__device__ __forceinline__ bool qt_contains(int4 nd, int2 q) {
    const int side = 1 << nd.z;
    return q.x >= nd.x && q.x < nd.x + side && q.y >= nd.y && q.y < nd.y + side;
}
// The leaf below `node` (which holds q) that holds q.
__device__ __forceinline__ int qt_descend(const int4* qn, int node, int2 q) {
    int4 nd = qn[node];
    while (nd.w >= 0) {
        const int h = 1 << (nd.z - 1);
        node = nd.w + (q.x >= nd.x + h ? 1 : 0) + (q.y >= nd.y + h ? 2 : 0);
        nd = qn[node];
    }
    return node;
}
// The block (leaf) that receives a point moved to q from leaf `old` in
// direction dir -- "new-block" of Fig. 4: its own leaf, else through the
// direct link to the neighbour on that side (Fig. 3, O(1) when the
// neighbour is a leaf), else down from the root (O(log4 B)); *how = 0, 1, 2.
__device__ __forceinline__ int qt_owner_after_move(const GlobalDev& g, int old, int2 q, int dir, int* how) {
    if (qt_contains(g.qn[old], q)) {
        *how = 0;
        return old;
    }
    const int4 lk = g.ql[old];
    const int nb = dir == 0 ? lk.x : (dir == 1 ? lk.y : (dir == 2 ? lk.z : lk.w));
    if (nb >= 0 && qt_contains(g.qn[nb], q)) {
        *how = 1;
        return qt_descend(g.qn, nb, q);
    }
    *how = 2;
    return qt_descend(g.qn, 0, q);
}
// The cell of a moved point, for either partition; counts how quad-tree
// transfers were routed.
__device__ __forceinline__ int cell_after_move(const GlobalDev& g, int old, int2 q, int dir) {
    if (!g.qt) return owner_after_move(g, old, q);
    int how = 0;
    const int nc = qt_owner_after_move(g, old, q, dir, &how);
    if (how > 0 && lane_id() == 0)
        atomicAdd(&g.gstats[how == 1 ? KDT_GSTAT_LINK : KDT_GSTAT_TREE], 1ull);
    return nc;
}

// ---- Quad-treeDvision on the device (Fig. 4, step 5): the quad-tree of
// the current positions from scratch, breadth first.  Level l's nodes are
// qlev[l] .. qlev[l+1]-1; a node holding more than the threshold (and wider
// than one lattice cell) gets its four quarters at the end of level l+1,
// in node order (a scan), and then every point in it moves one level down.
constexpr int QT_LEVELS = 26;
__global__ void k_qt_reset(GlobalDev g, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) g.powner[p] = 0;
    if (p == 0) {
        g.qcnt[0] = n;
        g.qn[0].w = -1;
        g.qlev[0] = 0;
        g.qlev[1] = 1;
    }
}
// One workgroup: the children of level `lvl`'s nodes.  qlev[lvl + 2] and the
// count of nodes cut (in qlev[QT_LEVELS]) for the host; a level beyond the
// arrays' capacity cuts nothing and reports -1.
__global__ void __launch_bounds__(1024) k_qt_alloc(GlobalDev g, int lvl) {
    __shared__ int wsum[16];
    __shared__ int base;
    const int k0 = g.qlev[lvl], k1 = g.qlev[lvl + 1];
    const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
    if (t == 0) base = 0;
    __syncthreads();
    bool room = true;
    for (int c0 = k0; c0 < k1; c0 += 1024) {
        const int k = c0 + t;
        const int4 nd = k < k1 ? g.qn[k] : make_int4(0, 0, 0, -1);
        const bool cut = k < k1 && g.qcnt[k] > g.qthr && nd.z > 0;
        const uint64_t m = ballot(cut);
        if (lane == 0) wsum[wv] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int i = 0; i < 16; ++i) {
            before += i < wv ? wsum[i] : 0;
            total += wsum[i];
        }
        const int idx = base + before + lanes_below(m);
        const int c = k1 + 4 * idx;
        if (cut && c + 4 <= g.qcap) {
            g.qn[k].w = c;
            const int h = 1 << (nd.z - 1);
            for (int q = 0; q < 4; ++q) {
                g.qn[c + q] = make_int4(nd.x + (q & 1) * h, nd.y + (q >> 1) * h, nd.z - 1, -1);
                g.qcnt[c + q] = 0;
            }
        } else if (cut) {
            room = false;
        }
        __syncthreads();
        if (t == 0) base += total;
        __syncthreads();
    }
    const bool full = __syncthreads_or(!room);
    if (t == 0) {
        g.qlev[lvl + 2] = k1 + 4 * base;
        g.qlev[QT_LEVELS] = full ? -1 : base;
    }
}
__global__ void k_qt_down(const DevState s, GlobalDev g, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int cur = g.powner[p];
    const int4 nd = g.qn[cur];
    if (nd.w < 0) return;
    const int2 q = s.xy[p];
    const int h = 1 << (nd.z - 1);
    const int c = nd.w + (q.x >= nd.x + h ? 1 : 0) + (q.y >= nd.y + h ? 2 : 0);
    g.powner[p] = c;
    atomicAdd(&g.qcnt[c], 1);
}
// The node across each side of every leaf (equal or larger), or -1.
__device__ __forceinline__ int qt_probe_dev(const int4* qn, long long px, long long py, int lg) {
    const int4 r = qn[0];
    const long long side = 1ll << r.z;
    if (px < r.x || py < r.y || px >= r.x + side || py >= r.y + side) return -1;
    int node = 0;
    int4 nd = r;
    while (nd.w >= 0 && nd.z > lg) {
        const long long h = 1ll << (nd.z - 1);
        node = nd.w + (px >= nd.x + h ? 1 : 0) + (py >= nd.y + h ? 2 : 0);
        nd = qn[node];
    }
    return node;
}
__global__ void k_qt_links(GlobalDev g, int nodes) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nodes) return;
    const int4 nd = g.qn[k];
    if (nd.w >= 0) {
        g.ql[k] = make_int4(-1, -1, -1, -1);
        return;
    }
    const long long side = 1ll << nd.z;
    g.ql[k] = make_int4(qt_probe_dev(g.qn, nd.x + side, nd.y, nd.z), qt_probe_dev(g.qn, nd.x - 1ll, nd.y, nd.z),
                        qt_probe_dev(g.qn, nd.x, nd.y + side, nd.z), qt_probe_dev(g.qn, nd.x, nd.y - 1ll, nd.z));
}

__device__ __forceinline__ void stats_zero(WaveLDS& S) {
    constexpr int NF = sizeof(BlockStats) / sizeof(long long);
    if (lane_id() < NF) reinterpret_cast<long long*>(&S.st)[lane_id()] = 0;
    wsync();
}
__device__ __forceinline__ void stats_flush(const DevState& s, WaveLDS& S) {
    constexpr int NF = sizeof(BlockStats) / sizeof(long long);
    wsync();
    if (lane_id() < NF) {
        const long long v = reinterpret_cast<const long long*>(&S.st)[lane_id()];
        if (v) atomicAdd(reinterpret_cast<unsigned long long*>(&s.stats[0]) + lane_id(), (unsigned long long)v);
    }
}

// Round r of a step (or of a chunk of a build) stamps its claims with
// ctr[GC_STAMP] + r; the base advances past the rounds once they are done.
__global__ void k_add(int* p, int v) { *p += v; }

__global__ void k_set(int* p, int v) { *p = v; }


__global__ void k_g_prep(DevState s, GlobalDev g, const kdt_move_t* __restrict__ mv, int M,
                         int8_t* applied) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    // loads and the hash insertions (which wait for their old values) come
    // before this thread's plain stores: a load issued after a store waits
    // for that store
    const kdt_move_t r = mv[m];
    const bool bad = r.point < 0 || r.point >= (int)s.pt_off[1] || r.dir < 0 || r.dir > 3 || r.dist < 1;
    if (!bad) {
        const int2 o = s.xy[r.point];
        int2 q;
        cell_add(g, cell_key(o));
        if (move_target(o, r.dir, r.dist, s.frame[0], &q)) cell_add(g, cell_key(q));
        cell_add(g, point_key(r.point));
    }
    g.rsn[m] = 0;
    if (applied) applied[m] = 0;
    g.mstate[m] = bad ? MS_DONE : MS_PEND;
    if (bad) fail_global(s, ST_ARG);
}

__global__ void k_g_classify(DevState s, GlobalDev g, const kdt_move_t* __restrict__ mv, int M) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || g.mstate[m] != MS_PEND) return;
    const kdt_move_t r = mv[m];
    // a point moved twice in the step: its second move starts where the
    // first ended, a cell the hash does not name -- the whole step runs in
    // list order (the ordered pass)
    if (cell_count(g, point_key(r.point)) > 1) g.ctr[GC_REPEAT] = 1;
    const int2 o = s.xy[r.point];
    int2 q;
    if (!move_target(o, r.dir, r.dist, s.frame[0], &q)) {  // outside the domain: blocked
        g.mstate[m] = MS_DONE;
        atomicAdd(reinterpret_cast<unsigned long long*>(&s.stats[0].blocked), 1ull);
        return;
    }
    if (cell_count(g, cell_key(o)) > 1 || cell_count(g, cell_key(q)) > 1) {
        g.mstate[m] = MS_SERIAL;
        g.serial[atomicAdd(&g.ctr[GC_SERIAL], 1)] = m;
        atomicAdd(&g.gstats[KDT_GSTAT_INTERACTING], 1ull);
    }
}

// Plans (the global mode's rounds and the multi-wavefront rounds) use a
// write-back table of PLAN_HT entries: a plan that needs more goes to the
// sequential path, which has the full table; two thirds of a step
// wavefront's LDS, so more planning wavefronts share a compute unit.
constexpr int PLAN_HT = 128;
using PlanWave = WaveLDST<PLAN_HT>;

__global__ void __launch_bounds__(WAVE) k_g_plan(DevState s, GlobalDev g,
                                                 const kdt_move_t* __restrict__ mv, int M, int round) {
    __shared__ PlanWave S;
    const int lane = lane_id();
    BlockView B = view_of(s, 0);
    if (round == 0) {  // the step's cell hash has been read: empty it for the next step
        for (int h = blockIdx.x * WAVE + lane; h <= g.hmask; h += gridDim.x * WAVE) {
            g.hkey[h] = 0ull;
            g.hcnt[h] = 0;
        }
    }
    // a step that moves a point twice runs wholly in the ordered pass: no
    // plan, so the last round hands every pending move on
    if (g.ctr[GC_REPEAT]) return;
    // a fixed grid strides over the step's moves (later rounds have few left)
    for (int m = blockIdx.x; m < M; m += gridDim.x) {
        if (g.mstate[m] != MS_PEND || s.status[0] != 0) continue;
        scratch_init(S);
        MovePlan pl{};
        int app = 0;
        const int rc = apply_move(B, S, mv[m], s.frame[0], nullptr, &app, MV_PLAN, &pl);
        if (rc != ST_OK) {
            if (lane == 0) {
                g.mstate[m] = MS_DONE;
                fail_global(s, rc);
            }
            continue;
        }
        if (app == 0) {  // target held by a point that stays put this step
            if (lane == 0) {
                g.mstate[m] = MS_DONE;
                atomicAdd(reinterpret_cast<unsigned long long*>(&s.stats[0].blocked), 1ull);
            }
            continue;
        }
        // the records the plan changed (table entries marked dirty)
        int ndirty = 0;
        for (int base = 0; base < pl.used; base += WAVE) {
            const int u = base + lane;
            ndirty += __popcll(ballot(u < pl.used && (S.tflag[S.tused[u]] & F_DIRTY)));
        }
        const int total = pl.k + pl.used + pl.npath;
        if (pl.npath > WPMAX || total > RSMAX || ndirty > PRECMAX || pl.nvt > PVTMAX) {
            if (lane == 0) {
                g.mstate[m] = MS_SERIAL;
                g.serial[atomicAdd(&g.ctr[GC_SERIAL], 1)] = m;
                atomicAdd(&g.gstats[KDT_GSTAT_OVERFLOW], 1ull);
            }
            continue;
        }
        // claim every slot read; keep the plan's writes for the commit
        const unsigned long long stamp = stamp_of(g.ctr[GC_STAMP] + round, pb_prio(m));
        int* out = g.rs + (long long)m * RSMAX;
        for (int i = lane; i < total; i += WAVE) {
            const int slot = i < pl.k ? S.star_slot[i]
                                      : (i < pl.k + pl.used ? S.tkey[S.tused[i - pl.k]] : S.wpath[i - pl.k - pl.used]);
            out[i] = slot;
            claim_max(&g.claim[slot], stamp);
        }
        int* ps = g.pslot + (long long)m * PRECMAX;
        Tri* pr = g.prec + (long long)m * PRECMAX;
        int nrec = 0;
        for (int base = 0; base < pl.used; base += WAVE) {
            const int u = base + lane;
            const int h = u < pl.used ? S.tused[u] : 0;
            const bool d = u < pl.used && (S.tflag[h] & F_DIRTY);
            const uint64_t dm = ballot(d);
            if (d) {
                const int r = nrec + lanes_below(dm);
                ps[r] = S.tkey[h];
                pr[r] = S.trec[h];
            }
            nrec += __popcll(dm);
        }
        int2* pv = g.pvt + (long long)m * PVTMAX;
        for (int i = lane; i < pl.nvt; i += WAVE) pv[i] = make_int2(S.vt_v[i], S.vt_s[i]);
        if (lane == 0) {
            g.phdr[m] = make_int4(nrec, pl.nvt_del, pl.nvt, pl.fast);
            g.pq[m] = pl.q;
            g.rsn[m] = total;
        }
        wsync();
    }
}

// A move that holds every claim of its plan writes the plan out: nothing the
// plan read has changed since (every writer holds the claims of all it reads
// and writes), so the recorded records are still the right ones.
__global__ void __launch_bounds__(WAVE) k_g_commit(DevState s, GlobalDev g,
                                                   const kdt_move_t* __restrict__ mv, int M, int round,
                                                   int last, int8_t* applied) {
    const int lane = lane_id();
    long long n_app = 0, n_fast = 0, n_alg = 0, n_tr = 0;
    for (int m = blockIdx.x; m < M; m += gridDim.x) {
        if (g.mstate[m] != MS_PEND || s.status[0] != 0) continue;
        const int nrs = g.rsn[m];
        const unsigned long long stamp = stamp_of(g.ctr[GC_STAMP] + round, pb_prio(m));
        const int* in = g.rs + (long long)m * RSMAX;
        bool held = nrs > 0;
        for (int i = lane; i < nrs; i += WAVE) held &= claim_get(&g.claim[in[i]]) == stamp;
        const bool won = nrs > 0 && !ballot(!held && lane < nrs);
        if (won) {
            BlockView B = view_of(s, 0);
            const int4 h = g.phdr[m];
            const int* ps = g.pslot + (long long)m * PRECMAX;
            const Tri* pr = g.prec + (long long)m * PRECMAX;
            const int2* pv = g.pvt + (long long)m * PVTMAX;
            for (int i = lane; i < h.x; i += WAVE) B.tri[ps[i]] = pr[i];
            // the deletion's updates, then the insertion's (a point in both
            // gets the later value: one wavefront's stores to one address
            // land in program order)
            for (int i = lane; i < h.y; i += WAVE)
                if (pv[i].x != GHOST) B.vtri[pv[i].x] = pv[i].y;
            for (int i = h.y + lane; i < h.z; i += WAVE)
                if (pv[i].x != GHOST) B.vtri[pv[i].x] = pv[i].y;
            const int p = mv[m].point;
            const int2 q = g.pq[m];
            const int oc = g.powner[p];
            const int nc = cell_after_move(g, oc, q, mv[m].dir);
            if (lane == 0) {
                B.xy[p] = q;
                if (nc != oc) g.powner[p] = nc;
                if (applied) applied[m] = 1;
                g.mstate[m] = MS_DONE;
            }
            // counted per workgroup, added up by the ordered pass (one
            // atomic per move on a shared counter would serialise)
            n_app += 1;
            n_fast += h.w ? 1 : 0;
            n_alg += 64LL * (nrs + h.x) + 4LL * h.z + 32;  // records read and written, updates, move
            n_tr += nc != oc ? 1 : 0;
        } else if (lane == 0) {
            g.rsn[m] = 0;
            atomicAdd(&g.gstats[KDT_GSTAT_LOST], 1ull);
            if (last) {
                g.mstate[m] = MS_SERIAL;
                g.serial[atomicAdd(&g.ctr[GC_SERIAL], 1)] = m;
            }
        }
    }
    if (lane == 0 && blockIdx.x < G_PART_MAX && (n_app | n_tr)) {
        unsigned long long* pp = g.part + 4 * blockIdx.x;
        pp[0] += n_app;
        pp[1] += n_fast;
        pp[2] += n_alg;
        pp[3] += n_tr;
    }
}

__global__ void __launch_bounds__(WAVE) k_g_serial(DevState s, GlobalDev g,
                                                   const kdt_move_t* __restrict__ mv, int M,
                                                   int8_t* applied, int parts) {
    __shared__ WaveLDS S;
    __shared__ int tmp[G_SERIAL_LDS], list[G_SERIAL_LDS];
    const int lane = lane_id();
    const int cnt = g.ctr[GC_SERIAL];
    scratch_init(S);
    stats_zero(S);
    BlockView B = view_of(s, 0);
    const int4 fr = s.frame[0];
    auto one = [&](int m) {
        int app = 0;
        const int p = mv[m].point;
        const int oc = g.powner[p];
        const int rc = apply_move(B, S, mv[m], fr, &S.st, &app);
        gsync();  // the new position is visible to every lane
        const int nc = rc == ST_OK && app ? cell_after_move(g, oc, s.xy[p], mv[m].dir) : oc;
        if (lane == 0) {
            if (rc != ST_OK) fail_global(s, rc);
            if (nc != oc) {
                g.powner[p] = nc;
                atomicAdd(&g.gstats[KDT_GSTAT_TRANSFERS], 1ull);
            }
            if (applied) applied[m] = (int8_t)app;
            g.mstate[m] = MS_DONE;
        }
        gsync();  // this move's stores are visible to the next
        return rc;
    };
    if (s.status[0] == 0 && cnt > 0) {
        if (cnt <= G_SERIAL_LDS) {
            // list order: an entry's rank is the number of smaller entries
            for (int i = lane; i < cnt; i += WAVE) tmp[i] = g.serial[i];
            wsync();
            for (int i = lane; i < cnt; i += WAVE) {
                const int v = tmp[i];
                int r = 0;
                for (int j = 0; j < cnt; ++j) r += tmp[j] < v ? 1 : 0;
                list[r] = v;
            }
            wsync();
            for (int i = 0; i < cnt; ++i) {
                const int m = list[i];
                if (m < 0 || m >= M) {  // the list names each move at most once
                    if (lane == 0) fail_global(s, ST_INTERNAL);
                    break;
                }
                if (one(m) != ST_OK) break;
            }
        } else {
            bool ok = true;
            for (int base = 0; base < M && ok; base += WAVE) {
                uint64_t mask = ballot(base + lane < M && g.mstate[base + lane] == MS_SERIAL);
                while (mask && ok) {
                    const int j = first_lane(mask);
                    mask &= mask - 1;
                    ok = one(base + j) == ST_OK;
                }
            }
        }
        if (lane == 0) atomicAdd(&g.gstats[KDT_GSTAT_SERIAL], (unsigned long long)cnt);
    }
    // the commit rounds' per-workgroup counters: all read first, then
    // cleared (a load issued after a store waits for that store, so
    // interleaving them would cost a round trip per group of 64)
    long long a = 0, f = 0, b = 0, t = 0;
#pragma unroll 4
    for (int w = lane; w < parts; w += WAVE) {
        const ulonglong2 p01 = *reinterpret_cast<const ulonglong2*>(g.part + 4 * w);
        const ulonglong2 p23 = *reinterpret_cast<const ulonglong2*>(g.part + 4 * w + 2);
        a += (long long)p01.x;
        f += (long long)p01.y;
        b += (long long)p23.x;
        t += (long long)p23.y;
    }
    wsync();
    for (int w = lane; w < parts; w += WAVE) {
        *reinterpret_cast<ulonglong2*>(g.part + 4 * w) = make_ulonglong2(0ull, 0ull);
        *reinterpret_cast<ulonglong2*>(g.part + 4 * w + 2) = make_ulonglong2(0ull, 0ull);
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        f += __shfl_xor(f, off);
        b += __shfl_xor(b, off);
        t += __shfl_xor(t, off);
    }
    if (lane == 0) {
        S.st.applied += a;
        S.st.fast += f;
        S.st.alg_bytes += b;
        if (t) atomicAdd(&g.gstats[KDT_GSTAT_TRANSFERS], (unsigned long long)t);
    }
    stats_flush(s, S);
    if (lane == 0) {
        g.ctr[GC_SERIAL] = 0;
        g.ctr[GC_REPEAT] = 0;
        g.ctr[GC_STAMP] += G_ROUNDS;  // past this step's rounds
    }
}

// ------------------------------------------------------------------ several wavefronts per block
// A block's moves in one time step, shared by the NW wavefronts of one
// workgroup (per-step launch with block_waves = NW > 1).  A step of a block
// with k moves is otherwise as long as k moves one after another on one
// wavefront, and the blocks with the most moves set the step's length.
//
// When no point moves twice in the block's step, the moves whose source and
// target cells are named by no other move of the step commute with every
// other move: each is blocked exactly when its target cell is held at the
// start of the step, whatever the order, and changes no cell another move
// names.  (A point that moves twice starts its second move where the first
// ended, which no start-of-step cell tells: such a block runs its moves in
// list order.)
// They are applied in reservation rounds: each wavefront takes the next
// pending one (in list order), plans it without writing (apply_move in plan
// mode: the star, every record the repair reads, the walk's path, all in
// the wavefront's table), and claims every slot it read in an LDS hash with
// its move index; after a barrier, a plan whose every slot is claimed by no
// lower move index commits (its table goes to memory) -- the winners have
// disjoint read sets, and every record a move writes is one it read, so
// nothing a winner read has changed -- and the others plan again in the next
// round.  The lowest pending move always wins.  Every other move (moves that
// share a cell with another, a plan beyond the plan or table capacities,
// every move of a block that takes the rebuild branch or has more moves than
// MW_KMAX) goes, in list order, to the block's rest list, which k_step_rest
// applies after the rounds one after another (the sequential path).  The
// commuting moves commute with them too, so the result is the sequential
// rule's, and DT* (unique) is the same triangulation.
constexpr int MW_MAX_WAVES = 4;
// The rounds' wavefronts plan with a write-back table of MW_HT entries (a
// move that needs more -- a long walk, a large cavity; the star-only moves
// take a few dozen -- goes to the rest list, whose sequential path has the
// full table): about half the LDS of a step wavefront's, so that four
// two-wavefront workgroups, or two four-wavefront ones, share a compute
// unit.  A plan then reads at most MW_RSMAX slots: its star, its table
// entries, its walk.
constexpr int MW_HT = 64;
using MwWave = WaveLDST<MW_HT>;
constexpr int MW_RSMAX = KMAX + MW_HT + WPMAX;
// claim hash entries: every slot of one round's NW plans (a power of two)
template <int NW>
constexpr int mw_hash() { return NW * MW_RSMAX <= 512 ? 512 : (NW * MW_RSMAX <= 1024 ? 1024 : 2048); }
static_assert(mw_hash<MW_MAX_WAVES>() >= MW_MAX_WAVES * MW_RSMAX && mw_hash<2>() >= 2 * MW_RSMAX,
              "claim hash smaller than the plans of one round");
constexpr int MW_KMAX = 64;  // moves of a block's step the rounds take; a block with more runs in the rest launch
constexpr int MWS_PEND = 0, MWS_DONE = 1, MWS_REST = 2;
constexpr int REST_ALL = -1;  // rest count of a block deferred whole

// The rest lists: per block up to DRYMAX moves (copies, list order) with
// their index in the step's move array; applied flags land in rest_app.
struct RestBuf {
    kdt_move_t* mv;  // [B][DRYMAX]
    int* idx;        // [B][DRYMAX]
    int8_t* app;     // [B][DRYMAX]
    int* cnt;        // [B]
};

template <int NW>
struct MwLDS {
    MwWave S[NW];
    BlockStats pst[NW];          // the counters of each wavefront's current plan
    int hkey[mw_hash<NW>()];     // slot, or -1
    int hprio[mw_hash<NW>()];    // lowest move index claiming it
    int mstate[MW_KMAX];         // MWS_* per move of the step (offset from m0)
    int list[MW_KMAX];           // pending commuting moves, list order
    int2 cs[MW_KMAX], ct[MW_KMAX];  // source and target cells (ct.x < 0: target outside the frame)
    int pt[MW_KMAX];             // moved point
    int outcome[NW];
    int np, head, defer_all, fail, nrest;  // pending moves: list[head .. np)
    float f[MLP_IN];
};

template <int H>
__device__ __forceinline__ int mw_home(int slot) {
    static_assert(H == 512 || H == 1024 || H == 2048, "claim hash size");
    return (int)(((unsigned)slot * 0x9E3779B1u) >> (32 - __builtin_ctz(H)));
}

// Slot i of a plan's read set: the star, then the table's entries, then the
// walk's path.
__device__ __forceinline__ int mw_read_slot(const MwWave& S, const MovePlan& pl, int i) {
    return i < pl.k ? S.star_slot[i] : (i < pl.k + pl.used ? S.tkey[S.tused[i - pl.k]] : S.wpath[i - pl.k - pl.used]);
}

static_assert(sizeof(MwLDS<4>) <= 160 * 1024, "four wavefronts' scratch exceeds a compute unit's LDS");
static_assert(4 * sizeof(MwLDS<2>) <= 160 * 1024, "four two-wavefront workgroups no longer share a compute unit");
static_assert(2 * sizeof(MwLDS<4>) <= 160 * 1024, "two four-wavefront workgroups no longer share a compute unit");

template <int NW>
__global__ void __launch_bounds__(NW * WAVE) k_step_mw(DevState s, const kdt_move_t* __restrict__ mv,
                                                       const int* __restrict__ off, int8_t* applied,
                                                       long long step, RestBuf rb,
                                                       const int* __restrict__ order = nullptr,
                                                       int part = PART_ALL) {
    extern __shared__ __align__(16) char dyn[];
    MwLDS<NW>& M = *reinterpret_cast<MwLDS<NW>*>(dyn);
    constexpr int HS = mw_hash<NW>();
    const int b = pick_block(s.n_blocks, order, part);
    if (b < 0) return;  // uniform over the workgroup
    const int tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
    constexpr int NT = NW * WAVE;
    const BlockHead h = load_head(s, b, off);
    if (head_skip(h)) return;  // uniform over the workgroup
    BlockView B;
    B.tri = s.tri + h.toff;
    B.xy = s.xy + h.p0;
    B.vtri = s.vtri + h.p0;
    B.n = (int)(h.p1 - h.p0);
    B.ntri = 2 * B.n - 2;
    const int4 fr = h.fr;
    const int m0 = h.m0, k = h.m1 - h.m0;
    constexpr int NF = sizeof(BlockStats) / sizeof(long long);
    MwWave& S = M.S[w];
    table_clear(S);
    if (lane < NF) reinterpret_cast<long long*>(&S.st)[lane] = 0;
    if (tid == 0) {
        M.defer_all = k > MW_KMAX ? 1 : 0;
        M.fail = ST_OK;
        M.np = 0;
        M.head = 0;
    }
    for (int i = tid; i < HS; i += NT) {
        M.hkey[i] = -1;
        M.hprio[i] = 0x7fffffff;
    }
    const bool pre = s.choice != nullptr;  // chosen (and its features logged) by k_choose
    const bool need_f = !pre && (s.policy != KDT_POLICY_REPAIR || s.log);
    __syncthreads();
    // wavefront 0 chooses the branch while the others warm the caches with
    // the movers' stars (a read-only hint, whatever the branch)
    if (w == 0) {
        if (pre) {
            if (lane == 0 && k > 0 && s.choice[b] != 0) M.defer_all = 1;  // the rebuild branch runs in k_step_rest
        } else if (need_f && !M.defer_all) {
            float f[MLP_IN];
            block_features(B.n, fr, mv, m0, h.m1, s.dlim, f);
            const int br = choose_branch(s, f);
            if (lane == 0) {
                if (br != 0) M.defer_all = 1;  // the rebuild branch runs in k_step_rest
                for (int i = 0; i < MLP_IN; ++i) M.f[i] = f[i];
            }
        }
    } else if (k > 1 && k <= MW_KMAX && s.prefetch) {
        prefetch_stars(B, mv, m0 + (w - 1) * WAVE, h.m1, s.prefetch);
    }
    __syncthreads();
    const long long c0 = wall_clock64();
    if (!M.defer_all) {
        // the moves' cells at the start of the step
        for (int i = tid; i < k; i += NT) {
            const kdt_move_t r = mv[m0 + i];
            const bool bad = r.point < 0 || r.point >= B.n || r.dir < 0 || r.dir > 3 || r.dist < 1;
            int2 o = make_int2(-1, -1 - i), q = make_int2(-1, -1);
            if (!bad) {
                o = B.xy[r.point];
                if (!move_target(o, r.dir, r.dist, fr, &q)) q = make_int2(-1, -1);
            } else {
                M.defer_all = 1;  // the sequential path reports the error
            }
            M.pt[i] = bad ? -1 - i : r.point;
            M.cs[i] = o;
            M.ct[i] = q;
        }
        __syncthreads();
        for (int i = tid; i < k; i += NT) {
            const int2 a = M.cs[i], t = M.ct[i];
            bool inter = false, again = false;
            for (int j = 0; j < k; ++j) {
                if (j == i) continue;
                const int2 a2 = M.cs[j], t2 = M.ct[j];
                again |= M.pt[j] == M.pt[i];
                inter |= same(a, a2) || (t.x >= 0 && (same(t, a2) || same(t, t2))) || (t2.x >= 0 && same(a, t2));
            }
            M.mstate[i] = inter ? MWS_REST : MWS_PEND;
            // a point that moves twice starts its second move where the first
            // ended, a cell the cells above do not name: the block's moves all
            // run in list order
            if (again) M.defer_all = 1;
        }
        __syncthreads();
        if (w == 0) {  // the pending moves in list order (k <= MW_KMAX = one wavefront)
            static_assert(MW_KMAX <= WAVE, "the pending list is compacted by one ballot");
            const bool pend = lane < k && M.mstate[lane] == MWS_PEND;
            const uint64_t pm = ballot(pend);
            if (pend) M.list[lanes_below(pm)] = lane;
            if (lane == 0) M.np = __popcll(pm);
        }
    }
    __syncthreads();
    // reservation rounds over the commuting moves
    while (!M.defer_all && M.np > M.head && M.fail == ST_OK) {
        const int head = M.head, np = M.np;
        const int i = w < np - head ? M.list[head + w] : -1;  // offset of this wavefront's move
        MovePlan pl{};
        int app = 0, rc = ST_OK, total = 0;
        if (i >= 0) {
            if (lane < NF) reinterpret_cast<long long*>(&M.pst[w])[lane] = 0;
            wsync();
            rc = apply_move(B, S, mv[m0 + i], fr, &M.pst[w], &app, MV_PLAN, &pl, s.repair == KDT_REPAIR_FLIP);
            if (rc == ST_OK && app == 2) {
                total = pl.k + pl.used + pl.npath;
                if (pl.npath > WPMAX || total > MW_RSMAX) {
                    rc = ST_CAPACITY;  // too large to reserve: the sequential path takes it
                } else {
                    for (int e = lane; e < total; e += WAVE) {
                        const int slot = mw_read_slot(S, pl, e);
                        int hh = mw_home<HS>(slot);
                        for (int t = 0; t < HS; ++t) {
                            const int old = atomicCAS(&M.hkey[hh], -1, slot);
                            if (old == -1 || old == slot) {
                                atomicMin(&M.hprio[hh], i);
                                break;
                            }
                            hh = (hh + 1) & (HS - 1);
                        }
                    }
                }
            }
        }
        __syncthreads();
        int outc = -1;  // 0 blocked, 1 won, 2 lost, 3 rest, < 0 error
        if (i >= 0) {
            if (rc == ST_CAPACITY) {
                outc = 3;
            } else if (rc != ST_OK) {
                outc = rc;
            } else if (app == 0) {
                outc = 0;
            } else {
                bool held = true;
                for (int e = lane; e < total; e += WAVE) {
                    const int slot = mw_read_slot(S, pl, e);
                    int hh = mw_home<HS>(slot);
                    for (int t = 0; t < HS && M.hkey[hh] != slot; ++t) hh = (hh + 1) & (HS - 1);
                    held &= M.hprio[hh] == i;
                }
                outc = ballot(!held) ? 2 : 1;
            }
        }
        __syncthreads();  // every wavefront has read the claims
        for (int e = tid; e < HS; e += NT) {
            M.hkey[e] = -1;
            M.hprio[e] = 0x7fffffff;
        }
        if (outc == 1) {
            commit(B, S, pl.used, pl.nvt_del, pl.nvt);
            if (lane == 0) {
                B.xy[mv[m0 + i].point] = pl.q;
                if (applied) applied[m0 + i] = 1;
                const BlockStats& P = M.pst[w];
                S.st.star_sum += P.star_sum;
                S.st.cavity_sum += P.cavity_sum;
                S.st.walk_sum += P.walk_sum;
                S.st.tri_touched += P.tri_touched + pl.npath;
                // move record, own position read and written, walk records
                S.st.alg_bytes += P.alg_bytes + 32 + 64LL * pl.npath;
                S.st.applied += 1;
                S.st.fast += pl.fast;
                S.st.flipped += P.flipped;
                S.st.flips += P.flips;
            }
        } else if (i >= 0) {
            if (app == 2) table_drop(S, pl.used);
            else table_clear(S);
            if (outc == 0 && lane == 0) {
                if (applied) applied[m0 + i] = 0;
                S.st.blocked += M.pst[w].blocked;
                S.st.walk_sum += M.pst[w].walk_sum;
            }
        }
        if (lane == 0) M.outcome[w] = i >= 0 ? outc : 2;
        __syncthreads();  // commits done, outcomes known
        if (w == 0) {
            // the round took list[head .. head + nt), one lane each; the plans
            // that lost go back just before the moves no wavefront took (list
            // order kept), the first error in list order fails the block
            const int nt = min(NW, np - head);
            const bool on = lane < nt;
            const int mi = on ? M.list[head + lane] : 0;
            const int o = on ? M.outcome[lane] : 0;
            const uint64_t lost = ballot(on && o == 2), bad = ballot(on && o < 0);
            const int nh = head + nt - __popcll(lost);
            if (on && o == 3) M.mstate[mi] = MWS_REST;
            else if (on && (o == 0 || o == 1)) M.mstate[mi] = MWS_DONE;
            if (bad && lane == first_lane(bad) && M.fail == ST_OK) M.fail = o;
            if (on && o == 2) M.list[nh + lanes_below(lost)] = mi;
            if (lane == 0) M.head = nh;
        }
        __syncthreads();
    }
    const long long c1 = wall_clock64();
    // the rest list, in list order (a block deferred whole keeps its moves
    // where they are: REST_ALL)
    if (tid == 0) {
        int n = 0;
        if (M.fail == ST_OK && !M.defer_all)
            for (int i = 0; i < k; ++i)
                if (M.mstate[i] == MWS_REST) {
                    rb.idx[(long long)b * DRYMAX + n] = m0 + i;
                    ++n;
                }
        M.nrest = n;
        rb.cnt[b] = M.fail == ST_OK && M.defer_all ? REST_ALL : n;
    }
    __syncthreads();
    for (int j = tid; j < M.nrest; j += NT) {
        const int m = rb.idx[(long long)b * DRYMAX + j];
        rb.mv[(long long)b * DRYMAX + j] = mv[m];
    }
    if (M.fail != ST_OK && tid == 0) {
        s.status[b] = M.fail;
        atomicMin(s.sticky, M.fail);
    }
    // counters: each wavefront adds its own
    wsync();
    if (lane < NF) {
        const long long v = reinterpret_cast<const long long*>(&S.st)[lane];
        if (v) atomicAdd(reinterpret_cast<unsigned long long*>(&s.stats[b]) + lane, (unsigned long long)v);
    }
    if (M.fail != ST_OK && tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&s.stats[b].errors), 1ull);
    // the log: features, branch (repair) and the rounds' ticks; a block whose
    // moves all went to the rest list is logged by k_step_rest
    if ((need_f || pre) && s.log && s.log_cap > 0 && !M.defer_all && k > 0 && tid < LOG_FIELDS &&
        !(pre && tid < MLP_IN)) {
        float* rec = s.log + ((step % s.log_cap) * (long long)s.n_blocks + b) * LOG_FIELDS;
        float v = 0.f;
        if (tid < MLP_IN) v = M.f[tid];
        else if (tid == 17) v = (float)(c1 - c0);
        else if (tid == 18) v = (float)k;
        rec[tid] = v;
    }
}

// The rest lists of a step (one wavefront per block): the moves the rounds
// left, in list order, by the sequential path (repair or rebuild branch); a
// block deferred whole runs its step's moves from the move array itself.
__global__ void __launch_bounds__(WAVE) k_step_rest(DevState s, const kdt_move_t* __restrict__ mv,
                                                    const int* __restrict__ off, RestBuf rb, int8_t* applied,
                                                    long long step) {
    __shared__ WaveLDS S;
    extern __shared__ __align__(16) char dynx[];
    const int b = blockIdx.x;
    const int cnt = rb.cnt[b];
    if (cnt == 0) return;
    if (cnt == REST_ALL) {
        const BlockHead h = load_head(s, b, off);
        if (!head_skip(h)) {
            scratch_init(S);
            run_block_moves(s, S, b, mv, h, applied, step, true, dynx);
        }
    } else {
        BlockHead h;
        h.status = s.status[b];
        h.m0 = b * DRYMAX;
        h.m1 = h.m0 + cnt;
        h.p0 = s.pt_off[b];
        h.p1 = s.pt_off[b + 1];
        h.toff = s.tri_off[b];
        h.fr = s.frame[b];
        if (!head_skip(h)) {
            scratch_init(S);
            run_block_moves(s, S, b, rb.mv, h, rb.app, step, true, dynx);
            gsync();
            if (applied)
                for (int j = lane_id(); j < cnt; j += WAVE)
                    applied[rb.idx[(long long)b * DRYMAX + j]] = rb.app[(long long)b * DRYMAX + j];
        }
    }
    if (lane_id() == 0) rb.cnt[b] = 0;
}

// ---- grid-wide builder: the rounds of the block builder with every chunk
// of a level planned by one thread per point, claims stamped per round

__global__ void k_gb_kidx(DevState s, GlobalDev g, GBuild gb) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x + 2;
    const int n = (int)s.pt_off[1];
    const int2 a = s.xy[gb.ord[0]], b = s.xy[gb.ord[1]];
    const bool off = i < n && orient(a, b, s.xy[gb.ord[i]]) != 0;
    // one atomic per wavefront: its first lane off the line has its smallest index
    const uint64_t m = ballot(off);
    if (m && (int)(threadIdx.x & (WAVE - 1)) == first_lane(m) && (int)i < g.ctr[GC_KIDX])
        atomicMin(&g.ctr[GC_KIDX], (int)i);
}

__global__ void k_gb_seed(DevState s, GlobalDev g, GBuild gb) {
    const int kidx = g.ctr[GC_KIDX];
    if (kidx >= (int)s.pt_off[1]) {
        fail_global(s, ST_DEGEN);
        return;
    }
    BlockView B = view_of(s, 0);
    seed_triangle(B, gb.ord[0], gb.ord[1], gb.ord[kidx]);
    g.ctr[GC_USED] = 4;
    g.ctr[GC_DEFER] = 0;
}

__global__ void k_gb_chunk(GlobalDev g, GBuild gb, int lvl, long long j0, int cnt) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const long long i = lvl + 2LL * lvl * (j0 + t);
    gb.pend[t] = (i != 1 && i != g.ctr[GC_KIDX]) ? 1 : 0;
    gb.plan[t] = make_int2(0, 0);
}

__global__ void k_gb_plan(DevState s, GlobalDev g, GBuild gb, int lvl, long long j0, int cnt, int round) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt || !gb.pend[t] || s.status[0] != 0) return;
    BlockView B = view_of(s, 0);
    const int i = (int)(lvl + 2LL * lvl * (j0 + t));
    const int v = gb.ord[i];
    const int used = g.ctr[GC_USED];
    const int hs = B.vtri[gb.ord[i - lvl]];
    const int hint = hs >= 0 && hs < used ? hs : 0;
    const AttView A{gb.att + t, GB_CHUNK, TCM};
    int nc = 0, nb = 0;
    const int rc = tplan(B, v, B.xy[v], hint, A, &nc, &nb);
    if (rc == 0) {
        const unsigned long long stamp = stamp_of(g.ctr[GC_STAMP] + round, pb_prio(i));
        for (int m = 0; m < nc; ++m) claim_max(&g.claim[A.cav(m)], stamp);
        for (int e = 0; e < nb; ++e) claim_max(&g.claim[A.bout(e) >> 2], stamp);
        gb.plan[t] = make_int2(nc, nb);
    } else {
        gb.pend[t] = 0;
        if (rc == 1) {  // cavity too large for one thread's attempt: at the end, alone
            const int d = atomicAdd(&g.ctr[GC_DEFER], 1);
            if (d < GB_DEFER) gb.deferred[d] = i;
            else fail_global(s, ST_CAPACITY);
        } else {
            fail_global(s, rc);
        }
    }
}

__global__ void k_gb_commit(DevState s, GlobalDev g, GBuild gb, int lvl, long long j0, int cnt, int round) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    BlockView B = view_of(s, 0);
    int i = 0;
    int2 pl = make_int2(0, 0);
    bool won = false, pend = false;
    const AttView A{gb.att + t, GB_CHUNK, TCM};
    if (t < cnt && gb.pend[t] && s.status[0] == 0) {
        pend = true;
        pl = gb.plan[t];
        i = (int)(lvl + 2LL * lvl * (j0 + t));
        if (pl.x > 0) {
            const unsigned long long stamp = stamp_of(g.ctr[GC_STAMP] + round, pb_prio(i));
            won = true;
            for (int m = 0; m < pl.x; ++m) won &= claim_get(&g.claim[A.cav(m)]) == stamp;
            for (int e = 0; e < pl.y; ++e) won &= claim_get(&g.claim[A.bout(e) >> 2]) == stamp;
            gb.plan[t] = make_int2(0, 0);
        }
    }
    // two fresh slots per winner, one atomic per wavefront (this kernel's
    // workgroups hold several wavefronts: lanes are counted within the wave)
    const int wl = (int)(threadIdx.x & (WAVE - 1));
    const uint64_t wm = ballot(won);
    int base = 0;
    if (wm) {
        const int leader = first_lane(wm);
        if (wl == leader) base = atomicAdd(&g.ctr[GC_USED], 2 * __popcll(wm));
        base = __shfl(base, leader);
    }
    if (won) {
        const int f = base + 2 * __popcll(wm & ((1ull << wl) - 1ull));
        const int v = gb.ord[i];
        const int rc = f + 1 < B.ntri ? tcommit(B, A, pl.x, pl.y, v, B.xy[v], f, f + 1) : ST_INTERNAL;
        if (rc != ST_OK) fail_global(s, rc);
        gb.pend[t] = 0;
        pend = false;
    }
    const uint64_t pm = ballot(pend);
    if (pm && wl == first_lane(pm)) atomicAdd(&g.ctr[GC_PEND], __popcll(pm));
}

__global__ void k_gb_defer_rest(DevState s, GlobalDev g, GBuild gb, int lvl, long long j0, int cnt) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt || !gb.pend[t]) return;
    gb.pend[t] = 0;
    const int d = atomicAdd(&g.ctr[GC_DEFER], 1);
    if (d < GB_DEFER) gb.deferred[d] = (int)(lvl + 2LL * lvl * (j0 + t));
    else fail_global(s, ST_CAPACITY);
}

// Deferred points one by one (one thread), then the slot count check.
__global__ void k_gb_serial(DevState s, GlobalDev g, GBuild gb) {
    BlockView B = view_of(s, 0);
    const int nd = min(g.ctr[GC_DEFER], GB_DEFER);
    const AttView A{gb.big, 1, GB_BIG};
    for (int d = 0; d < nd && s.status[0] == 0; ++d) {
        const int i = gb.deferred[d];
        const int v = gb.ord[i];
        const int used = g.ctr[GC_USED];
        const int hs = B.vtri[gb.ord[i - 1]];
        int nc = 0, nb = 0;
        const int rc = tplan(B, v, B.xy[v], hs >= 0 && hs < used ? hs : 0, A, &nc, &nb);
        if (rc != 0) {
            fail_global(s, rc == 1 ? ST_CAPACITY : rc);
            return;
        }
        g.ctr[GC_USED] = used + 2;
        const int rc2 = used + 1 < B.ntri ? tcommit(B, A, nc, nb, v, B.xy[v], used, used + 1) : ST_INTERNAL;
        if (rc2 != ST_OK) {
            fail_global(s, rc2);
            return;
        }
    }
    if (s.status[0] == 0 && g.ctr[GC_USED] != B.ntri) fail_global(s, ST_INTERNAL);
}

// ------------------------------------------------------------------ MLP

__global__ void k_mlp_forward(const float* __restrict__ W, const float* __restrict__ X, long long n,
                              float* __restrict__ out) {
    __shared__ float w[MLP_NPARAM];
    for (int i = threadIdx.x; i < MLP_NPARAM; i += blockDim.x) w[i] = W[i];
    __syncthreads();
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float x[MLP_IN], h1[MLP_H], h2[MLP_H], o[MLP_OUT];
    for (int i = 0; i < MLP_IN; ++i) x[i] = X[s * MLP_IN + i];
    mlp_forward1(w, x, h1, h2, o);
    for (int i = 0; i < MLP_OUT; ++i) out[s * MLP_OUT + i] = o[i];
}

// Gradient of the summed loss 0.5 * |out - y|^2 over samples [0, n), and
// the loss: workgroup g takes chunks g, g + G, g + 2G, ... (G = gridDim.x)
// and writes its sums, added in chunk order, to out[g * stride ..
// g * stride + MLP_GRAD_N).  With one workgroup out holds the whole
// gradient; with one workgroup per chunk, k_mlp_reduce adds the rows in
// chunk order, which gives the same floats (kdt_mlp.hpp).
__global__ void __launch_bounds__(MLP_THREADS) k_mlp_grad(const float* __restrict__ W, const float* __restrict__ X,
                                                          const float* __restrict__ Y, long long n, float* out,
                                                          long long stride) {
#pragma clang fp contract(off)
    __shared__ MlpChunkLDS L;
    for (int i = threadIdx.x; i < MLP_NPARAM; i += MLP_THREADS) L.w[i] = W[i];
    float acc[MLP_OWN];
    for (int k = 0; k < MLP_OWN; ++k) acc[k] = 0.f;
    const long long nch = (n + MLP_CHUNK - 1) / MLP_CHUNK;
    for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
        __syncthreads();  // the previous chunk's sums are done with L
        mlp_chunk_pass(L, X, Y, n, c * MLP_CHUNK);
        for (int k = 0; k < MLP_OWN; ++k) {
            const int p = threadIdx.x + k * MLP_THREADS;
            if (p < MLP_GRAD_N) acc[k] += mlp_chunk_term(L, p);
        }
    }
    float* o = out + blockIdx.x * stride;
    for (int k = 0; k < MLP_OWN; ++k) {
        const int p = threadIdx.x + k * MLP_THREADS;
        if (p < MLP_GRAD_N) o[p] = acc[k];
    }
}

// total[p] = sum over rows r = 0 .. rows-1, in order, of part[r * stride + p]
__global__ void k_mlp_reduce(const float* __restrict__ part, int rows, long long stride, float* total) {
#pragma clang fp contract(off)
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_GRAD_N) return;
    float a = 0.f;
    for (int r = 0; r < rows; ++r) a += part[r * stride + p];
    total[p] = a;
}

// W -= lr * g / n (mean gradient step)
__global__ void k_mlp_sgd(float* W, const float* g, float lr, float inv_n) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_NPARAM) W[i] -= lr * g[i] * inv_n;
}

// query: number the real triangles of every block (list == null) or of the
// listed blocks (workgroup i takes block list[i]); counts go to qcount[i]
__global__ void __launch_bounds__(WAVE) k_qcount(DevState s, const int* list, int* qmap, int* qcount) {
    const int b = list ? list[blockIdx.x] : (int)blockIdx.x;
    const int lane = lane_id();
    BlockView B = view_of(s, b);
    int* map = qmap + s.tri_off[b];
    int base = 0;
    for (int i0 = 0; i0 < B.ntri; i0 += WAVE) {
        const int i = i0 + lane;
        const bool real = i < B.ntri && B.tri[i].v.z != GHOST;
        const uint64_t m = ballot(real);
        if (i < B.ntri) map[i] = real ? base + lanes_below(m) : -1;
        base += __popcll(m);
    }
    if (lane == 0) qcount[blockIdx.x] = base;
}

// ... and write them: block list[i] (or i) from row qoff[i] on, global ids,
// each triangle rotated to start at its smallest id; adj[t][j] is the row of
// the triangle across the edge opposite vertex j, -1 on the block's hull
__global__ void __launch_bounds__(WAVE) k_qwrite(DevState s, const int* list, const int* qmap,
                                                 const long long* qoff, int* tris, int* adj) {
    const int b = list ? list[blockIdx.x] : (int)blockIdx.x;
    BlockView B = view_of(s, b);
    const int* map = qmap + s.tri_off[b];
    const long long o = qoff[blockIdx.x];
    const int g0 = (int)s.pt_off[b];
    for (int i = lane_id(); i < B.ntri; i += WAVE) {
        const int idx = map[i];
        if (idx < 0) continue;
        const Tri t = B.tri[i];
        int r = 0;
        if (t.v.y < vget(t.v, r)) r = 1;
        if (t.v.z < vget(t.v, r)) r = 2;
        for (int j = 0; j < 3; ++j) {
            const int e = (r + j) % 3;
            tris[3 * (o + idx) + j] = g0 + vget(t.v, e);
            if (adj) {
                const int nb = vget(t.n, e) >> 2;
                const int m = bad_slot(B, nb) ? -1 : map[nb];
                adj[3 * (o + idx) + j] = m < 0 ? -1 : (int)(o + m);
            }
        }
    }
}

// ------------------------------------------------------------------ d-calculation
// Sec. III ("Notation and definitions"), Sec. IV: for a constant N, the
// distance of every point to its N-th nearest neighbour, its minimum over
// the block (mindistance), the minimum over all blocks; and the block's
// diameter for its N-spread.  One wavefront per block, one point per lane.
//
// The N nearest neighbours come from the triangulation: the (i+1)-th
// nearest neighbour of p is a DT neighbour of p or of one of its i nearest
// (the nearest-neighbour search along Delaunay edges of Dickerson, Drysdale
// and Sack), so a best-first search -- take the closest candidate not yet
// taken, add its DT neighbours -- takes them in order; every comparison is
// of exact integer squared distances.
constexpr int DC_CAP = 64;   // candidates one point's search holds
constexpr int DC_NMAX = 8;   // largest N
constexpr long long DC_NONE = 0x7fffffffffffffffll;

__device__ __forceinline__ long long d2_of(int2 a, int2 b) {
    const long long dx = (long long)a.x - b.x, dy = (long long)a.y - b.y;
    return dx * dx + dy * dy;
}

struct DcLDS {
    int id[DC_CAP][WAVE];        // candidate points (lane-contiguous)
    long long d2[DC_CAP][WAVE];  // their squared distances (-1: taken)
    int hull[1024];              // hull vertices of the block (diameter)
    int nhull;
};

__global__ void __launch_bounds__(WAVE) k_dcalc(DevState s, int N, long long* mind2, long long* diam2,
                                                unsigned long long* gmin, int* err) {
    __shared__ DcLDS L;
    const int b = blockIdx.x, lane = lane_id();
    const BlockView B = view_of(s, b);
    long long best = DC_NONE;
    bool over = false;
    for (int p = lane; p < B.n && N < B.n; p += WAVE) {
        const int2 pp = B.xy[p];
        int nc = 0;
        long long last = DC_NONE;
        int v = p;
        for (int it = 0; it < N; ++it) {
            // the DT neighbours of v (a closed fan: ghosts close it at the hull)
            const int t0 = B.vtri[v];
            int cur = t0;
            for (int g = 0; g < 4 * KMAX && !over; ++g) {
                if (bad_slot(B, cur)) { over = true; break; }
                const Tri t = load_tri(B.tri + cur);
                const int i = t.v.x == v ? 0 : (t.v.y == v ? 1 : 2);
                const int u = vget(t.v, (i + 1) % 3);
                if (u != GHOST && u != p) {
                    bool seen = false;
                    for (int c = 0; c < nc && !seen; ++c) seen = L.id[c][lane] == u;
                    if (!seen) {
                        if (nc == DC_CAP) {
                            over = true;
                        } else {
                            L.id[nc][lane] = u;
                            L.d2[nc][lane] = d2_of(pp, cget(t, (i + 1) % 3));
                            ++nc;
                        }
                    }
                }
                cur = vget(t.n, (i + 2) % 3) >> 2;
                if (cur == t0) break;
            }
            if (over) break;
            // the closest candidate not taken yet (ties: smaller id) is the
            // (it+1)-th nearest neighbour: a neighbour of p or of one of the
            // it nearest, whose neighbours are all candidates by now
            int j = -1;
            for (int c = 0; c < nc; ++c) {
                const long long dc = L.d2[c][lane];
                if (dc < 0) continue;
                if (j < 0 || dc < L.d2[j][lane] || (dc == L.d2[j][lane] && L.id[c][lane] < L.id[j][lane])) j = c;
            }
            if (j < 0) { over = true; break; }
            last = L.d2[j][lane];
            L.d2[j][lane] = -1;
            v = L.id[j][lane];
        }
        if (!over) best = min(best, last);
    }
    for (int off = 32; off > 0; off >>= 1) best = min(best, (long long)__shfl_xor(best, off));
    // diameter: the farthest pair lies on the convex hull; hull vertices are
    // the finite corners of the ghosts
    if (lane == 0) L.nhull = 0;
    wsync();
    for (int i = lane; i < B.ntri; i += WAVE) {
        const Tri t = load_tri(B.tri + i);
        if (t.v.z == GHOST) {
            const int h = atomicAdd(&L.nhull, 1);
            if (h < 1024) L.hull[h] = t.v.x;
        }
    }
    wsync();
    const int nh = L.nhull;
    long long dmax = 0;
    if (nh <= 1024) {
        for (int a = lane; a < nh; a += WAVE) {
            const int2 pa = B.xy[L.hull[a]];
            for (int c = 0; c < nh; ++c) dmax = max(dmax, d2_of(pa, B.xy[L.hull[c]]));
        }
    } else {  // more hull vertices than the list holds: every pair of points
        for (int a = lane; a < B.n; a += WAVE) {
            const int2 pa = B.xy[a];
            for (int c = 0; c < B.n; ++c) dmax = max(dmax, d2_of(pa, B.xy[c]));
        }
    }
    for (int off = 32; off > 0; off >>= 1) dmax = max(dmax, (long long)__shfl_xor(dmax, off));
    const bool bad = ballot(over) != 0;
    if (lane == 0) {
        mind2[b] = bad ? DC_NONE : best;
        diam2[b] = dmax;
        if (bad) atomicAdd(err, 1);
        else if (best != DC_NONE) atomicMin(gmin, (unsigned long long)best);
    }
}

// Order-independent digest of a block's triangulation: the wrapping sum,
// over its real triangles rotated to start at their smallest global id
// (a, b, c), of mix(a ^ mix(b ^ mix(c))), mix = splitmix64's finaliser.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(WAVE) k_digest(DevState s, unsigned long long* out) {
    const int b = blockIdx.x;
    BlockView B = view_of(s, b);
    const unsigned long long g0 = (unsigned long long)s.pt_off[b];
    unsigned long long acc = 0;
    for (int i = lane_id(); i < B.ntri; i += WAVE) {
        const Tri t = B.tri[i];
        if (t.v.z == GHOST) continue;
        int r = 0;
        if (t.v.y < vget(t.v, r)) r = 1;
        if (t.v.z < vget(t.v, r)) r = 2;
        const unsigned long long a = g0 + vget(t.v, r), bb = g0 + vget(t.v, (r + 1) % 3),
                                 c = g0 + vget(t.v, (r + 2) % 3);
        acc += mix64(a ^ mix64(bb ^ mix64(c)));
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if (lane_id() == 0) out[b] = acc;
}

// ------------------------------------------------------------------ host

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t tri, xy, vtri, order, pt_off, tri_off, frame, status, stats, qmap, own2, rb_flag, qcount, qoff,
        qtris, qadj, qlist, stage_mv, stage_off, stage_app, sticky, lpt, sorder, rest_mv, rest_idx, rest_app,
        rest_cnt, dc_mind2, dc_diam2, dc_g, choice, total;
};

Layout make_layout(int64_t n, int32_t B, int32_t max_staged) {
    Layout L;
    const int64_t ntri = 2 * n - 2 * (int64_t)B;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    L.tri = take(sizeof(Tri) * ntri);
    L.xy = take(sizeof(int2) * n);
    L.vtri = take(sizeof(int) * n);
    L.order = take(sizeof(int) * n);
    L.pt_off = take(sizeof(long long) * (B + 1));
    L.tri_off = take(sizeof(long long) * (B + 1));
    L.frame = take(sizeof(int4) * B);
    L.status = take(sizeof(int) * B);
    L.stats = take(sizeof(BlockStats) * B);
    L.qmap = take(sizeof(int) * ntri);
    L.own2 = take(sizeof(int) * ntri);
    L.rb_flag = take(sizeof(int) * (B + 2));
    L.choice = take((size_t)B * CHOOSE_STEPS);
    L.qcount = take(sizeof(int) * B);
    L.qoff = take(sizeof(long long) * (B + 1));
    L.qtris = take(sizeof(int) * 3 * ntri);
    L.qadj = take(sizeof(int) * 3 * ntri);
    L.qlist = take(sizeof(int) * B);
    L.stage_mv = take(sizeof(kdt_move_t) * (size_t)std::max(max_staged, 1));
    L.stage_off = take(sizeof(int) * (B + 1));
    L.stage_app = take((size_t)std::max(max_staged, 1));
    L.sticky = take(sizeof(int) * 4);
    L.lpt = take(sizeof(int) * (B + 1));
    L.sorder = take(sizeof(int) * (size_t)(B + 2) * ORDER_STEPS);
    L.rest_mv = take(sizeof(kdt_move_t) * (size_t)B * DRYMAX);
    L.rest_idx = take(sizeof(int) * (size_t)B * DRYMAX);
    L.rest_app = take((size_t)B * DRYMAX);
    L.rest_cnt = take(sizeof(int) * B);
    L.dc_mind2 = take(sizeof(long long) * B);
    L.dc_diam2 = take(sizeof(long long) * B);
    L.dc_g = take(sizeof(unsigned long long) * 2);
    L.total = o;
    return L;
}

// Global mode: the extra regions after the per-block layout of one block.
struct GLayout {
    size_t claim, mstate, rs, rsn, pslot, prec, pvt, phdr, pq, hkey, hcnt, ctr, serial, split, powner, gstats,
        part, att, pend, plan, deferred, big, qn, ql, qcnt, qlev, total;
    int hsize;
};

GLayout make_glayout(size_t base, int64_t n, int32_t depth, int32_t max_moves, int64_t n_qt = 0) {
    GLayout G;
    size_t o = align_up(base);
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    const int64_t ntri = 2 * n - 2;
    int hs = 1024;
    while (hs < 8 * (int64_t)max_moves) hs *= 2;
    G.hsize = hs;
    G.claim = take(sizeof(unsigned long long) * ntri);
    G.mstate = take(sizeof(int) * max_moves);
    G.rs = take(sizeof(int) * (size_t)RSMAX * max_moves);
    G.rsn = take(sizeof(int) * max_moves);
    G.pslot = take(sizeof(int) * (size_t)PRECMAX * max_moves);
    G.prec = take(sizeof(Tri) * (size_t)PRECMAX * max_moves);
    G.pvt = take(sizeof(int2) * (size_t)PVTMAX * max_moves);
    G.phdr = take(sizeof(int4) * max_moves);
    G.pq = take(sizeof(int2) * max_moves);
    G.hkey = take(sizeof(unsigned long long) * hs);
    G.hcnt = take(sizeof(int) * hs);
    G.ctr = take(sizeof(int) * GC_N);
    G.serial = take(sizeof(int) * max_moves);
    G.split = take(sizeof(int2) * ((size_t)1 << depth));
    G.powner = take(sizeof(int) * n);
    G.gstats = take(sizeof(unsigned long long) * KDT_GSTAT_N);
    G.part = take(sizeof(unsigned long long) * 4 * G_PART_MAX);
    G.att = take(sizeof(int) * (size_t)ATT_INTS * GB_CHUNK);
    G.pend = take(sizeof(int) * GB_CHUNK);
    G.plan = take(sizeof(int2) * GB_CHUNK);
    G.deferred = take(sizeof(int) * GB_DEFER);
    G.big = take(sizeof(int) * (4 * (size_t)GB_BIG + 6));
    G.qn = take(sizeof(int4) * (size_t)std::max<int64_t>(n_qt, 1));
    G.ql = take(sizeof(int4) * (size_t)std::max<int64_t>(n_qt, 1));
    G.qcnt = take(sizeof(int) * (size_t)std::max<int64_t>(n_qt, 1));
    G.qlev = take(sizeof(int) * (QT_LEVELS + 1));
    G.total = o;
    return G;
}

// kd partition of the initial points: node `node` at `level` keeps the
// first half (by (x, y) at even levels, (y, x) at odd ones) on the left and
// records the key of the first right point; leaves give each point its cell.
void kd_build(const int32_t* xy, std::vector<int>& idx, size_t lo, size_t hi, int node, int level,
              int depth, std::vector<int2>& split, std::vector<int>& cell) {
    if (level == depth) {
        for (size_t i = lo; i < hi; ++i) cell[idx[i]] = node - (1 << depth);
        return;
    }
    const int d = level & 1;
    auto key = [&](int a) { return std::make_pair(xy[2 * (size_t)a + d], xy[2 * (size_t)a + 1 - d]); };
    const size_t h = lo + (hi - lo) / 2;
    std::nth_element(idx.begin() + lo, idx.begin() + h, idx.begin() + hi,
                     [&](int a, int b) { return key(a) < key(b); });
    const auto k = key(idx[h]);
    split[node] = make_int2(k.first, k.second);
    kd_build(xy, idx, lo, h, 2 * node, level + 1, depth, split, cell);
    kd_build(xy, idx, h, hi, 2 * node + 1, level + 1, depth, split, cell);
}

// Quad-tree of the initial points (Sec. III "Data structure"): the root is
// the smallest power-of-two square at the domain's lower-left corner that
// covers the domain; a node holding more than `thr` points (and wider than
// one lattice cell) is cut into its four quarters, kept in the order (low x,
// low y), (high x, low y), (low x, high y), (high x, high y) -- empty
// quarters too, so that the leaves tile the square.  nodes: {x0, y0, log2
// side, first child or -1}; cell: the leaf of every point.
struct QtHost {
    std::vector<int4> nodes, links;
    std::vector<int> cell;
};
void qt_node(const int32_t* xy, std::vector<int>& idx, size_t lo, size_t hi, int node, int64_t thr, QtHost& T) {
    const int4 nd = T.nodes[node];
    if ((int64_t)(hi - lo) <= thr || nd.z == 0) {
        for (size_t i = lo; i < hi; ++i) T.cell[idx[i]] = node;
        return;
    }
    const int h = 1 << (nd.z - 1);
    const int c0 = (int)T.nodes.size();
    T.nodes[node].w = c0;
    for (int q = 0; q < 4; ++q) T.nodes.push_back(make_int4(nd.x + (q & 1) * h, nd.y + (q >> 1) * h, nd.z - 1, -1));
    auto quad = [&](int a) {
        return (xy[2 * (size_t)a] >= nd.x + h ? 1 : 0) + (xy[2 * (size_t)a + 1] >= nd.y + h ? 2 : 0);
    };
    size_t cut[5];
    cut[0] = lo;
    for (int q = 0; q < 4; ++q) {
        const auto mid = std::stable_partition(idx.begin() + cut[q], idx.begin() + hi, [&](int a) { return quad(a) == q; });
        cut[q + 1] = (size_t)(mid - idx.begin());
    }
    for (int q = 0; q < 4; ++q) qt_node(xy, idx, cut[q], cut[q + 1], c0 + q, thr, T);
}
// The node across each side of every leaf: the node holding the first
// lattice cell past that side, at the leaf's size or larger.
int qt_probe(const QtHost& T, int64_t px, int64_t py, int lg) {
    const int4 r = T.nodes[0];
    const int64_t side = (int64_t)1 << r.z;
    if (px < r.x || py < r.y || px >= r.x + side || py >= r.y + side) return -1;
    int node = 0;
    while (T.nodes[node].w >= 0 && T.nodes[node].z > lg) {
        const int4 nd = T.nodes[node];
        const int64_t h = (int64_t)1 << (nd.z - 1);
        node = nd.w + (px >= nd.x + h ? 1 : 0) + (py >= nd.y + h ? 2 : 0);
    }
    return node;
}
void qt_build_host(const int32_t* xy, int64_t n, const int32_t* domain, int64_t thr, QtHost& T) {
    int lg = 0;
    const int32_t ext = std::max(domain[2] - domain[0], domain[3] - domain[1]);
    while ((1 << lg) < ext) ++lg;
    T.nodes.assign(1, make_int4(domain[0], domain[1], lg, -1));
    T.cell.assign(n, 0);
    std::vector<int> idx(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = (int)i;
    qt_node(xy, idx, 0, (size_t)n, 0, thr, T);
    T.links.assign(T.nodes.size(), make_int4(-1, -1, -1, -1));
    for (size_t k = 0; k < T.nodes.size(); ++k) {
        const int4 nd = T.nodes[k];
        if (nd.w >= 0) continue;
        const int64_t side = (int64_t)1 << nd.z;
        T.links[k] = make_int4(qt_probe(T, nd.x + side, nd.y, nd.z), qt_probe(T, (int64_t)nd.x - 1, nd.y, nd.z),
                               qt_probe(T, nd.x, nd.y + side, nd.z), qt_probe(T, nd.x, (int64_t)nd.y - 1, nd.z));
    }
}

// Nodes the quad-tree arrays hold: the initial tree, and any tree of n
// points with this threshold (a level cuts at most n / (thr + 1) nodes,
// each into 4, over at most log2 side levels).
int64_t qt_capacity(const QtHost& T, int64_t n, int64_t thr) {
    const int64_t lg = T.nodes.empty() ? 0 : T.nodes[0].z;
    return std::max<int64_t>((int64_t)T.nodes.size(), 1 + 4 * lg * ((n + thr) / (thr + 1)));
}

// Hilbert index of (x, y) on a 2^16 x 2^16 grid (classic rotate-and-flip
// construction); used only to order insertions for short walks.
uint64_t hilbert16(uint32_t x, uint32_t y) {
    uint64_t d = 0;
    for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
        uint32_t rx = (x & s) ? 1 : 0, ry = (y & s) ? 1 : 0;
        d += (uint64_t)s * s * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) { x = s - 1 - x; y = s - 1 - y; }
            std::swap(x, y);
        }
    }
    return d;
}

}  // namespace

struct kdt_ctx {
    hipStream_t stream;
    int32_t B;
    int64_t n;
    int32_t max_staged;
    DevState dev;
    char* ws;
    Layout L;
    std::vector<long long> pt_off, tri_off;
    std::vector<kdt_move_t> staged;
    std::vector<int32_t> staged_block;
    int sticky;
    int device = 0;
    int cus = 256;
    int wpc = 4;  // workgroups (one wavefront each) that fit a compute unit's LDS: step ones, or the global rounds' planning ones
    long long step_count = 0;  // time steps launched so far (log index)
    long long epoch = 0;       // changes of policy, log or launch shape (graphs record theirs)
    int persist_per_cu = 4;  // workgroups per compute unit of the persistent launch
    int block_waves = 1;     // wavefronts per block of the per-step launch (1, 2 or 4)
    int block_order = 0;     // 1: the per-step launch takes blocks most moves first
    int heavy_cut = 0;       // > 0 (with block_waves > 1): only blocks of this many moves get several wavefronts
    int mid_cut = 0;         // > 0 (with block_waves 4): blocks of mid_cut .. heavy_cut - 1 moves get two
    hipStream_t side = nullptr, side2 = nullptr;         // streams of the heavy and middle classes
    hipEvent_t fork_ev = nullptr, join_ev = nullptr, join2_ev = nullptr;  // fork, joins
    RestBuf rest{};          // rest lists of the multi-wavefront launch
    // d-calculation over time (kdt_dcalc): running minimum of the squared
    // mindistance, every block's running maximum N-spread, for one N
    int dc_n = 0;
    long long dc_d2 = 0x7fffffffffffffffll;
    std::vector<double> dc_spread;
    bool timing = false;
    int timing_period = 1;        // launches one event pair spans
    long long timing_count = 0;   // launches covered by closed pairs since timing was enabled
    int timing_open = 0;          // launches in the open pair (0: none open)
    int pb_lds = 0;         // dynamic LDS of k_build_blocks at init
    int pb_lds_follow = 0;  // ... after a step, for the blocks too large for the step kernels
    bool follow = false;    // some block is too large to be rebuilt inside the step kernels
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;  // recorded pairs
    size_t ev_used = 0;
    // global mode: one triangulation over all points (block 0)
    bool global = false;
    int32_t depth = 0;
    int32_t max_moves = 0;
    int hsize = 0;
    GlobalDev g{};
    GBuild gb{};
    int qt_count = 0;        // quad-tree cells: nodes in use
    bool qt_every_step = false;  // re-partition after every step
    long long build_rounds = 0;
};

namespace {

int check_hip(kdt_ctx* c, hipError_t e) {
    if (e == hipSuccess) return KDT_OK;
    if (c) c->sticky = KDT_E_DEVICE;
    return KDT_E_DEVICE;
}

// When timing is on, one event pair spans each run of timing_period
// consecutive launches: the first launch of a run records the start, the
// last one the end.
hipEvent_t timing_begin(kdt_ctx* c) {
    if (!c->timing) return nullptr;
    if (c->timing_open == 0) {
        if (c->ev_used == c->ev.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return nullptr;
            if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return nullptr; }
            c->ev.push_back({a, b});
        }
        (void)hipEventRecord(c->ev[c->ev_used].first, c->stream);
    }
    return c->ev[c->ev_used].first;
}
void timing_close(kdt_ctx* c) {
    (void)hipEventRecord(c->ev[c->ev_used].second, c->stream);
    c->ev_used++;
    c->timing_count += c->timing_open;
    c->timing_open = 0;
}
void timing_end(kdt_ctx* c, hipEvent_t a) {
    if (!a) return;
    if (++c->timing_open >= c->timing_period) timing_close(c);
}
void release_events(kdt_ctx* c) {
    for (auto& p : c->ev) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    c->ev.clear();
    c->ev_used = 0;
}

// Workgroups per compute unit that the LDS holds, each taking `bytes`.
int wg_per_cu(int dev, size_t bytes) {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || lds < 1)
        lds = 160 * 1024;
    return std::max(1, lds / (int)bytes);
}
// Step workgroups per compute unit (each takes a WaveLDS).
int step_wg_per_cu(int dev) { return wg_per_cu(dev, sizeof(WaveLDS)); }

// Dynamic LDS for the block build: PB_LDS_BYTES if the device lets a
// kernel have that much, else the default limit.
int pb_lds_bytes() {
    static int bytes = -1;
    if (bytes < 0) {
        bytes = hipFuncSetAttribute((const void*)k_build_blocks, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    PB_LDS_BYTES) == hipSuccess &&
                        hipFuncSetAttribute((const void*)k_build_listed, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            PB_LDS_BYTES) == hipSuccess
                    ? PB_LDS_BYTES
                    : 64 * 1024;
        (void)hipGetLastError();
    }
    return bytes;
}

// Dynamic LDS the step kernels may have on top of their static LDS under a
// rebuilding policy (two workgroups per compute unit still fit), or 0 if the
// device refuses it.
constexpr int STEP_LDS_EXTRA_MAX = 44 * 1024;
int step_lds_limit() {
    static int bytes = -1;
    if (bytes < 0) {
        bool ok = true;
        for (const void* k : {(const void*)k_step, (const void*)k_step_persist, (const void*)k_run_fused,
                              (const void*)k_step_rest})
            ok = ok && hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, STEP_LDS_EXTRA_MAX) ==
                           hipSuccess;
        (void)hipGetLastError();
        bytes = ok ? STEP_LDS_EXTRA_MAX : 0;
    }
    return bytes;
}

// The multi-wavefront step kernels take more than the default 64 KB of
// dynamic LDS: allowed once per process.
bool mw_lds_ok() {
    static int ok = -1;
    if (ok < 0) {
        ok = hipFuncSetAttribute((const void*)k_step_mw<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sizeof(MwLDS<4>)) == hipSuccess &&
             hipFuncSetAttribute((const void*)k_step_mw<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sizeof(MwLDS<2>)) == hipSuccess;
        (void)hipGetLastError();
    }
    return ok == 1;
}

// Largest LDS need of a block build above `above` and within `limit` (0 if none).
size_t max_block_need(const kdt_ctx* c, size_t above, size_t limit) {
    size_t best = 0;
    for (int32_t b = 0; b < c->B; ++b) {
        const size_t need = pb_block_lds(c->pt_off[b + 1] - c->pt_off[b]);
        if (need > above && need <= limit) best = std::max(best, need);
    }
    return best;
}

// Launch sizes for the rebuild branch under the current policy: the step
// kernels get room to build the largest block that fits their extra LDS;
// larger blocks are built by k_build_listed after the step.
void plan_rebuild_lds(kdt_ctx* c) {
    c->dev.step_lds = 0;
    c->follow = false;
    if (c->dev.policy == KDT_POLICY_REPAIR) return;
    c->dev.step_lds = (int)((max_block_need(c, 0, (size_t)step_lds_limit()) + 255) & ~(size_t)255);
    for (int32_t b = 0; b < c->B && !c->follow; ++b)
        c->follow = pb_block_lds(c->pt_off[b + 1] - c->pt_off[b]) > (size_t)c->dev.step_lds;
    c->pb_lds_follow =
        (int)(pb_fixed_lds() + max_block_need(c, (size_t)c->dev.step_lds, pb_lds_bytes() - pb_fixed_lds()));
}

int64_t orient_h(const int32_t* a, const int32_t* b, const int32_t* c) {
    return (int64_t)(b[0] - a[0]) * (c[1] - a[1]) - (int64_t)(b[1] - a[1]) * (c[0] - a[0]);
}

// Build the global DT* from the current positions with the grid-wide
// builder: Hilbert-order levels, chunks of GB_CHUNK points, reservation
// rounds until a chunk is done (the host reads the pending count after each
// round), then the deferred points one by one.
int gbuild(kdt_ctx* c) {
    hipStream_t st = c->stream;
    const int n = (int)c->n;
    k_set<<<1, 1, 0, st>>>(c->g.ctr + GC_KIDX, 0x7fffffff);
    k_gb_kidx<<<(n - 2 + 255) / 256, 256, 0, st>>>(c->dev, c->g, c->gb);
    k_gb_seed<<<1, 1, 0, st>>>(c->dev, c->g, c->gb);
    if (check_hip(c, hipGetLastError()) != KDT_OK) return KDT_E_DEVICE;
    int top = 1;
    while (top * 2 < n) top *= 2;
    for (int lvl = top; lvl >= 1; lvl >>= 1) {
        const long long count = (n - 1 - lvl) / (2LL * lvl) + 1;
        for (long long j0 = 0; j0 < count; j0 += GB_CHUNK) {
            const int cnt = (int)std::min<long long>(GB_CHUNK, count - j0);
            const int grid = (cnt + 255) / 256;
            k_gb_chunk<<<grid, 256, 0, st>>>(c->g, c->gb, lvl, j0, cnt);
            int r = 0;
            for (; r < GB_ROUNDS; ++r) {
                k_set<<<1, 1, 0, st>>>(c->g.ctr + GC_PEND, 0);
                k_gb_plan<<<grid, 256, 0, st>>>(c->dev, c->g, c->gb, lvl, j0, cnt, r);
                k_gb_commit<<<grid, 256, 0, st>>>(c->dev, c->g, c->gb, lvl, j0, cnt, r);
                int pend = 0;
                if (check_hip(c, hipGetLastError()) ||
                    check_hip(c, hipMemcpyAsync(&pend, c->g.ctr + GC_PEND, sizeof(int), hipMemcpyDeviceToHost, st)) ||
                    check_hip(c, hipStreamSynchronize(st)))
                    return KDT_E_DEVICE;
                ++c->build_rounds;
                if (pend == 0) break;
            }
            if (r == GB_ROUNDS) k_gb_defer_rest<<<grid, 256, 0, st>>>(c->dev, c->g, c->gb, lvl, j0, cnt);
            k_add<<<1, 1, 0, st>>>(c->g.ctr + GC_STAMP, GB_ROUNDS + 1);  // past this chunk's rounds
        }
    }
    k_gb_serial<<<1, 1, 0, st>>>(c->dev, c->g, c->gb);
    if (check_hip(c, hipGetLastError()) || check_hip(c, hipStreamSynchronize(st))) return KDT_E_DEVICE;
    int sticky = 0;
    if (check_hip(c, hipMemcpy(&sticky, c->dev.sticky, sizeof(int), hipMemcpyDeviceToHost))) return KDT_E_DEVICE;
    return sticky;
}

// ---- library-side partition (Sec. III, "Data structure"): the smallest
// square with a power-of-two side covering the points, cut into four equal
// squares again and again.
struct PartBlock {
    int64_t lo, hi;  // range in Morton order
    int32_t x0, y0, side;
};

// Points of a Morton-ordered range [lo, hi) all on one line (or < 3 points).
bool range_collinear(const int32_t* xy, const std::vector<int64_t>& ord, int64_t lo, int64_t hi) {
    if (hi - lo < 3) return true;
    const int32_t* a = xy + 2 * ord[lo];
    const int32_t* b = xy + 2 * ord[lo + 1];
    for (int64_t i = lo + 2; i < hi; ++i)
        if (orient_h(a, b, xy + 2 * ord[i]) != 0) return false;
    return true;
}

// Quad-tree leaves of node (x0, y0, side) holding Morton range [lo, hi): a
// node with more than `thr` points is cut into its four quarters (in Morton
// order: low x low y, high x low y, low x high y, high x high y), quarters
// holding no point are dropped; a node whose cut would leave a quarter with
// fewer than 4 points or with all its points on one line stays whole.
void quad_leaves(const int32_t* xy, const std::vector<int64_t>& ord, const std::vector<uint64_t>& code,
                 int64_t lo, int64_t hi, int32_t x0, int32_t y0, int32_t side, int bits, int64_t thr,
                 std::vector<PartBlock>& out) {
    if (hi - lo > thr && side > 1) {
        const int h = bits - 1;  // the quarter is bits (2h+1, 2h) of the code
        int64_t cut[5];
        cut[0] = lo;
        cut[4] = hi;
        for (int q = 1; q < 4; ++q) {
            const uint64_t key = (code[lo] >> (2 * h + 2) << (2 * h + 2)) | ((uint64_t)q << (2 * h));
            cut[q] = std::lower_bound(code.begin() + lo, code.begin() + hi, key) - code.begin();
        }
        bool ok = true;
        for (int q = 0; q < 4 && ok; ++q) {
            const int64_t m = cut[q + 1] - cut[q];
            if (m == 0) continue;
            ok = m >= 4 && !range_collinear(xy, ord, cut[q], cut[q + 1]);
        }
        if (ok) {
            const int32_t hs = side / 2;
            for (int q = 0; q < 4; ++q)
                if (cut[q + 1] > cut[q])
                    quad_leaves(xy, ord, code, cut[q], cut[q + 1], x0 + (q & 1) * hs, y0 + (q >> 1) * hs, hs, h,
                                thr, out);
            return;
        }
    }
    out.push_back(PartBlock{lo, hi, x0, y0, side});
}

uint64_t morton24(uint32_t x, uint32_t y) {
    uint64_t m = 0;
    for (int i = 0; i < 24; ++i) m |= ((uint64_t)((x >> i) & 1) << (2 * i)) | ((uint64_t)((y >> i) & 1) << (2 * i + 1));
    return m;
}

}  // namespace

// ---- scratch of kdt_mlp_train_noalloc: the per-chunk gradient sums of one
// batch (one row of NOALLOC_ROW floats per chunk of MLP_CHUNK samples, up to
// NOALLOC_ROWS rows: batches of at most KDT_MLP_NOALLOC_BATCH samples), then
// the batch's gradient.  Each GPU holds its own copy until the process ends.
// Host code never passes the array's name to a kernel: it uses the address
// hipGetSymbolAddress gives on the device (noalloc_scratch).
constexpr int NOALLOC_ROWS = KDT_MLP_NOALLOC_BATCH / MLP_CHUNK;
constexpr long long NOALLOC_ROW = (MLP_GRAD_N + 63) / 64 * 64;  // 256-byte rows
static_assert(NOALLOC_ROWS * MLP_CHUNK == KDT_MLP_NOALLOC_BATCH, "batch limit is whole chunks");
static __device__ __align__(256) float scratch[(NOALLOC_ROWS + 1) * NOALLOC_ROW];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
float* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current).
int noalloc_scratch(float** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return KDT_E_DEVICE;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KDT_E_DEVICE;
        noalloc_ptr[dev] = static_cast<float*>(p);
    }
    *out = noalloc_ptr[dev];
    return KDT_OK;
}

}  // namespace

extern "C" {

const char* kdt_strerror(int code) {
    switch (code) {
    case KDT_OK: return "ok";
    case KDT_E_ARG: return "bad argument";
    case KDT_E_RANGE: return "coordinate out of range or outside its frame";
    case KDT_E_DUP: return "duplicate point in a block";
    case KDT_E_DEGEN: return "block with fewer than 4 points or all collinear";
    case KDT_E_CAPACITY: return "capacity exceeded";
    case KDT_E_DEVICE: return "HIP runtime error";
    case KDT_E_STATE: return "call out of order";
    case KDT_E_INTERNAL: return "device invariant check failed";
    default: return "unknown status";
    }
}

int kdt_partition(const int32_t* xy, int64_t n, int32_t scheme, int64_t param, int64_t* perm,
                  int64_t* block_off, int32_t* frames, int32_t cap_blocks, int32_t* n_blocks) {
    if (!xy || !perm || !n_blocks || n < 1 || cap_blocks < 0 || (cap_blocks > 0 && (!block_off || !frames)))
        return KDT_E_ARG;
    if (scheme != KDT_PART_GRID && scheme != KDT_PART_QUADTREE) return KDT_E_ARG;
    *n_blocks = 0;
    int depth = 0;
    if (scheme == KDT_PART_GRID) {
        // param = number of cells, a power of four
        int64_t p = 1;
        while (p < param && depth < 12) { p *= 4; ++depth; }  // at most 4^12 cells
        if (param < 1 || p != param) return KDT_E_ARG;
    } else if (param < 4) {
        return KDT_E_ARG;
    }
    int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = INT32_MIN, mxy = INT32_MIN;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t x = xy[2 * i], y = xy[2 * i + 1];
        if (x < 0 || y < 0 || x >= KDT_COORD_LIMIT || y >= KDT_COORD_LIMIT) return KDT_E_RANGE;
        mnx = std::min(mnx, x); mny = std::min(mny, y);
        mxx = std::max(mxx, x); mxy = std::max(mxy, y);
    }
    // covering square: lower-left corner at the minima, power-of-two side
    const int32_t ext = std::max(mxx - mnx, mxy - mny) + 1;
    int bits = 0;
    while ((1 << bits) < ext) ++bits;
    bits = std::max(bits, depth);
    std::vector<int64_t> ord(n);
    std::vector<uint64_t> code(n);
    {
        std::vector<std::pair<uint64_t, int64_t>> key(n);
        for (int64_t i = 0; i < n; ++i)
            key[i] = {morton24((uint32_t)(xy[2 * i] - mnx), (uint32_t)(xy[2 * i + 1] - mny)), i};
        std::sort(key.begin(), key.end());
        for (int64_t i = 0; i < n; ++i) {
            if (i > 0 && key[i].first == key[i - 1].first) return KDT_E_DUP;
            ord[i] = key[i].second;
            code[i] = key[i].first;
        }
    }
    std::vector<PartBlock> leaves;
    if (scheme == KDT_PART_QUADTREE) {
        quad_leaves(xy, ord, code, 0, n, mnx, mny, 1 << bits, bits, param, leaves);
    } else {
        // every cell of the depth-`depth` grid that holds a point, row by row
        const int cb = bits - depth;  // a cell's side is 2^cb
        const int64_t cells = 1LL << depth;
        std::vector<std::pair<int64_t, int64_t>> key(n);  // (row-major cell, point)
        for (int64_t i = 0; i < n; ++i)
            key[i] = {(((int64_t)(xy[2 * i + 1] - mny) >> cb) * cells) + ((xy[2 * i] - mnx) >> cb), i};
        std::sort(key.begin(), key.end());
        for (int64_t i = 0; i < n; ++i) {
            ord[i] = key[i].second;
            if (i == 0 || key[i].first != key[i - 1].first) {
                const int64_t c = key[i].first;
                leaves.push_back(PartBlock{i, i, mnx + (int32_t)((c % cells) << cb),
                                           mny + (int32_t)((c / cells) << cb), 1 << cb});
            }
            leaves.back().hi = i + 1;
        }
    }
    *n_blocks = (int32_t)leaves.size();
    if ((int64_t)leaves.size() > cap_blocks) return KDT_E_CAPACITY;
    block_off[0] = 0;
    for (size_t b = 0; b < leaves.size(); ++b) {
        const PartBlock& L = leaves[b];
        // a block's points in input order (so local order follows global id order)
        std::vector<int64_t> pts(ord.begin() + L.lo, ord.begin() + L.hi);
        std::sort(pts.begin(), pts.end());
        for (size_t k = 0; k < pts.size(); ++k) perm[L.lo + (int64_t)k] = pts[k];
        block_off[b + 1] = L.hi;
        frames[4 * b + 0] = L.x0;
        frames[4 * b + 1] = L.y0;
        frames[4 * b + 2] = (int32_t)std::min<int64_t>((int64_t)L.x0 + L.side, KDT_COORD_LIMIT);
        frames[4 * b + 3] = (int32_t)std::min<int64_t>((int64_t)L.y0 + L.side, KDT_COORD_LIMIT);
    }
    return KDT_OK;
}

int kdt_workspace_size(int64_t n, int32_t n_blocks, const int64_t* block_off, int32_t max_staged,
                       size_t* dev_bytes) {
    if (!dev_bytes || !block_off || n_blocks < 1 || n < 1 || max_staged < 0) return KDT_E_ARG;
    if (block_off[0] != 0 || block_off[n_blocks] != n) return KDT_E_ARG;
    if (2 * n >= (int64_t)1 << 31) return KDT_E_CAPACITY;
    *dev_bytes = make_layout(n, n_blocks, max_staged).total;
    return KDT_OK;
}

int kdt_init(kdt_ctx** out, const int32_t* xy, int64_t n, int32_t n_blocks,
             const int64_t* block_off, const int32_t* frames, int32_t max_staged, void* dev_ws,
             size_t ws_bytes, void* stream) {
    if (!out) return KDT_E_ARG;
    *out = nullptr;
    if (!xy || !block_off || n_blocks < 1 || n < 1 || max_staged < 0) return KDT_E_ARG;
    if (block_off[0] != 0 || block_off[n_blocks] != n) return KDT_E_ARG;
    if (2 * n >= (int64_t)1 << 31) return KDT_E_CAPACITY;
    for (int32_t b = 0; b < n_blocks; ++b) {
        const int64_t cnt = block_off[b + 1] - block_off[b];
        if (cnt < 0) return KDT_E_ARG;
        if (cnt < 4) return KDT_E_DEGEN;
        if (cnt > (1 << 22)) return KDT_E_CAPACITY;  // link indices are packed in 8 bits, slots in 30
    }
    // frames
    std::vector<int4> fr(n_blocks);
    for (int32_t b = 0; b < n_blocks; ++b) {
        if (frames) {
            const int32_t* f = frames + 4 * b;
            if (f[0] < 0 || f[1] < 0 || f[2] > KDT_COORD_LIMIT || f[3] > KDT_COORD_LIMIT ||
                f[0] >= f[2] || f[1] >= f[3])
                return KDT_E_RANGE;
            fr[b] = make_int4(f[0], f[1], f[2], f[3]);
        } else {
            fr[b] = make_int4(0, 0, KDT_COORD_LIMIT, KDT_COORD_LIMIT);
        }
    }
    // per block: range, frame, duplicates, collinearity; Hilbert order
    std::vector<int> order(n);
    {
        std::vector<std::pair<uint64_t, int>> key;
        for (int32_t b = 0; b < n_blocks; ++b) {
            const int64_t lo = block_off[b], hi = block_off[b + 1];
            const int4 f = fr[b];
            int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = 0, mxy = 0;
            for (int64_t i = lo; i < hi; ++i) {
                const int32_t x = xy[2 * i], y = xy[2 * i + 1];
                if (x < 0 || y < 0 || x >= KDT_COORD_LIMIT || y >= KDT_COORD_LIMIT) return KDT_E_RANGE;
                if (x < f.x || x >= f.z || y < f.y || y >= f.w) return KDT_E_RANGE;
                mnx = std::min(mnx, x); mny = std::min(mny, y);
                mxx = std::max(mxx, x); mxy = std::max(mxy, y);
            }
            key.clear();
            for (int64_t i = lo; i < hi; ++i)
                key.push_back({((uint64_t)(uint32_t)xy[2 * i] << 32) | (uint32_t)xy[2 * i + 1], (int)(i - lo)});
            std::sort(key.begin(), key.end());
            for (size_t i = 1; i < key.size(); ++i)
                if (key[i].first == key[i - 1].first) return KDT_E_DUP;
            bool off_line = false;
            const int32_t* p0 = xy + 2 * lo;
            const int32_t* p1 = xy + 2 * (lo + 1);
            for (int64_t i = lo + 2; i < hi && !off_line; ++i) off_line = orient_h(p0, p1, xy + 2 * i) != 0;
            if (!off_line) return KDT_E_DEGEN;
            // Hilbert order over the block's bounding box
            const double sx = 65535.0 / std::max(1, mxx - mnx), sy = 65535.0 / std::max(1, mxy - mny);
            key.clear();
            for (int64_t i = lo; i < hi; ++i) {
                const uint32_t hx = (uint32_t)((xy[2 * i] - mnx) * sx), hy = (uint32_t)((xy[2 * i + 1] - mny) * sy);
                key.push_back({hilbert16(hx, hy), (int)(i - lo)});
            }
            std::sort(key.begin(), key.end());
            for (int64_t i = lo; i < hi; ++i) order[i] = key[i - lo].second;
        }
    }
    const Layout L = make_layout(n, n_blocks, max_staged);
    if (!dev_ws || ws_bytes < L.total) return KDT_E_CAPACITY;
    if (((uintptr_t)dev_ws & 255) != 0) return KDT_E_ARG;

    kdt_ctx* c = new (std::nothrow) kdt_ctx();
    if (!c) return KDT_E_CAPACITY;
    c->stream = (hipStream_t)stream;
    c->B = n_blocks;
    c->n = n;
    c->max_staged = max_staged;
    c->ws = (char*)dev_ws;
    c->L = L;
    c->sticky = KDT_OK;
    (void)hipGetDevice(&c->device);
    c->pt_off.assign(block_off, block_off + n_blocks + 1);
    c->tri_off.resize(n_blocks + 1);
    c->tri_off[0] = 0;
    for (int32_t b = 0; b < n_blocks; ++b)
        c->tri_off[b + 1] = c->tri_off[b] + 2 * (c->pt_off[b + 1] - c->pt_off[b]) - 2;
    char* w = c->ws;
    c->dev.tri = (Tri*)(w + L.tri);
    c->dev.xy = (int2*)(w + L.xy);
    c->dev.vtri = (int*)(w + L.vtri);
    c->dev.pt_off = (const long long*)(w + L.pt_off);
    c->dev.tri_off = (const long long*)(w + L.tri_off);
    c->dev.frame = (const int4*)(w + L.frame);
    c->dev.status = (int*)(w + L.status);
    c->dev.stats = (BlockStats*)(w + L.stats);
    c->dev.sticky = (int*)(w + L.sticky);
    c->dev.order = (const int*)(w + L.order);
    c->dev.owner = (int*)(w + L.qmap);
    c->dev.own2 = (int*)(w + L.own2);
    c->dev.rb_list = (int*)(w + L.rb_flag);
    c->dev.policy = KDT_POLICY_REPAIR;
    c->dev.tau = 0.f;
    c->dev.dlim = 0.f;
    c->dev.prefetch = 1;
    c->dev.mlp_w = nullptr;
    c->dev.log = nullptr;
    c->dev.log_cap = 0;
    c->dev.n_blocks = n_blocks;
    hipStream_t s = c->stream;
    int rc = KDT_OK;
    // The host arrays are pageable: these copies complete before returning.
    rc |= check_hip(c, hipMemcpyAsync(w + L.xy, xy, sizeof(int2) * n, hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + L.order, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + L.pt_off, c->pt_off.data(), sizeof(long long) * (n_blocks + 1), hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + L.tri_off, c->tri_off.data(), sizeof(long long) * (n_blocks + 1), hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + L.frame, fr.data(), sizeof(int4) * n_blocks, hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemsetAsync(w + L.status, 0, sizeof(int) * n_blocks, s));
    rc |= check_hip(c, hipMemsetAsync(w + L.rb_flag, 0, sizeof(int) * (n_blocks + 2), s));
    rc |= check_hip(c, hipMemsetAsync(w + L.stats, 0, sizeof(BlockStats) * n_blocks, s));
    rc |= check_hip(c, hipMemsetAsync(w + L.sticky, 0, sizeof(int) * 4, s));
    rc |= check_hip(c, hipMemsetAsync(w + L.rest_cnt, 0, sizeof(int) * n_blocks, s));
    c->rest.mv = (kdt_move_t*)(w + L.rest_mv);
    c->rest.idx = (int*)(w + L.rest_idx);
    c->rest.app = (int8_t*)(w + L.rest_app);
    c->rest.cnt = (int*)(w + L.rest_cnt);
    {
        // block order of the persistent launch: largest blocks first
        std::vector<int> lpt(n_blocks);
        for (int32_t b = 0; b < n_blocks; ++b) lpt[b] = b;
        std::stable_sort(lpt.begin(), lpt.end(), [&](int x, int y) {
            return c->pt_off[x + 1] - c->pt_off[x] > c->pt_off[y + 1] - c->pt_off[y];
        });
        rc |= check_hip(c, hipMemcpyAsync(w + L.lpt, lpt.data(), sizeof(int) * n_blocks, hipMemcpyHostToDevice, s));
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
        c->cus = cus;
        c->wpc = step_wg_per_cu(dev);
    }
    if (rc != KDT_OK) { delete c; return KDT_E_DEVICE; }
    c->pb_lds = (int)(pb_fixed_lds() + max_block_need(c, 0, pb_lds_bytes() - pb_fixed_lds()));
    c->dev.step_lds = 0;
    k_build_blocks<<<n_blocks, PB_THREADS, c->pb_lds, s>>>(c->dev, c->pb_lds);
    if (check_hip(c, hipGetLastError()) != KDT_OK) { delete c; return KDT_E_DEVICE; }
    rc = check_hip(c, hipStreamSynchronize(s));
    if (rc != KDT_OK) { delete c; return rc; }
    // a block whose build failed (a local limit, an invariant) fails the init
    int built = 0;
    if (check_hip(c, hipMemcpy(&built, c->dev.sticky, sizeof(int), hipMemcpyDeviceToHost)) != KDT_OK) {
        delete c;
        return KDT_E_DEVICE;
    }
    if (built != 0) { delete c; return built; }
    *out = c;
    return KDT_OK;
}

// Validation of one staged move: KDT_OK, KDT_E_ARG or KDT_E_CAPACITY.
static int stage_one(kdt_ctx* c, int32_t block, int64_t point, int32_t dir, int32_t dist) {
    if (block < 0 || block >= c->B) return KDT_E_ARG;
    if (point < 0 || point >= c->pt_off[block + 1] - c->pt_off[block]) return KDT_E_ARG;
    if (dir < 0 || dir > 3 || dist < 1) return KDT_E_ARG;
    if ((int64_t)c->staged.size() >= c->max_staged) return KDT_E_CAPACITY;
    kdt_move_t m;
    m.point = (int32_t)point;
    m.dir = dir;
    m.dist = dist;
    m.pad = 0;
    c->staged.push_back(m);
    c->staged_block.push_back(block);
    return KDT_OK;
}

int kdt_move(kdt_ctx* c, int32_t block, int64_t point, int32_t dir, int32_t dist) {
    if (!c) return KDT_E_ARG;
    if (c->global) return KDT_E_STATE;
    return stage_one(c, block, point, dir, dist);
}

int kdt_moves(kdt_ctx* c, const int32_t* blocks, const kdt_move_t* moves, int64_t count, int32_t* status) {
    if (!c || count < 0 || (count > 0 && (!blocks || !moves))) return KDT_E_ARG;
    if (c->global) return KDT_E_STATE;
    int rc = KDT_OK;
    for (int64_t i = 0; i < count; ++i) {
        const int st = stage_one(c, blocks[i], moves[i].point, moves[i].dir, moves[i].dist);
        if (status) status[i] = st;
        if (st != KDT_OK && rc == KDT_OK) rc = st;
    }
    return rc;
}

}  // extern "C"

namespace {

// Launch the staged moves as one time step: grouped by block (list order
// kept within a block), copied to the workspace, one k_step launch; `order`
// (if given) receives the staging index of each launched move.
int launch_staged(kdt_ctx* c, int8_t* applied, std::vector<int>* order) {
    std::vector<int> idx(c->staged.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int a, int b) { return c->staged_block[a] < c->staged_block[b]; });
    std::vector<kdt_move_t> mv(idx.size());
    std::vector<int> off(c->B + 1, 0);
    for (size_t i = 0; i < idx.size(); ++i) {
        mv[i] = c->staged[idx[i]];
        off[c->staged_block[idx[i]] + 1]++;
    }
    for (int32_t b = 0; b < c->B; ++b) off[b + 1] += off[b];
    c->staged.clear();
    c->staged_block.clear();
    char* w = c->ws;
    int rc = KDT_OK;
    if (!mv.empty())
        rc |= check_hip(c, hipMemcpyAsync(w + c->L.stage_mv, mv.data(), sizeof(kdt_move_t) * mv.size(),
                                          hipMemcpyHostToDevice, c->stream));
    rc |= check_hip(c, hipMemcpyAsync(w + c->L.stage_off, off.data(), sizeof(int) * (c->B + 1),
                                      hipMemcpyHostToDevice, c->stream));
    // the host vectors are pageable: wait before they go out of scope
    rc |= check_hip(c, hipStreamSynchronize(c->stream));
    if (rc != KDT_OK) return KDT_E_DEVICE;
    hipEvent_t e0 = timing_begin(c);
    k_step<<<c->B, WAVE, c->dev.step_lds, c->stream>>>(c->dev, (const kdt_move_t*)(w + c->L.stage_mv),
                                                       (const int*)(w + c->L.stage_off), applied, c->step_count);
    if (c->dev.policy != KDT_POLICY_REPAIR && c->follow)  // blocks the rebuild branch listed
        k_build_listed<<<std::min(c->B, 8 * c->cus), PB_THREADS, c->pb_lds_follow, c->stream>>>(c->dev, c->step_count,
                                                                                            c->pb_lds_follow);
    c->step_count++;
    timing_end(c, e0);
    if (order) order->swap(idx);
    return check_hip(c, hipGetLastError());
}

}  // namespace

extern "C" {

int kdt_step(kdt_ctx* c) {
    if (!c) return KDT_E_ARG;
    if (c->global) return KDT_E_STATE;
    if (c->sticky != KDT_OK) return KDT_E_STATE;
    return launch_staged(c, nullptr, nullptr);
}

int kdt_step_status(kdt_ctx* c, int32_t* status) {
    if (!c) return KDT_E_ARG;
    if (c->global) return KDT_E_STATE;
    if (c->sticky != KDT_OK) return KDT_E_STATE;
    const size_t m = c->staged.size();
    if (m > 0 && !status) return KDT_E_ARG;
    int8_t* app = (int8_t*)(c->ws + c->L.stage_app);
    std::vector<int> order;
    int rc = KDT_OK;
    if (m > 0) rc = check_hip(c, hipMemsetAsync(app, 0, m, c->stream));
    if (rc == KDT_OK) rc = launch_staged(c, app, &order);
    if (rc != KDT_OK) return rc;
    rc = kdt_sync(c);
    if (rc != KDT_OK) return rc;
    std::vector<int8_t> h(m);
    if (m > 0 && check_hip(c, hipMemcpy(h.data(), app, m, hipMemcpyDeviceToHost))) return KDT_E_DEVICE;
    for (size_t i = 0; i < m; ++i) status[order[i]] = h[i] ? KDT_OK : KDT_BLOCKED;
    return KDT_OK;
}

}  // extern "C"

namespace {

// Enqueue n_steps time steps on the context's stream (timing events if on).
int enqueue_steps(kdt_ctx* c, const kdt_move_t* moves, const int32_t* step_off, int32_t n_steps,
                  int8_t* applied, int32_t flags, bool timed) {
    char* w = c->ws;
    if (flags == KDT_RUN_FUSED) {
        hipEvent_t e0 = timed ? timing_begin(c) : nullptr;
        k_run_fused<<<c->B, WAVE, c->dev.step_lds, c->stream>>>(c->dev, moves, step_off, n_steps, c->B, applied,
                                                                c->step_count);
        c->step_count += n_steps;
        if (timed) timing_end(c, e0);
        return check_hip(c, hipGetLastError());
    }
    const int grid = std::max(1, std::min(c->B, c->cus * c->persist_per_cu));
    for (int32_t t = 0; t < n_steps; ++t) {
        const int32_t* off = step_off + (int64_t)t * (c->B + 1);
        hipEvent_t e0 = timed ? timing_begin(c) : nullptr;
        if (flags == KDT_RUN_PERSISTENT) {
            k_step_persist<<<grid, WAVE, c->dev.step_lds, c->stream>>>(c->dev, moves, off, (const int*)(w + c->L.lpt),
                                                                       c->B, applied, c->step_count);
        } else {
            // a rebuilding policy: every block's branch chosen first, by all
            // blocks at once, so the step kernels only read it
            DevState dv = c->dev;
            if (c->dev.policy != KDT_POLICY_REPAIR) {
                // a chunk of steps at a time (one step when logging: the log
                // ring may hold fewer steps than a chunk)
                const int chunk = c->dev.log ? 1 : CHOOSE_STEPS;
                int8_t* ch = (int8_t*)(w + c->L.choice);
                if (t % chunk == 0)
                    k_choose<<<dim3(c->B, std::min(chunk, n_steps - t)), WAVE, 0, c->stream>>>(
                        c->dev, moves, off, c->step_count, ch);
                dv.choice = ch + (long long)(t % chunk) * c->B;
            }
            // the step's order (most moves first) and, for the split launch,
            // its heavy class: the blocks with at least heavy_cut moves
            int* ord = nullptr;
            const bool split = c->block_waves > 1 && c->heavy_cut > 0;
            const bool mid = split && c->block_waves == 4 && c->mid_cut > 0;
            if (c->block_order || split) {
                // the orders of up to ORDER_STEPS steps at a time
                int* ord0 = (int*)(w + c->L.sorder);
                const int cut = split ? c->heavy_cut : DRYMAX + 2;
                if (t % ORDER_STEPS == 0)
                    k_order<<<std::min(ORDER_STEPS, n_steps - t), 1024, 0, c->stream>>>(
                        off, c->B, cut, mid ? c->mid_cut : cut, ord0);
                ord = ord0 + (long long)(t % ORDER_STEPS) * (c->B + 2);
            }
            hipStream_t mws = c->stream;
            if (split) {  // heavy (and middle) blocks on side streams, at the same time as the others
                if (check_hip(c, hipEventRecord(c->fork_ev, c->stream)) ||
                    check_hip(c, hipStreamWaitEvent(c->side, c->fork_ev, 0)) ||
                    (mid && check_hip(c, hipStreamWaitEvent(c->side2, c->fork_ev, 0))))
                    return KDT_E_DEVICE;
                mws = c->side;
            }
            if (c->block_waves == 4)
                k_step_mw<4><<<c->B, 4 * WAVE, sizeof(MwLDS<4>), mws>>>(
                    dv, moves, off, applied, c->step_count, c->rest, ord, split ? PART_HEAVY : PART_ALL);
            else if (c->block_waves == 2)
                k_step_mw<2><<<c->B, 2 * WAVE, sizeof(MwLDS<2>), mws>>>(
                    dv, moves, off, applied, c->step_count, c->rest, ord, split ? PART_HEAVY : PART_ALL);
            if (mid)
                k_step_mw<2><<<c->B, 2 * WAVE, sizeof(MwLDS<2>), c->side2>>>(dv, moves, off, applied,
                                                                            c->step_count, c->rest, ord, PART_MID);
            if (c->block_waves == 1 || split)
                k_step<<<c->B, WAVE, c->dev.step_lds, c->stream>>>(dv, moves, off, applied, c->step_count, ord,
                                                                   split ? PART_LIGHT : PART_ALL);
            if (split && (check_hip(c, hipEventRecord(c->join_ev, c->side)) ||
                          check_hip(c, hipStreamWaitEvent(c->stream, c->join_ev, 0))))
                return KDT_E_DEVICE;
            if (mid && (check_hip(c, hipEventRecord(c->join2_ev, c->side2)) ||
                        check_hip(c, hipStreamWaitEvent(c->stream, c->join2_ev, 0))))
                return KDT_E_DEVICE;
            if (c->block_waves > 1)
                k_step_rest<<<c->B, WAVE, c->dev.step_lds, c->stream>>>(dv, moves, off, c->rest, applied,
                                                                        c->step_count);
        }
        if (c->dev.policy != KDT_POLICY_REPAIR && c->follow)  // blocks the rebuild branch listed
            k_build_listed<<<std::min(c->B, 8 * c->cus), PB_THREADS, c->pb_lds_follow, c->stream>>>(
                c->dev, c->step_count, c->pb_lds_follow);
        c->step_count++;
        if (timed) timing_end(c, e0);
    }
    return check_hip(c, hipGetLastError());
}

bool valid_flags(int32_t f) { return f == KDT_RUN_PER_STEP || f == KDT_RUN_FUSED || f == KDT_RUN_PERSISTENT; }

}  // namespace

struct kdt_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    kdt_ctx* ctx;
    long long epoch;  // the context's epoch when captured
};

extern "C" {

int kdt_run(kdt_ctx* c, const kdt_move_t* moves, const int32_t* step_off, int32_t n_steps,
            int8_t* applied, int32_t flags) {
    if (!c || n_steps < 0 || (n_steps > 0 && (!moves || !step_off))) return KDT_E_ARG;
    if (!valid_flags(flags)) return KDT_E_ARG;
    if (c->sticky != KDT_OK || c->global) return KDT_E_STATE;
    if (n_steps == 0) return KDT_OK;
    return enqueue_steps(c, moves, step_off, n_steps, applied, flags, true);
}

int kdt_set_launch(kdt_ctx* c, int32_t persist_per_cu) {
    if (!c || persist_per_cu < 1 || persist_per_cu > 64) return KDT_E_ARG;
    c->persist_per_cu = persist_per_cu;
    c->epoch++;
    return KDT_OK;
}

int kdt_set_repair(kdt_ctx* c, int32_t variant) {
    if (!c || (variant != KDT_REPAIR_DELINS && variant != KDT_REPAIR_FLIP)) return KDT_E_ARG;
    if (c->global) return KDT_E_STATE;
    c->dev.repair = variant;
    c->epoch++;
    return KDT_OK;
}

int kdt_set_prefetch(kdt_ctx* c, int32_t depth) {
    if (!c || depth < 0 || depth > 2) return KDT_E_ARG;
    c->dev.prefetch = depth;
    c->epoch++;
    return KDT_OK;
}

int kdt_set_block_order(kdt_ctx* c, int32_t order, int32_t heavy_cut, int32_t mid_cut) {
    if (!c || (order != 0 && order != 1) || heavy_cut < 0 || (heavy_cut > 0 && !order) || mid_cut < 0 ||
        (mid_cut > 0 && (heavy_cut == 0 || mid_cut >= heavy_cut)))
        return KDT_E_ARG;
    if (c->global) return KDT_E_STATE;
    // the class streams and events belong to the context's device
    int cur = 0;
    if ((heavy_cut > 0 && !c->side) || (mid_cut > 0 && !c->side2)) {
        if (check_hip(c, hipGetDevice(&cur)) || check_hip(c, hipSetDevice(c->device))) return KDT_E_DEVICE;
        int rc = KDT_OK;
        if (heavy_cut > 0 && !c->side &&
            (check_hip(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking)) ||
             check_hip(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming)) ||
             check_hip(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming))))
            rc = KDT_E_DEVICE;
        if (rc == KDT_OK && mid_cut > 0 && !c->side2 &&
            (check_hip(c, hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking)) ||
             check_hip(c, hipEventCreateWithFlags(&c->join2_ev, hipEventDisableTiming))))
            rc = KDT_E_DEVICE;
        if (check_hip(c, hipSetDevice(cur))) rc = KDT_E_DEVICE;
        if (rc != KDT_OK) return rc;
    }
    c->block_order = order;
    c->heavy_cut = heavy_cut;
    c->mid_cut = mid_cut;
    c->epoch++;
    return KDT_OK;
}

int kdt_set_block_waves(kdt_ctx* c, int32_t waves) {
    if (!c || (waves != 1 && waves != 2 && waves != 4)) return KDT_E_ARG;
    if (c->global) return KDT_E_STATE;
    if (waves > 1 && !mw_lds_ok()) return KDT_E_DEVICE;
    c->block_waves = waves;
    c->epoch++;
    return KDT_OK;
}

int kdt_graph_build(kdt_ctx* c, const kdt_move_t* moves, const int32_t* step_off, int32_t n_steps,
                    int8_t* applied, int32_t flags, kdt_graph** out) {
    if (!c || !out || n_steps < 1 || !moves || !step_off || !valid_flags(flags)) return KDT_E_ARG;
    *out = nullptr;
    if (c->sticky != KDT_OK || c->global) return KDT_E_STATE;
    if (c->stream == nullptr) return KDT_E_STATE;  // the null stream cannot be captured
    kdt_graph* g = new (std::nothrow) kdt_graph();
    if (!g) return KDT_E_CAPACITY;
    g->ctx = c;
    g->epoch = c->epoch;
    if (check_hip(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal))) {
        delete g;
        return KDT_E_DEVICE;
    }
    const int rc = enqueue_steps(c, moves, step_off, n_steps, applied, flags, false);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (rc != KDT_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        c->sticky = KDT_E_DEVICE;
        return KDT_E_DEVICE;
    }
    g->graph = graph;
    if (check_hip(c, hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0))) {
        (void)hipGraphDestroy(graph);
        delete g;
        return KDT_E_DEVICE;
    }
    *out = g;
    return KDT_OK;
}

int kdt_graph_launch(kdt_ctx* c, kdt_graph* g) {
    if (!c || !g || g->ctx != c) return KDT_E_ARG;
    if (c->sticky != KDT_OK || g->epoch != c->epoch) return KDT_E_STATE;
    return check_hip(c, hipGraphLaunch(g->exec, c->stream));
}

void kdt_graph_destroy(kdt_graph* g) {
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}

int kdt_set_policy(kdt_ctx* c, int32_t policy, float tau, const float* mlp_w) {
    if (!c || policy < KDT_POLICY_REPAIR || policy > KDT_POLICY_DLIMIT) return KDT_E_ARG;
    if (policy == KDT_POLICY_MLP && !mlp_w) return KDT_E_ARG;
    c->dev.policy = policy;
    c->dev.tau = tau;
    c->dev.mlp_w = mlp_w;
    c->epoch++;
    if (!c->global) plan_rebuild_lds(c);
    return KDT_OK;
}

int kdt_set_log(kdt_ctx* c, float* log, int64_t cap_steps) {
    if (!c || cap_steps < 0 || (cap_steps > 0 && !log)) return KDT_E_ARG;
    c->dev.log = cap_steps > 0 ? log : nullptr;
    c->dev.log_cap = cap_steps;
    c->step_count = 0;
    c->epoch++;
    return KDT_OK;
}

int kdt_mlp_forward(const float* w, const float* x, int64_t n, float* out, void* stream) {
    if (!w || n < 0 || (n > 0 && (!x || !out))) return KDT_E_ARG;
    if (n == 0) return KDT_OK;
    k_mlp_forward<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(w, x, n, out);
    return hipGetLastError() == hipSuccess ? KDT_OK : KDT_E_DEVICE;
}

int kdt_mlp_grad(const float* w, const float* x, const float* y, int64_t n, float* grad, void* stream) {
    if (!w || !grad || n < 1 || !x || !y) return KDT_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    k_mlp_grad<<<1, MLP_THREADS, 0, s>>>(w, x, y, n, grad, 0);
    return hipGetLastError() == hipSuccess ? KDT_OK : KDT_E_DEVICE;
}

int kdt_mlp_train(float* w, const float* x, const float* y, int64_t n, int32_t epochs, int32_t batch,
                  float lr, float* gbuf, void* stream) {
    if (!w || !x || !y || !gbuf || n < 1 || epochs < 0 || batch < 1) return KDT_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    for (int32_t e = 0; e < epochs; ++e) {
        for (int64_t b0 = 0; b0 < n; b0 += batch) {
            const int64_t nb = std::min<int64_t>(batch, n - b0);
            k_mlp_grad<<<1, MLP_THREADS, 0, s>>>(w, x + b0 * MLP_IN, y + b0 * MLP_OUT, nb, gbuf, 0);
            k_mlp_sgd<<<(KDT_MLP_PARAMS + 255) / 256, 256, 0, s>>>(w, gbuf, lr, 1.f / (float)nb);
        }
    }
    return hipGetLastError() == hipSuccess ? KDT_OK : KDT_E_DEVICE;
}

int kdt_mlp_train_noalloc(float* w, const float* x, const float* y, int64_t n, int32_t epochs, int32_t batch,
                          float lr, void* stream) {
    if (!w || !x || !y || n < 1 || epochs < 0 || batch < 1) return KDT_E_ARG;
    if (batch > KDT_MLP_NOALLOC_BATCH) return KDT_E_CAPACITY;
    float* S = nullptr;
    const int rc = noalloc_scratch(&S);
    if (rc != KDT_OK) return rc;
    float* total = S + (long long)NOALLOC_ROWS * NOALLOC_ROW;
    hipStream_t s = (hipStream_t)stream;
    for (int32_t e = 0; e < epochs; ++e) {
        for (int64_t b0 = 0; b0 < n; b0 += batch) {
            const int64_t nb = std::min<int64_t>(batch, n - b0);
            const int rows = (int)((nb + MLP_CHUNK - 1) / MLP_CHUNK);  // one workgroup per chunk
            k_mlp_grad<<<rows, MLP_THREADS, 0, s>>>(w, x + b0 * MLP_IN, y + b0 * MLP_OUT, nb, S, NOALLOC_ROW);
            k_mlp_reduce<<<(MLP_GRAD_N + 255) / 256, 256, 0, s>>>(S, rows, NOALLOC_ROW, total);
            k_mlp_sgd<<<(KDT_MLP_PARAMS + 255) / 256, 256, 0, s>>>(w, total, lr, 1.f / (float)nb);
        }
    }
    return hipGetLastError() == hipSuccess ? KDT_OK : KDT_E_DEVICE;
}

int kdt_sync(kdt_ctx* c) {
    if (!c) return KDT_E_ARG;
    if (c->sticky != KDT_OK) return c->sticky;
    if (check_hip(c, hipStreamSynchronize(c->stream)) != KDT_OK) return KDT_E_DEVICE;
    int dev_sticky = 0;
    if (check_hip(c, hipMemcpy(&dev_sticky, c->dev.sticky, sizeof(int), hipMemcpyDeviceToHost)) != KDT_OK)
        return KDT_E_DEVICE;
    if (dev_sticky != 0) c->sticky = dev_sticky;
    return c->sticky;
}

int kdt_query(kdt_ctx* c, int32_t* tris, int32_t* adj, int64_t* blk_off, int64_t cap, int64_t* n_tri) {
    if (!c || !n_tri || cap < 0 || (cap > 0 && !tris)) return KDT_E_ARG;
    int rc = kdt_sync(c);
    if (rc != KDT_OK) return rc;
    char* w = c->ws;
    int* qmap = (int*)(w + c->L.qmap);
    int* qcount = (int*)(w + c->L.qcount);
    k_qcount<<<c->B, WAVE, 0, c->stream>>>(c->dev, nullptr, qmap, qcount);
    if (check_hip(c, hipGetLastError()) != KDT_OK) return KDT_E_DEVICE;
    std::vector<int> cnt(c->B);
    if (check_hip(c, hipMemcpyAsync(cnt.data(), qcount, sizeof(int) * c->B, hipMemcpyDeviceToHost, c->stream)) ||
        check_hip(c, hipStreamSynchronize(c->stream)))
        return KDT_E_DEVICE;
    std::vector<long long> off(c->B + 1, 0);
    for (int32_t b = 0; b < c->B; ++b) off[b + 1] = off[b] + cnt[b];
    *n_tri = off[c->B];
    if (blk_off)
        for (int32_t b = 0; b <= c->B; ++b) blk_off[b] = off[b];
    if (off[c->B] > cap) return KDT_E_CAPACITY;
    if (check_hip(c, hipMemcpyAsync(w + c->L.qoff, off.data(), sizeof(long long) * (c->B + 1),
                                    hipMemcpyHostToDevice, c->stream)))
        return KDT_E_DEVICE;
    k_qwrite<<<c->B, WAVE, 0, c->stream>>>(c->dev, nullptr, qmap, (const long long*)(w + c->L.qoff), tris, adj);
    if (check_hip(c, hipGetLastError()) || check_hip(c, hipStreamSynchronize(c->stream))) return KDT_E_DEVICE;
    return KDT_OK;
}

int kdt_query_canonical(kdt_ctx* c, int32_t* host_tris, int64_t cap, int64_t* n_tri) {
    if (!c || !n_tri || cap < 0 || (cap > 0 && !host_tris)) return KDT_E_ARG;
    // device staging of the compacted list lives in the workspace
    const int64_t max_tri = 2 * c->n - 2 * (int64_t)c->B;
    void* dbuf = c->ws + c->L.qtris;
    int64_t nt = 0;
    int rc = kdt_query(c, (int32_t*)dbuf, nullptr, nullptr, max_tri, &nt);
    *n_tri = nt;
    std::vector<int32_t> h;
    if (rc == KDT_OK) {
        h.resize(3 * (size_t)nt);
        if (check_hip(c, hipMemcpy(h.data(), dbuf, sizeof(int32_t) * 3 * (size_t)nt, hipMemcpyDeviceToHost)))
            rc = KDT_E_DEVICE;
    }
    if (rc != KDT_OK) return rc;
    if (nt > cap) return KDT_E_CAPACITY;
    std::vector<int64_t> idx(nt);
    for (int64_t i = 0; i < nt; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        const int32_t* x = &h[3 * a];
        const int32_t* y = &h[3 * b];
        if (x[0] != y[0]) return x[0] < y[0];
        if (x[1] != y[1]) return x[1] < y[1];
        return x[2] < y[2];
    });
    for (int64_t i = 0; i < nt; ++i)
        for (int j = 0; j < 3; ++j) host_tris[3 * i + j] = h[3 * idx[i] + j];
    return KDT_OK;
}

int kdt_query_blocks(kdt_ctx* c, const int32_t* blocks, int32_t count, int32_t* host_tris, int32_t* host_adj,
                     int64_t cap, int64_t* host_off) {
    if (!c || !blocks || !host_off || count < 1 || cap < 0 || (cap > 0 && !host_tris)) return KDT_E_ARG;
    if (c->global ? count != 1 : count > c->B) return KDT_E_ARG;
    {
        std::vector<char> seen(c->B, 0);
        for (int32_t i = 0; i < count; ++i) {
            const int32_t b = blocks[i];
            if (b < 0 || b >= c->B || seen[b]) return KDT_E_ARG;  // each block at most once
            seen[b] = 1;
        }
    }
    // blocks are independent: the listed ones can be read while another
    // block has failed (its error is sticky for the context), unless one of
    // them is the failed block or the runtime failed
    if (check_hip(c, hipStreamSynchronize(c->stream))) return KDT_E_DEVICE;
    int rc = kdt_sync(c);
    if (rc == KDT_E_DEVICE || (rc != KDT_OK && c->global)) return rc;
    if (rc != KDT_OK) {
        std::vector<int32_t> bst(c->B);
        if (check_hip(c, hipMemcpyAsync(bst.data(), c->dev.status, sizeof(int32_t) * c->B, hipMemcpyDeviceToHost,
                                        c->stream)) ||
            check_hip(c, hipStreamSynchronize(c->stream)))
            return KDT_E_DEVICE;
        for (int32_t i = 0; i < count; ++i)
            if (bst[blocks[i]] != 0) return bst[blocks[i]];
    }
    char* w = c->ws;
    int* qmap = (int*)(w + c->L.qmap);
    int* qcount = (int*)(w + c->L.qcount);
    int* qlist = (int*)(w + c->L.qlist);
    int* dtris = (int*)(w + c->L.qtris);
    int* dadj = (int*)(w + c->L.qadj);
    std::vector<int> cnt(count);
    if (check_hip(c, hipMemcpyAsync(qlist, blocks, sizeof(int) * count, hipMemcpyHostToDevice, c->stream)))
        return KDT_E_DEVICE;
    k_qcount<<<count, WAVE, 0, c->stream>>>(c->dev, qlist, qmap, qcount);
    if (check_hip(c, hipGetLastError()) ||
        check_hip(c, hipMemcpyAsync(cnt.data(), qcount, sizeof(int) * count, hipMemcpyDeviceToHost, c->stream)) ||
        check_hip(c, hipStreamSynchronize(c->stream)))
        return KDT_E_DEVICE;
    std::vector<long long> off(count + 1, 0);
    for (int32_t i = 0; i < count; ++i) off[i + 1] = off[i] + cnt[i];
    for (int32_t i = 0; i <= count; ++i) host_off[i] = off[i];
    const int64_t nt = off[count];
    if (nt > cap) return KDT_E_CAPACITY;
    if (check_hip(c, hipMemcpyAsync(w + c->L.qoff, off.data(), sizeof(long long) * (count + 1),
                                    hipMemcpyHostToDevice, c->stream)))
        return KDT_E_DEVICE;
    k_qwrite<<<count, WAVE, 0, c->stream>>>(c->dev, qlist, qmap, (const long long*)(w + c->L.qoff), dtris,
                                            host_adj ? dadj : nullptr);
    std::vector<int32_t> t(3 * (size_t)nt), a(host_adj ? 3 * (size_t)nt : 0);
    if (check_hip(c, hipGetLastError()) ||
        (nt > 0 && check_hip(c, hipMemcpyAsync(t.data(), dtris, sizeof(int32_t) * 3 * nt, hipMemcpyDeviceToHost,
                                               c->stream))) ||
        (nt > 0 && host_adj &&
         check_hip(c, hipMemcpyAsync(a.data(), dadj, sizeof(int32_t) * 3 * nt, hipMemcpyDeviceToHost, c->stream))) ||
        check_hip(c, hipStreamSynchronize(c->stream)))
        return KDT_E_DEVICE;
    // canonical order within every listed block; adjacency rows follow
    std::vector<int64_t> idx, inv;
    for (int32_t i = 0; i < count; ++i) {
        const int64_t o0 = off[i], m = off[i + 1] - off[i];
        idx.resize(m);
        for (int64_t k = 0; k < m; ++k) idx[k] = o0 + k;
        std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
            const int32_t* p = &t[3 * x];
            const int32_t* q = &t[3 * y];
            if (p[0] != q[0]) return p[0] < q[0];
            if (p[1] != q[1]) return p[1] < q[1];
            return p[2] < q[2];
        });
        if (host_adj) {
            inv.resize(m);
            for (int64_t k = 0; k < m; ++k) inv[idx[k] - o0] = o0 + k;
        }
        for (int64_t k = 0; k < m; ++k)
            for (int j = 0; j < 3; ++j) {
                host_tris[3 * (o0 + k) + j] = t[3 * idx[k] + j];
                if (host_adj) {
                    const int32_t r = a[3 * idx[k] + j];
                    host_adj[3 * (o0 + k) + j] = r < 0 ? -1 : (int32_t)inv[r - o0];
                }
            }
    }
    return KDT_OK;
}

int kdt_digest(kdt_ctx* c, uint64_t* host_per_block) {
    if (!c || !host_per_block) return KDT_E_ARG;
    int rc = kdt_sync(c);
    if (rc != KDT_OK) return rc;
    unsigned long long* d = (unsigned long long*)(c->ws + c->L.qtris);  // query staging, >= 8 B per block
    k_digest<<<c->B, WAVE, 0, c->stream>>>(c->dev, d);
    if (check_hip(c, hipGetLastError())) return KDT_E_DEVICE;
    if (check_hip(c, hipMemcpyAsync(host_per_block, d, sizeof(uint64_t) * c->B, hipMemcpyDeviceToHost, c->stream)) ||
        check_hip(c, hipStreamSynchronize(c->stream)))
        return KDT_E_DEVICE;
    return KDT_OK;
}

int kdt_dcalc(kdt_ctx* c, int32_t N, int64_t* host_mind2, int64_t* host_diam2, int64_t* d2_now, int64_t* d2_min,
              double* host_spread) {
    if (!c || N < 1 || N > DC_NMAX) return KDT_E_ARG;
    int rc = kdt_sync(c);
    if (rc != KDT_OK) return rc;
    char* w = c->ws;
    long long* mind2 = (long long*)(w + c->L.dc_mind2);
    long long* diam2 = (long long*)(w + c->L.dc_diam2);
    unsigned long long* g = (unsigned long long*)(w + c->L.dc_g);
    const unsigned long long init[2] = {(unsigned long long)DC_NONE, 0ull};
    if (check_hip(c, hipMemcpyAsync(g, init, sizeof(init), hipMemcpyHostToDevice, c->stream))) return KDT_E_DEVICE;
    k_dcalc<<<c->B, WAVE, 0, c->stream>>>(c->dev, N, mind2, diam2, g, (int*)(g + 1));
    std::vector<long long> m(c->B), d(c->B);
    unsigned long long gh[2];
    if (check_hip(c, hipGetLastError()) ||
        check_hip(c, hipMemcpyAsync(m.data(), mind2, sizeof(long long) * c->B, hipMemcpyDeviceToHost, c->stream)) ||
        check_hip(c, hipMemcpyAsync(d.data(), diam2, sizeof(long long) * c->B, hipMemcpyDeviceToHost, c->stream)) ||
        check_hip(c, hipMemcpyAsync(gh, g, sizeof(gh), hipMemcpyDeviceToHost, c->stream)) ||
        check_hip(c, hipStreamSynchronize(c->stream)))
        return KDT_E_DEVICE;
    if (gh[1] != 0) return KDT_E_CAPACITY;  // a search beyond its candidate capacity
    if (N != c->dc_n) {  // a new N starts a new history
        c->dc_n = N;
        c->dc_d2 = DC_NONE;
        c->dc_spread.assign(c->B, 0.0);
    }
    const long long now = (long long)gh[0];
    c->dc_d2 = std::min(c->dc_d2, now);
    if (now != DC_NONE)
        for (int32_t b = 0; b < c->B; ++b)
            c->dc_spread[b] = std::max(c->dc_spread[b], std::sqrt((double)d[b] / (double)now));
    if (host_mind2) std::memcpy(host_mind2, m.data(), sizeof(long long) * c->B);
    if (host_diam2) std::memcpy(host_diam2, d.data(), sizeof(long long) * c->B);
    if (d2_now) *d2_now = now;
    if (d2_min) *d2_min = c->dc_d2;
    if (host_spread) std::memcpy(host_spread, c->dc_spread.data(), sizeof(double) * c->B);
    // the selector's view of d (feature 15, the d-limit rule): the running d
    if (c->dc_d2 != DC_NONE) {
        c->dev.dlim = (float)std::sqrt((double)c->dc_d2);
        c->epoch++;
    }
    return KDT_OK;
}

int kdt_positions(kdt_ctx* c, int32_t* host_xy) {
    if (!c || !host_xy) return KDT_E_ARG;
    int rc = kdt_sync(c);
    if (rc != KDT_OK && rc != KDT_E_INTERNAL && rc != KDT_E_CAPACITY) return rc;
    if (check_hip(c, hipMemcpy(host_xy, c->dev.xy, sizeof(int2) * c->n, hipMemcpyDeviceToHost))) return KDT_E_DEVICE;
    return KDT_OK;
}

int kdt_stats(kdt_ctx* c, kdt_stats_t* out) {
    if (!c || !out) return KDT_E_ARG;
    if (check_hip(c, hipStreamSynchronize(c->stream))) return KDT_E_DEVICE;
    std::vector<BlockStats> st(c->B);
    if (check_hip(c, hipMemcpy(st.data(), c->dev.stats, sizeof(BlockStats) * c->B, hipMemcpyDeviceToHost)))
        return KDT_E_DEVICE;
    std::memset(out, 0, sizeof(*out));
    for (const BlockStats& s : st) {
        out->applied += s.applied;
        out->blocked += s.blocked;
        out->star_sum += s.star_sum;
        out->cavity_sum += s.cavity_sum;
        out->walk_sum += s.walk_sum;
        out->tri_touched += s.tri_touched;
        out->alg_bytes += s.alg_bytes;
        out->errors += s.errors;
        out->t_star += s.t_star;
        out->t_locate += s.t_locate;
        out->t_hole += s.t_hole;
        out->t_insert += s.t_insert;
        for (int i = 0; i < 16; ++i) out->hist[i] += s.hist[i];
        out->fast += s.fast;
        out->rebuilt += s.rebuilt;
        out->flipped += s.flipped;
        out->flips += s.flips;
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess) out->clock_khz = khz;
    return KDT_OK;
}

int kdt_block_status(kdt_ctx* c, int32_t* host_status) {
    if (!c || !host_status) return KDT_E_ARG;
    if (check_hip(c, hipStreamSynchronize(c->stream))) return KDT_E_DEVICE;
    if (check_hip(c, hipMemcpy(host_status, c->dev.status, sizeof(int) * c->B, hipMemcpyDeviceToHost)))
        return KDT_E_DEVICE;
    return KDT_OK;
}

int kdt_timing(kdt_ctx* c, int32_t enable) {
    if (!c) return KDT_E_ARG;
    if (check_hip(c, hipStreamSynchronize(c->stream))) return KDT_E_DEVICE;
    if (enable < 0) return KDT_E_ARG;
    c->ev_used = 0;
    c->timing = enable != 0;
    c->timing_period = enable > 0 ? enable : 1;
    c->timing_count = 0;
    c->timing_open = 0;
    if (!c->timing) release_events(c);
    return KDT_OK;
}

int kdt_timing_read(kdt_ctx* c, double* total_ms, int64_t* launches) {
    if (!c || !total_ms || !launches) return KDT_E_ARG;
    if (c->timing_open > 0) timing_close(c);  // a run cut short ends here
    if (check_hip(c, hipStreamSynchronize(c->stream))) return KDT_E_DEVICE;
    double tot = 0.0;
    for (size_t i = 0; i < c->ev_used; ++i) {
        float ms = 0.f;
        if (check_hip(c, hipEventElapsedTime(&ms, c->ev[i].first, c->ev[i].second))) return KDT_E_DEVICE;
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)c->timing_count;
    return KDT_OK;
}

int kdt_workspace_size_global(int64_t n, int32_t depth, int32_t max_moves, size_t* dev_bytes) {
    if (!dev_bytes || n < 1 || depth < 0 || depth > 20 || max_moves < 1 || max_moves > (1 << 22))
        return KDT_E_ARG;
    if (n > (1 << 22)) return KDT_E_CAPACITY;
    const Layout L = make_layout(n, 1, 0);
    *dev_bytes = make_glayout(L.total, n, depth, max_moves).total;
    return KDT_OK;
}

}  // extern "C"

// Quad-treeDvision of the current positions on the device (k_qt_*), level
// by level; the host reads each level's cut count to know when to stop.
static int qt_repartition(kdt_ctx* c) {
    hipStream_t st = c->stream;
    const int n = (int)c->n;
    k_qt_reset<<<(n + 255) / 256, 256, 0, st>>>(c->g, n);
    int nodes = 1;
    for (int lvl = 0; lvl + 2 < QT_LEVELS; ++lvl) {
        k_qt_alloc<<<1, 1024, 0, st>>>(c->g, lvl);
        int info[2] = {0, 0};
        if (check_hip(c, hipGetLastError()) ||
            check_hip(c, hipMemcpyAsync(&info[0], c->g.qlev + lvl + 2, sizeof(int), hipMemcpyDeviceToHost, st)) ||
            check_hip(c, hipMemcpyAsync(&info[1], c->g.qlev + QT_LEVELS, sizeof(int), hipMemcpyDeviceToHost, st)) ||
            check_hip(c, hipStreamSynchronize(st)))
            return KDT_E_DEVICE;
        if (info[1] < 0) return KDT_E_CAPACITY;
        nodes = info[0];
        if (info[1] == 0) break;
        k_qt_down<<<(n + 255) / 256, 256, 0, st>>>(c->dev, c->g, n);
    }
    k_qt_links<<<(nodes + 255) / 256, 256, 0, st>>>(c->g, nodes);
    c->qt_count = nodes;
    return check_hip(c, hipGetLastError());
}

// A global context with kd cells of depth `depth` (qt_thr == 0) or the
// quad-tree cells of threshold qt_thr.
static int init_global(kdt_ctx** out, const int32_t* xy, int64_t n, int32_t depth, int64_t qt_thr,
                       const int32_t* domain, int32_t max_moves, void* dev_ws, size_t ws_bytes, void* stream) {
    if (!out) return KDT_E_ARG;
    *out = nullptr;
    if (!xy || !domain || n < 1 || depth < 0 || depth > 20 || max_moves < 1 || max_moves > (1 << 22))
        return KDT_E_ARG;
    if (n < 4) return KDT_E_DEGEN;
    if (n > (1 << 22)) return KDT_E_CAPACITY;
    if (n < ((int64_t)1 << depth)) return KDT_E_ARG;
    const int32_t* f = domain;
    if (f[0] < 0 || f[1] < 0 || f[2] > KDT_COORD_LIMIT || f[3] > KDT_COORD_LIMIT || f[0] >= f[2] || f[1] >= f[3])
        return KDT_E_RANGE;
    const int4 fr = make_int4(f[0], f[1], f[2], f[3]);
    int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = 0, mxy = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t x = xy[2 * i], y = xy[2 * i + 1];
        if (x < fr.x || x >= fr.z || y < fr.y || y >= fr.w) return KDT_E_RANGE;
        mnx = std::min(mnx, x); mny = std::min(mny, y);
        mxx = std::max(mxx, x); mxy = std::max(mxy, y);
    }
    std::vector<std::pair<uint64_t, int>> key(n);
    for (int64_t i = 0; i < n; ++i)
        key[i] = {((uint64_t)(uint32_t)xy[2 * i] << 32) | (uint32_t)xy[2 * i + 1], (int)i};
    std::sort(key.begin(), key.end());
    for (int64_t i = 1; i < n; ++i)
        if (key[i].first == key[i - 1].first) return KDT_E_DUP;
    bool off_line = false;
    for (int64_t i = 2; i < n && !off_line; ++i) off_line = orient_h(xy, xy + 2, xy + 2 * i) != 0;
    if (!off_line) return KDT_E_DEGEN;
    // insertion order: Hilbert order over the bounding box
    const double sx = 65535.0 / std::max(1, mxx - mnx), sy = 65535.0 / std::max(1, mxy - mny);
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t hx = (uint32_t)((xy[2 * i] - mnx) * sx), hy = (uint32_t)((xy[2 * i + 1] - mny) * sy);
        key[i] = {hilbert16(hx, hy), (int)i};
    }
    std::sort(key.begin(), key.end());
    std::vector<int> order(n);
    for (int64_t i = 0; i < n; ++i) order[i] = key[i].second;
    // kd cells or quad-tree cells of the initial points
    std::vector<int2> split((size_t)1 << depth, make_int2(0, 0));
    std::vector<int> cell(n), idx(n);
    QtHost QT;
    if (qt_thr > 0) {
        qt_build_host(xy, n, domain, qt_thr, QT);
        cell = QT.cell;
    } else {
        for (int64_t i = 0; i < n; ++i) idx[i] = (int)i;
        kd_build(xy, idx, 0, (size_t)n, 1, 0, depth, split, cell);
    }

    const Layout L = make_layout(n, 1, 0);
    const GLayout G = make_glayout(L.total, n, depth, max_moves, qt_thr > 0 ? qt_capacity(QT, n, qt_thr) : 0);
    if (!dev_ws || ws_bytes < G.total) return KDT_E_CAPACITY;
    if (((uintptr_t)dev_ws & 255) != 0) return KDT_E_ARG;
    kdt_ctx* c = new (std::nothrow) kdt_ctx();
    if (!c) return KDT_E_CAPACITY;
    c->stream = (hipStream_t)stream;
    c->B = 1;
    c->n = n;
    c->max_staged = 0;
    c->ws = (char*)dev_ws;
    c->L = L;
    c->sticky = KDT_OK;
    c->global = true;
    c->depth = depth;
    c->max_moves = max_moves;
    c->hsize = G.hsize;
    (void)hipGetDevice(&c->device);
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
            c->cus = cus;
        c->wpc = wg_per_cu(c->device, sizeof(PlanWave));  // planning workgroups of the rounds
    }
    c->pt_off = {0, (long long)n};
    c->tri_off = {0, 2 * (long long)n - 2};
    char* w = c->ws;
    c->dev.tri = (Tri*)(w + L.tri);
    c->dev.xy = (int2*)(w + L.xy);
    c->dev.vtri = (int*)(w + L.vtri);
    c->dev.pt_off = (const long long*)(w + L.pt_off);
    c->dev.tri_off = (const long long*)(w + L.tri_off);
    c->dev.frame = (const int4*)(w + L.frame);
    c->dev.status = (int*)(w + L.status);
    c->dev.stats = (BlockStats*)(w + L.stats);
    c->dev.sticky = (int*)(w + L.sticky);
    c->dev.order = (const int*)(w + L.order);
    c->dev.owner = (int*)(w + L.qmap);
    c->dev.own2 = (int*)(w + L.own2);
    c->dev.rb_list = (int*)(w + L.rb_flag);
    c->dev.policy = KDT_POLICY_REPAIR;
    c->dev.n_blocks = 1;
    c->g.claim = (unsigned long long*)(w + G.claim);
    c->g.mstate = (int*)(w + G.mstate);
    c->g.rs = (int*)(w + G.rs);
    c->g.rsn = (int*)(w + G.rsn);
    c->g.pslot = (int*)(w + G.pslot);
    c->g.prec = (Tri*)(w + G.prec);
    c->g.pvt = (int2*)(w + G.pvt);
    c->g.phdr = (int4*)(w + G.phdr);
    c->g.pq = (int2*)(w + G.pq);
    c->g.hkey = (unsigned long long*)(w + G.hkey);
    c->g.hcnt = (int*)(w + G.hcnt);
    c->g.hmask = G.hsize - 1;
    c->g.ctr = (int*)(w + G.ctr);
    c->g.serial = (int*)(w + G.serial);
    c->g.split = (const int2*)(w + G.split);
    c->g.depth = depth;
    c->g.qt = qt_thr > 0 ? 1 : 0;
    c->g.qn = (int4*)(w + G.qn);
    c->g.ql = (int4*)(w + G.ql);
    c->g.qcnt = (int*)(w + G.qcnt);
    c->g.qlev = (int*)(w + G.qlev);
    c->g.qcap = qt_thr > 0 ? (int)qt_capacity(QT, n, qt_thr) : 0;
    c->g.qthr = qt_thr;
    c->qt_count = (int)QT.nodes.size();
    c->g.powner = (int*)(w + G.powner);
    c->g.gstats = (unsigned long long*)(w + G.gstats);
    c->g.part = (unsigned long long*)(w + G.part);
    c->gb.ord = (const int*)(w + L.order);
    c->gb.att = (int*)(w + G.att);
    c->gb.pend = (int*)(w + G.pend);
    c->gb.plan = (int2*)(w + G.plan);
    c->gb.deferred = (int*)(w + G.deferred);
    c->gb.big = (int*)(w + G.big);
    hipStream_t s = c->stream;
    int rc = KDT_OK;
    int ctr[GC_N] = {0};
    ctr[GC_STAMP] = 1;
    // The host arrays are pageable: these copies complete before returning.
    rc |= check_hip(c, hipMemcpyAsync(w + L.xy, xy, sizeof(int2) * n, hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + L.order, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + L.pt_off, c->pt_off.data(), sizeof(long long) * 2, hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + L.tri_off, c->tri_off.data(), sizeof(long long) * 2, hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + L.frame, &fr, sizeof(int4), hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + G.split, split.data(), sizeof(int2) * split.size(), hipMemcpyHostToDevice, s));
    if (qt_thr > 0) {
        rc |= check_hip(c, hipMemcpyAsync(w + G.qn, QT.nodes.data(), sizeof(int4) * QT.nodes.size(),
                                          hipMemcpyHostToDevice, s));
        rc |= check_hip(c, hipMemcpyAsync(w + G.ql, QT.links.data(), sizeof(int4) * QT.links.size(),
                                          hipMemcpyHostToDevice, s));
    }
    rc |= check_hip(c, hipMemcpyAsync(w + G.powner, cell.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemcpyAsync(w + G.ctr, ctr, sizeof(ctr), hipMemcpyHostToDevice, s));
    rc |= check_hip(c, hipMemsetAsync(w + L.status, 0, sizeof(int), s));
    rc |= check_hip(c, hipMemsetAsync(w + L.stats, 0, sizeof(BlockStats), s));
    rc |= check_hip(c, hipMemsetAsync(w + L.sticky, 0, sizeof(int) * 4, s));
    rc |= check_hip(c, hipMemsetAsync(w + G.claim, 0, sizeof(unsigned long long) * (2 * n - 2), s));
    rc |= check_hip(c, hipMemsetAsync(w + G.gstats, 0, sizeof(unsigned long long) * KDT_GSTAT_N, s));
    rc |= check_hip(c, hipMemsetAsync(w + G.part, 0, sizeof(unsigned long long) * 4 * G_PART_MAX, s));
    rc |= check_hip(c, hipMemsetAsync(w + G.hkey, 0, sizeof(unsigned long long) * G.hsize, s));
    rc |= check_hip(c, hipMemsetAsync(w + G.hcnt, 0, sizeof(int) * G.hsize, s));
    if (rc == KDT_OK) rc = check_hip(c, hipStreamSynchronize(s));
    if (rc != KDT_OK) { delete c; return KDT_E_DEVICE; }
    rc = gbuild(c);
    if (rc != KDT_OK) { delete c; return rc; }
    *out = c;
    return KDT_OK;
}

extern "C" {

int kdt_init_global(kdt_ctx** out, const int32_t* xy, int64_t n, int32_t depth, const int32_t* domain,
                    int32_t max_moves, void* dev_ws, size_t ws_bytes, void* stream) {
    return init_global(out, xy, n, depth, 0, domain, max_moves, dev_ws, ws_bytes, stream);
}

int kdt_workspace_size_global_qt(const int32_t* xy, int64_t n, const int32_t* domain, int64_t threshold,
                                 int32_t max_moves, size_t* dev_bytes) {
    if (!dev_bytes || !xy || !domain || n < 1 || threshold < 1 || max_moves < 1 || max_moves > (1 << 22))
        return KDT_E_ARG;
    if (n > (1 << 22)) return KDT_E_CAPACITY;
    if (domain[0] < 0 || domain[1] < 0 || domain[2] > KDT_COORD_LIMIT || domain[3] > KDT_COORD_LIMIT ||
        domain[0] >= domain[2] || domain[1] >= domain[3])
        return KDT_E_RANGE;
    for (int64_t i = 0; i < n; ++i)
        if (xy[2 * i] < domain[0] || xy[2 * i] >= domain[2] || xy[2 * i + 1] < domain[1] || xy[2 * i + 1] >= domain[3])
            return KDT_E_RANGE;
    QtHost QT;
    qt_build_host(xy, n, domain, threshold, QT);
    const Layout L = make_layout(n, 1, 0);
    *dev_bytes = make_glayout(L.total, n, 0, max_moves, qt_capacity(QT, n, threshold)).total;
    return KDT_OK;
}

int kdt_init_global_qt(kdt_ctx** out, const int32_t* xy, int64_t n, const int32_t* domain, int64_t threshold,
                       int32_t max_moves, void* dev_ws, size_t ws_bytes, void* stream) {
    if (threshold < 1) {
        if (out) *out = nullptr;
        return KDT_E_ARG;
    }
    return init_global(out, xy, n, 0, threshold, domain, max_moves, dev_ws, ws_bytes, stream);
}

int kdt_quadtree(kdt_ctx* c, int32_t* host_nodes, int32_t cap, int32_t* n_nodes) {
    if (!c || !n_nodes || cap < 0 || (cap > 0 && !host_nodes)) return KDT_E_ARG;
    if (!c->global || !c->g.qt) return KDT_E_STATE;
    const int rc = kdt_sync(c);
    if (rc != KDT_OK) return rc;
    const int nn = c->qt_count;
    *n_nodes = nn;
    if (nn > cap) return KDT_E_CAPACITY;
    std::vector<int4> nd(nn), lk(nn);
    if (check_hip(c, hipMemcpy(nd.data(), c->g.qn, sizeof(int4) * nn, hipMemcpyDeviceToHost)) ||
        check_hip(c, hipMemcpy(lk.data(), c->g.ql, sizeof(int4) * nn, hipMemcpyDeviceToHost)))
        return KDT_E_DEVICE;
    for (int k = 0; k < nn; ++k) {
        int32_t* r = host_nodes + 8 * (int64_t)k;
        r[0] = nd[k].x; r[1] = nd[k].y; r[2] = 1 << nd[k].z; r[3] = nd[k].w;
        const bool leaf = nd[k].w < 0;
        r[4] = leaf ? lk[k].x : -1; r[5] = leaf ? lk[k].y : -1; r[6] = leaf ? lk[k].z : -1; r[7] = leaf ? lk[k].w : -1;
    }
    return KDT_OK;
}

int kdt_repartition(kdt_ctx* c) {
    if (!c) return KDT_E_ARG;
    if (!c->global || !c->g.qt || c->sticky != KDT_OK) return KDT_E_STATE;
    const int rc = qt_repartition(c);
    if (rc != KDT_OK) c->sticky = rc;
    return rc;
}

int kdt_set_repartition(kdt_ctx* c, int32_t every_step) {
    if (!c || every_step < 0 || every_step > 1) return KDT_E_ARG;
    if (!c->global || !c->g.qt) return KDT_E_STATE;
    c->qt_every_step = every_step != 0;
    c->epoch++;
    return KDT_OK;
}

}  // extern "C"

namespace {

int check_global_steps(kdt_ctx* c, const kdt_move_t* moves, const int64_t* step_off, int32_t n_steps) {
    if (!c || n_steps < 0 || (n_steps > 0 && (!moves || !step_off))) return KDT_E_ARG;
    if (!c->global || c->sticky != KDT_OK) return KDT_E_STATE;
    for (int32_t t = 0; t < n_steps; ++t) {
        const int64_t M = step_off[t + 1] - step_off[t];
        if (step_off[t] < 0 || M < 0) return KDT_E_ARG;
        if (M > c->max_moves) return KDT_E_CAPACITY;
    }
    return KDT_OK;
}

// Enqueue n_steps global steps on the context's stream (timing events and
// the per-step re-partition, which synchronises, only when not captured).
int enqueue_global(kdt_ctx* c, const kdt_move_t* moves, const int64_t* step_off, int32_t n_steps,
                   int8_t* applied, bool captured) {
    hipStream_t st = c->stream;
    for (int32_t t = 0; t < n_steps; ++t) {
        const int M = (int)(step_off[t + 1] - step_off[t]);
        if (M == 0) continue;
        const kdt_move_t* mv = moves + step_off[t];
        int8_t* ap = applied ? applied + step_off[t] : nullptr;
        hipEvent_t e0 = captured ? nullptr : timing_begin(c);
        k_g_prep<<<(M + 255) / 256, 256, 0, st>>>(c->dev, c->g, mv, M, ap);
        k_g_classify<<<(M + 255) / 256, 256, 0, st>>>(c->dev, c->g, mv, M);
        const int parts = std::min(M, std::min(8 * c->cus, G_PART_MAX));
        for (int r = 0; r < G_ROUNDS; ++r) {
            k_g_plan<<<std::min(M, c->wpc * c->cus), WAVE, 0, st>>>(c->dev, c->g, mv, M, r);
            k_g_commit<<<parts, WAVE, 0, st>>>(c->dev, c->g, mv, M, r, r == G_ROUNDS - 1 ? 1 : 0, ap);
        }
        k_g_serial<<<1, WAVE, 0, st>>>(c->dev, c->g, mv, M, ap, parts);
        if (c->qt_every_step && !captured) {  // Quad-treeDvision after the step (Fig. 4)
            const int rc = qt_repartition(c);
            if (rc != KDT_OK) {
                c->sticky = rc;
                return rc;
            }
        }
        if (!captured) timing_end(c, e0);
        if (check_hip(c, hipGetLastError()) != KDT_OK) return KDT_E_DEVICE;
        c->step_count++;
    }
    return KDT_OK;
}

}  // namespace

extern "C" {

int kdt_run_global(kdt_ctx* c, const kdt_move_t* moves, const int64_t* step_off, int32_t n_steps,
                   int8_t* applied) {
    const int rc = check_global_steps(c, moves, step_off, n_steps);
    return rc != KDT_OK ? rc : enqueue_global(c, moves, step_off, n_steps, applied, false);
}

int kdt_graph_build_global(kdt_ctx* c, const kdt_move_t* moves, const int64_t* step_off, int32_t n_steps,
                           int8_t* applied, kdt_graph** out) {
    if (!out || n_steps < 1) return KDT_E_ARG;
    *out = nullptr;
    int rc = check_global_steps(c, moves, step_off, n_steps);
    if (rc != KDT_OK) return rc;
    if (c->stream == nullptr || c->qt_every_step) return KDT_E_STATE;  // the re-partition synchronises
    kdt_graph* g = new (std::nothrow) kdt_graph();
    if (!g) return KDT_E_CAPACITY;
    g->ctx = c;
    g->epoch = c->epoch;
    if (check_hip(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal))) {
        delete g;
        return KDT_E_DEVICE;
    }
    rc = enqueue_global(c, moves, step_off, n_steps, applied, true);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (rc != KDT_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        c->sticky = KDT_E_DEVICE;
        return KDT_E_DEVICE;
    }
    g->graph = graph;
    if (check_hip(c, hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0))) {
        (void)hipGraphDestroy(graph);
        delete g;
        return KDT_E_DEVICE;
    }
    *out = g;
    return KDT_OK;
}

int kdt_rebuild_global(kdt_ctx* c) {
    if (!c) return KDT_E_ARG;
    if (!c->global || c->sticky != KDT_OK) return KDT_E_STATE;
    const int rc = gbuild(c);
    if (rc != KDT_OK) c->sticky = rc;
    return rc;
}

int kdt_owner(kdt_ctx* c, int32_t* host_owner) {
    if (!c || !host_owner) return KDT_E_ARG;
    if (!c->global) return KDT_E_STATE;
    int rc = kdt_sync(c);
    if (rc != KDT_OK) return rc;
    if (check_hip(c, hipMemcpy(host_owner, c->g.powner, sizeof(int32_t) * c->n, hipMemcpyDeviceToHost)))
        return KDT_E_DEVICE;
    return KDT_OK;
}

int kdt_global_stats(kdt_ctx* c, uint64_t* host_counters) {
    if (!c || !host_counters) return KDT_E_ARG;
    if (!c->global) return KDT_E_STATE;
    int rc = kdt_sync(c);
    if (rc != KDT_OK) return rc;
    if (check_hip(c, hipMemcpy(host_counters, c->g.gstats, sizeof(uint64_t) * KDT_GSTAT_N, hipMemcpyDeviceToHost)))
        return KDT_E_DEVICE;
    host_counters[KDT_GSTAT_BUILD_ROUNDS] = (uint64_t)c->build_rounds;
    return KDT_OK;
}

void kdt_destroy(kdt_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release_events(c);
    for (hipStream_t st : {c->side, c->side2})
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    for (hipEvent_t e : {c->fork_ev, c->join_ev, c->join2_ev})
        if (e) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
