// Parallel from-scratch construction of DT*: many points are inserted at
// once, one per thread, by Bowyer-Watson with conflict resolution.
//
// A round has three phases separated by barriers:
//   plan     every thread walks to its point, grows the point's cavity by a
//            breadth-first search over a consistent snapshot (nobody
//            writes), and claims each cavity triangle and each triangle
//            behind the cavity boundary (whose back-pointer it will patch);
//   commit   a thread that no contender of smaller priority conflicts with
//            takes two fresh slots and writes its fan; the others write
//            nothing;
//   release  claims are cleared (or outdated by the next round's stamps).
// Two attempts conflict when a cavity triangle of one is a cavity triangle
// or a boundary neighbour of the other.  Two attempts that only share a
// boundary neighbour patch different edges of it (their cavities, on the
// other side of those edges, are disjoint) and do not conflict.  Winners
// therefore touch disjoint records, and every commit sees exactly the
// triangles it planned on: a triangle the new point's fan creates has its
// circumcircle inside the union of the circumcircles of the cavity triangle
// and the surviving triangle on its edge, so it conflicts with no other
// winner's point.  The contender with the smallest priority always wins,
// so each round makes progress.  Points are taken level by
// level along a Hilbert order (stride 2^L, 2^(L-1), ..., 1): a point's walk
// starts at a triangle of its neighbour one stride back, already inserted at
// a coarser level.  DT* is unique, so the order of insertions never changes
// the result.
//
// Two users: the block builder below (one workgroup per block, its records
// and claims in LDS when they fit) and the grid-wide builder of the global
// mode (claims stamped with a round number, attempts in global memory).
#pragma once

#include "kdt_device.hpp"

namespace kdt {

constexpr int TCM = 24;                // cavity triangles one thread's attempt can hold (grid-wide build)
constexpr int ATT_INTS = 4 * TCM + 6;  // ints one such attempt spans
constexpr int TCM_B = 12;                  // the same in the block builder (larger cavities wait)
constexpr int ATT_B_INTS = 4 * TCM_B + 6;
constexpr int FREE_OWNER = 0x7fffffff;
constexpr int PB_ROUNDS = 64;  // rounds of one chunk before its points are deferred
constexpr int PB_DEFER = 256;  // deferred points a block can hold

// Claims live in global memory and are taken with atomics, which are
// performed in L2; every access to them is an agent-scope atomic so that no
// thread reads a claim from a stale line of its compute unit's L1.
__device__ __forceinline__ int own_get(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void own_set(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void own_min(int* p, int v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One thread's insertion attempt: the cavity's slots and the boundary edges
// (a, b), each with the edge reference of the surviving triangle behind it.
// Element k of an array sits at base[k * stride]: the threads of a
// workgroup interleave (stride = thread count, conflict-free in LDS), a lone
// thread uses stride 1 and a larger capacity.
struct AttView {
    int* base;
    int stride;
    int cap;  // cavity capacity; the boundary holds cap + 2 edges
    __device__ int& cav(int k) const { return base[k * stride]; }
    __device__ int& ba(int k) const { return base[(cap + k) * stride]; }
    __device__ int& bb(int k) const { return base[(2 * cap + 2 + k) * stride]; }
    __device__ int& bout(int k) const { return base[(3 * cap + 4 + k) * stride]; }
};

// Plan point v at q: walk from `hint`, then grow the cavity.  Returns 0
// (planned: *nc cavity triangles, *nb = *nc + 2 boundary edges), 1 (cavity
// larger than the attempt holds) or an error code.  Reads only.
__device__ int tplan(const BlockView& B, int v, int2 q, int hint, const AttView& A, int* nc_out,
                     int* nb_out) {
    int hit, hops = 0;
    const int seed = walk<false, WaveLDS>(B, nullptr, hint, q, &hit, &hops);
    if (seed < 0) return ST_INTERNAL;
    if (hit >= 0) return ST_INTERNAL;  // duplicate points are rejected before building
    int nc = 1, nb = 0;
    A.cav(0) = seed;
    for (int head = 0; head < nc; ++head) {
        const Tri r = B.tri[A.cav(head)];
        if (bad_tri(B, r.v)) return ST_INTERNAL;
        Tri nr[3];
        int ns[3];
        bool in[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            ns[e] = vget(r.n, e) >> 2;
            if (bad_slot(B, ns[e])) return ST_INTERNAL;
            in[e] = false;
            for (int m = 0; m < nc; ++m) in[e] |= A.cav(m) == ns[e];
            if (!in[e]) nr[e] = B.tri[ns[e]];  // the three loads go out together
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (in[e]) continue;
            bool dup = false;  // accepted earlier in this loop
            for (int m = 0; m < nc; ++m) dup |= A.cav(m) == ns[e];
            if (dup) continue;
            if (bad_tri(B, nr[e].v)) return ST_INTERNAL;
            if (conflicts(nr[e], q, v)) {
                if (nc == A.cap) return 1;
                A.cav(nc++) = ns[e];
            } else {
                if (nb == A.cap + 2) return 1;
                A.ba(nb) = vget(r.v, (e + 1) % 3);
                A.bb(nb) = vget(r.v, (e + 2) % 3);
                A.bout(nb) = vget(r.n, e);
                ++nb;
            }
        }
    }
    if (nb != nc + 2) return ST_INTERNAL;
    *nc_out = nc;
    *nb_out = nb;
    return 0;
}

// Write the fan of a won attempt into its cavity slots and f0, f1.
__device__ int tcommit(const BlockView& B, const AttView& A, int nc, int nb, int v, int2 q, int f0,
                       int f1) {
    for (int i = 0; i < nb; ++i) {
        const int a = A.ba(i), b = A.bb(i), out = A.bout(i);
        const int slot = i < nc ? A.cav(i) : (i == nc ? f0 : f1);
        const int3 ph = fan_phys(a, b);
        int jn = -1, jm = -1;
        for (int m = 0; m < nb; ++m) {
            jn = A.ba(m) == b ? m : jn;
            jm = A.bb(m) == a ? m : jm;
        }
        if (jn < 0 || jm < 0) return ST_INTERNAL;
        const int sjn = jn < nc ? A.cav(jn) : (jn == nc ? f0 : f1);
        const int sjm = jm < nc ? A.cav(jm) : (jm == nc ? f0 : f1);
        const int3 pjn = fan_phys(A.ba(jn), A.bb(jn));
        const int3 pjm = fan_phys(A.ba(jm), A.bb(jm));
        Tri r;
        r.v = make_int4(0, 0, 0, 0);
        r.n = make_int4(0, 0, 0, 0);
        r.c01 = make_int4(0, 0, 0, 0);
        r.c2 = make_int4(0, 0, 0, 0);
        vset(r.v, ph.x, a);
        vset(r.v, ph.y, b);
        vset(r.v, ph.z, v);
        if (a != GHOST) cset(r, ph.x, B.xy[a]);
        if (b != GHOST) cset(r, ph.y, B.xy[b]);
        cset(r, ph.z, q);
        vset(r.n, ph.z, out);
        vset(r.n, ph.x, sjn * 4 + pjn.y);
        vset(r.n, ph.y, sjm * 4 + pjm.x);
        B.tri[slot] = r;
        reinterpret_cast<int*>(&B.tri[out >> 2].n)[out & 3] = slot * 4 + ph.z;
        if (a != GHOST) B.vtri[a] = slot;
        if (i == 0) B.vtri[v] = slot;
    }
    return ST_OK;
}

// The first triangle of points a, c1 and c (c not on the line a c1), made
// counter-clockwise, with its three ghosts, in slots 0..3.
__device__ void seed_triangle(const BlockView& B, int a, int c1, int c) {
    int2 pa = B.xy[a], pb = B.xy[c1];
    const int2 pc = B.xy[c];
    if (orient(pa, pb, pc) < 0) {
        const int t = a; a = c1; c1 = t;
        const int2 tp = pa; pa = pb; pb = tp;
    }
    Tri t;
    t.v = make_int4(a, c1, c, 0); t.n = make_int4(2 * 4 + 2, 3 * 4 + 2, 1 * 4 + 2, 0);
    t.c01 = make_int4(pa.x, pa.y, pb.x, pb.y); t.c2 = make_int4(pc.x, pc.y, 0, 0);
    B.tri[0] = t;
    t.v = make_int4(c1, a, GHOST, 0); t.n = make_int4(3 * 4 + 1, 2 * 4 + 0, 0 * 4 + 2, 0);
    t.c01 = make_int4(pb.x, pb.y, pa.x, pa.y); t.c2 = make_int4(0, 0, 0, 0);
    B.tri[1] = t;
    t.v = make_int4(c, c1, GHOST, 0); t.n = make_int4(1 * 4 + 1, 3 * 4 + 0, 0 * 4 + 0, 0);
    t.c01 = make_int4(pc.x, pc.y, pb.x, pb.y);
    B.tri[2] = t;
    t.v = make_int4(a, c, GHOST, 0); t.n = make_int4(2 * 4 + 1, 1 * 4 + 0, 0 * 4 + 1, 0);
    t.c01 = make_int4(pa.x, pa.y, pc.x, pc.y);
    B.tri[3] = t;
    B.vtri[a] = 0;
    B.vtri[c1] = 0;
    B.vtri[c] = 0;
}

// Priority of the point at index i of the insertion order (i < 2^22): eight
// hashed bits above the index.  Neighbours along the Hilbert curve compete
// for the same triangles; with the index alone their priorities would rise
// along the curve and a chain of contenders would resolve one per round.
// The hash makes local minima frequent; the index keeps priorities unique.
__device__ __forceinline__ int pb_prio(int i) {
    return (int)((((unsigned)i * 2654435761u) >> 24) << 22) | i;
}

// Where a block build keeps its working state: the records and incident
// triangles it writes (the block's own, or LDS copies written back at the
// end), the two claim arrays (one int per slot each) and the attempts
// (blockDim.x * ATT_B_INTS ints of LDS).
struct PBMem {
    Tri* tri;
    int* vtri;
    int* cown;  // smallest priority holding the triangle in its cavity
    int* bown;  // smallest priority holding it behind its cavity boundary
    int* att;
};

// Build block G's DT* from scratch with all threads of the workgroup.
// ord: the block's points in Hilbert order; lds: four ints of shared memory
// plus PB_DEFER for deferred points.  Every thread must call it.
__device__ int pbuild_block(const BlockView& G, const int* ord, const PBMem& M, int* lds) {
    const int tid = threadIdx.x, NT = blockDim.x;
    BlockView B = G;
    B.tri = M.tri;
    B.vtri = M.vtri;
    int* att = M.att;
    const int n = B.n;
    int& kmin = lds[0];    // index of the first point off the first line
    int& used = lds[1];    // triangle slots in use
    int& status = lds[2];  // first error
    int& ndef = lds[3];    // deferred points
    int* deferred = lds + 4;
    for (int i = tid; i < B.ntri; i += NT) {
        own_set(&M.cown[i], FREE_OWNER);
        own_set(&M.bown[i], FREE_OWNER);
    }
    if (tid == 0) {
        kmin = 0x7fffffff;
        used = 4;
        status = ST_OK;
        ndef = 0;
    }
    __syncthreads();
    const int a0 = ord[0], b0 = ord[1];
    const int2 pa0 = B.xy[a0], pb0 = B.xy[b0];
    for (int i = 2 + tid; i < n; i += NT)
        if (orient(pa0, pb0, B.xy[ord[i]]) != 0) atomicMin(&kmin, i);
    __syncthreads();
    const int kidx = kmin;
    if (kidx >= n) return ST_DEGEN;
    if (tid == 0) seed_triangle(B, a0, b0, ord[kidx]);
    __threadfence_block();
    __syncthreads();
    // levels of the Hilbert order: stride s takes the indices i = s (mod 2s);
    // index 0 and the first triangle's points are already in
    int top = 1;
    while (top * 2 < n) top *= 2;
    const AttView A{att + tid, NT, TCM_B};
    for (int s = top; s >= 1; s >>= 1) {
        const int count = s < n ? (n - 1 - s) / (2 * s) + 1 : 0;
        const int nch = (count + NT - 1) / NT;
        for (int ch = 0; ch < nch; ++ch) {
            const int j = ch + tid * nch;  // chunk ch takes every nch-th point of the level
            const int i = s + 2 * s * j;
            const bool mine = j < count && i != 1 && i != kidx;
            const int v = mine ? ord[i] : 0;
            const int2 q = mine ? B.xy[v] : make_int2(0, 0);
            const int hint_pt = mine ? ord[i - s] : 0;
            const int prio = pb_prio(i);
            bool pending = mine;
            int nc = 0, nb = 0;
            for (int round = 0; round < PB_ROUNDS; ++round) {
                bool planned = false;
                if (pending) {
                    // start at a live triangle: slots at or past `used` are not written yet
                    const int hs = B.vtri[hint_pt];
                    const int hint = hs >= 0 && hs < used ? hs : 0;
                    const int rc = tplan(B, v, q, hint, A, &nc, &nb);
                    if (rc == 0) {
                        planned = true;
                        for (int m = 0; m < nc; ++m) own_min(&M.cown[A.cav(m)], prio);
                        for (int e = 0; e < nb; ++e) own_min(&M.bown[A.bout(e) >> 2], prio);
                    } else if (rc == 1) {  // cavity too large for one thread: later, alone
                        const int d = atomicAdd(&ndef, 1);
                        if (d < PB_DEFER) deferred[d] = i;
                        else atomicMin(&status, ST_CAPACITY);
                        pending = false;
                    } else {
                        atomicMin(&status, rc);
                        pending = false;
                    }
                }
                __syncthreads();
                if (planned) {
                    bool won = true;
                    for (int m = 0; m < nc; ++m) {
                        const int t = A.cav(m);
                        won &= own_get(&M.cown[t]) == prio && own_get(&M.bown[t]) > prio;
                    }
                    for (int e = 0; e < nb; ++e) won &= own_get(&M.cown[A.bout(e) >> 2]) > prio;
                    if (won) {
                        const int f = atomicAdd(&used, 2);
                        const int rc = f + 1 < B.ntri ? tcommit(B, A, nc, nb, v, q, f, f + 1) : ST_INTERNAL;
                        if (rc != ST_OK) atomicMin(&status, rc);
                        pending = false;
                    }
                }
                __threadfence_block();
                __syncthreads();
                if (planned) {
                    for (int m = 0; m < nc; ++m) own_set(&M.cown[A.cav(m)], FREE_OWNER);
                    for (int e = 0; e < nb; ++e) own_set(&M.bown[A.bout(e) >> 2], FREE_OWNER);
                }
                __threadfence_block();
                if (!__syncthreads_or(pending)) break;
            }
            if (pending) {  // still contended after many rounds: defer
                const int d = atomicAdd(&ndef, 1);
                if (d < PB_DEFER) deferred[d] = i;
                else atomicMin(&status, ST_CAPACITY);
            }
            __syncthreads();
        }
    }
    // deferred points, one at a time by thread 0 (no contention), whose
    // attempt spans all the threads' attempt memory
    if (tid == 0) {
        const AttView big{att, 1, (NT * ATT_B_INTS - 6) / 4};
        const int nd = ndef < PB_DEFER ? ndef : PB_DEFER;
        for (int d = 0; d < nd && status == ST_OK; ++d) {
            const int i = deferred[d];
            const int v = ord[i];
            int nc = 0, nb = 0;
            const int rc = tplan(B, v, B.xy[v], 0, big, &nc, &nb);
            if (rc != 0) { status = rc == 1 ? ST_CAPACITY : rc; break; }
            const int f = used;
            used += 2;
            const int rc2 = f + 1 < B.ntri ? tcommit(B, big, nc, nb, v, B.xy[v], f, f + 1) : ST_INTERNAL;
            if (rc2 != ST_OK) status = rc2;
        }
        if (status == ST_OK && used != B.ntri) status = ST_INTERNAL;
    }
    __syncthreads();
    const int rc = status;
    if (rc == ST_OK && M.tri != G.tri) {  // built in LDS: write the block back
        for (int i = tid; i < B.ntri; i += NT) G.tri[i] = M.tri[i];
        for (int i = tid; i < n; i += NT) G.vtri[i] = M.vtri[i];
        __threadfence_block();
        __syncthreads();
    }
    return rc;
}

}  // namespace kdt
