// Device-side Delaunay maintenance for one block, executed by one wavefront.
//
// Method: Hadiniya & Ghodsi, Fig. 4 -- every block deletes its moved point
// and inserts it again at the new place (Sec. IV, "Insertion and Deletion":
// insertion by Bowyer-Watson; deletion by a simple method).  The triangulation
// kept is DT*, the Delaunay triangulation (Sec. I: empty circumcircles,
// unique) with ties on cocircular lattice points broken by lifting every
// point by an infinitesimal that grows with its id.
//
// Layout of one block in HBM:
//   tri[s]   32-byte record {v0, v1, v2, 0 | n0, n1, n2, 0}; v are local
//            point indices, GHOST (-1) for the vertex at infinity (a ghost
//            triangle keeps it in v2); n_e = 4 * slot + e' names the
//            triangle across the edge opposite v_e and that edge's index e'
//            in it.  A block of n points always holds exactly 2n - 2 records
//            (real triangles plus one ghost per hull edge).
//   xy[i]    int2 position of local point i
//   vtri[i]  slot of one triangle incident to point i
// Local point order follows global id order, so local indices serve as the
// perturbation order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kdt {

constexpr int GHOST = -1;
constexpr int WAVE = 64;
constexpr int KMAX = 64;         // largest degree of a deleted vertex
constexpr int TRIPLE_KMAX = 40;  // link-triple retriangulation limit
constexpr int CMAX = 320;        // largest Bowyer-Watson cavity
constexpr int BMAX = CMAX + 2;   // its boundary

// status codes (mirror kdt.h)
constexpr int ST_OK = 0;
constexpr int ST_ARG = -1;
constexpr int ST_CAPACITY = -5;
constexpr int ST_INTERNAL = -8;
constexpr int ST_DEGEN = -4;

struct alignas(32) Tri {
    int4 v;
    int4 n;
};

struct BlockView {
    Tri* tri;
    int2* xy;
    int* vtri;
    int n;
    int ntri;
};

// per-block counters, owned by the block's wavefront (no atomics needed)
struct BlockStats {
    long long applied, blocked, star_sum, cavity_sum, walk_sum, tri_touched, alg_bytes, errors;
};

// per-wavefront scratch in LDS
struct WaveLDS {
    int star_slot[KMAX];
    int link[KMAX];
    int outref[KMAX];
    int edge_tri[KMAX];  // link edge s -> 4 * hole triangle + edge index
    int hole_key[KMAX];  // packed link indices (i, j, l) of hole triangles
    Tri hole_rec[KMAX];
    int cav_slot[CMAX];
    Tri cav_rec[CMAX];
    int bnd_a[BMAX], bnd_b[BMAX], bnd_out[BMAX];
    int cand[WAVE];
    int ncav, nbnd, nhole, pad;
};

// ---------------------------------------------------------------- wave ops

__device__ __forceinline__ int lane_id() { return (int)threadIdx.x; }
__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }
__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}
__device__ __forceinline__ int lanes_below(uint64_t m) { return __popcll(m & lanemask_lt()); }
// LDS and global memory ordering between the lanes of the (single-wave)
// workgroup: a workgroup barrier carries the needed fence.
__device__ __forceinline__ void wsync() { __syncthreads(); }

// Every slot and vertex index read from memory is checked against the
// block's ranges before use, so corrupted state ends in an error code,
// never in an access outside the block.
__device__ __forceinline__ bool bad_slot(const BlockView& B, int s) {
    return (unsigned)s >= (unsigned)B.ntri;
}
__device__ __forceinline__ bool bad_vert(const BlockView& B, int v) {
    return v != -1 && (unsigned)v >= (unsigned)B.n;
}
__device__ __forceinline__ bool bad_tri(const BlockView& B, const int4& v) {
    return (unsigned)v.x >= (unsigned)B.n || (unsigned)v.y >= (unsigned)B.n || bad_vert(B, v.z);
}

__device__ __forceinline__ int vget(const int4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : v.z);
}
__device__ __forceinline__ void vset(int4& v, int i, int val) {
    if (i == 0) v.x = val;
    else if (i == 1) v.y = val;
    else v.z = val;
}

// ---------------------------------------------------------------- predicates
// Every coordinate is in [0, 2^24), so differences fit in 25 bits.

// Twice the signed area of (a, b, c): > 0 counter-clockwise.  Exact.
__device__ __forceinline__ long long orient(int2 a, int2 b, int2 c) {
    return (long long)(b.x - a.x) * (long long)(c.y - a.y) -
           (long long)(b.y - a.y) * (long long)(c.x - a.x);
}

__device__ __noinline__ int incircle_exact(long long al, long long bl, long long cl,
                                           long long m_bc, long long m_ca, long long m_ab) {
    __int128 d = (__int128)al * m_bc + (__int128)bl * m_ca + (__int128)cl * m_ab;
    return (d > 0) - (d < 0);
}

// Sign of the incircle determinant (> 0: d strictly inside the circle of the
// counter-clockwise a, b, c).  The three lifts |p - d|^2 and the three 2x2
// minors are exact integers below 2^49, hence exact doubles; only the three
// products and two sums round, so the computed value is within
// 3u(1 + O(u)) * P of the true one, P the sum of the product magnitudes
// (u = 2^-53).  A result larger than 4u * P in magnitude has the right sign;
// otherwise the determinant is recomputed in 128-bit integers.
__device__ __forceinline__ int incircle(int2 a, int2 b, int2 c, int2 d) {
#pragma clang fp contract(off)
    long long adx = a.x - d.x, ady = a.y - d.y;
    long long bdx = b.x - d.x, bdy = b.y - d.y;
    long long cdx = c.x - d.x, cdy = c.y - d.y;
    long long al = adx * adx + ady * ady;
    long long bl = bdx * bdx + bdy * bdy;
    long long cl = cdx * cdx + cdy * cdy;
    long long m_bc = bdx * cdy - bdy * cdx;
    long long m_ca = cdx * ady - cdy * adx;
    long long m_ab = adx * bdy - ady * bdx;
    double p1 = (double)al * (double)m_bc;
    double p2 = (double)bl * (double)m_ca;
    double p3 = (double)cl * (double)m_ab;
    double det = (p1 + p2) + p3;
    double perm = (fabs(p1) + fabs(p2)) + fabs(p3);
    double bound = perm * 0x1p-51;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return incircle_exact(al, bl, cl, m_bc, m_ca, m_ab);
}

__device__ __forceinline__ int sgn(long long v) { return (v > 0) - (v < 0); }

// Incircle with ties broken by the id lift: when a, b, c, d are exactly
// cocircular, the point with the largest rank is lifted most and decides
// through the cofactor of its height in the lifted 4x4 determinant
// (rows x, y, x^2+y^2, 1 in the order a, b, c, d).
__device__ __forceinline__ int incircle_star(int2 a, int ra, int2 b, int rb, int2 c, int rc,
                                             int2 d, int rd) {
    int s = incircle(a, b, c, d);
    if (s != 0) return s;
    if (ra > rb && ra > rc && ra > rd) return sgn(orient(b, c, d));
    if (rb > rc && rb > rd) return -sgn(orient(a, c, d));
    if (rc > rd) return sgn(orient(a, b, d));
    return -sgn(orient(a, b, c));
}

// Ghost (a, b, inf) covers the open half-plane left of a->b and the open
// segment ab; a new point there destroys it.
__device__ __forceinline__ bool ghost_conflict(int2 a, int2 b, int2 q) {
    long long o = orient(a, b, q);
    if (o != 0) return o > 0;
    long long t1 = (long long)(q.x - a.x) * (b.x - a.x) + (long long)(q.y - a.y) * (b.y - a.y);
    long long t2 = (long long)(q.x - b.x) * (a.x - b.x) + (long long)(q.y - b.y) * (a.y - b.y);
    return t1 > 0 && t2 > 0;
}

// Does inserting point q (rank rq) destroy triangle t?
__device__ __forceinline__ bool conflicts(const BlockView& B, const Tri& t, int2 q, int rq) {
    if (t.v.z == GHOST) return ghost_conflict(B.xy[t.v.x], B.xy[t.v.y], q);
    return incircle_star(B.xy[t.v.x], t.v.x, B.xy[t.v.y], t.v.y, B.xy[t.v.z], t.v.z, q, rq) > 0;
}

// ---------------------------------------------------------------- walk
// Visibility walk toward q (every lane runs it identically).  Ends at a
// triangle that q destroys: a real triangle whose closed area holds q, or a
// ghost whose half-plane holds q.  *hit gets the local index of a vertex
// sitting exactly at q (-1 if none).  Returns -1 if the step limit is hit.
__device__ int walk(const BlockView& B, int start, int2 q, int* hit, int* hops) {
    int cur = start, entry = -1;
    const int limit = 4 * B.ntri + 16;
    *hit = -1;
    for (int h = 0; h < limit; ++h) {
        if (bad_slot(B, cur)) return -1;
        Tri t = B.tri[cur];
        if (bad_tri(B, t.v)) return -1;
        if (t.v.z == GHOST) {
            if (ghost_conflict(B.xy[t.v.x], B.xy[t.v.y], q)) {
                *hops += h + 1;
                return cur;
            }
            int r = t.n.z;
            entry = r & 3;
            cur = r >> 2;
            continue;
        }
        int2 p0 = B.xy[t.v.x], p1 = B.xy[t.v.y], p2 = B.xy[t.v.z];
        int next = -1;
        if (entry != 0 && orient(p1, p2, q) < 0) next = 0;
        else if (entry != 1 && orient(p2, p0, q) < 0) next = 1;
        else if (entry != 2 && orient(p0, p1, q) < 0) next = 2;
        if (next < 0) {
            if (p0.x == q.x && p0.y == q.y) *hit = t.v.x;
            else if (p1.x == q.x && p1.y == q.y) *hit = t.v.y;
            else if (p2.x == q.x && p2.y == q.y) *hit = t.v.z;
            *hops += h + 1;
            return cur;
        }
        int r = vget(t.n, next);
        entry = r & 3;
        cur = r >> 2;
    }
    return -1;
}

// ---------------------------------------------------------------- insert
// Logical corners of the fan triangle on boundary edge (a, b): (a, b, q).
// A ghost keeps the vertex at infinity in slot 2, so the stored order is
// (a, b, q), (b, q, inf) when a is infinite, (q, a, inf) when b is.
// Returns the stored index of a, b and q.
__device__ __forceinline__ int3 fan_phys(int a, int b) {
    if (a == GHOST) return make_int3(2, 0, 1);
    if (b == GHOST) return make_int3(1, 2, 0);
    return make_int3(0, 1, 2);
}

// Insert point qv at q into the block's DT* (Bowyer-Watson, Sec. IV).
// `seed` is a triangle q destroys; f0, f1 are two free slots that take the
// two triangles the insertion adds.  The cavity grows level by level: the
// lanes test the frontier's neighbours, ballots and prefix counts compact
// the survivors.  Returns ST_OK or an error code (the block is then
// no longer valid and must be rebuilt).
__device__ int insert_vertex(BlockView& B, WaveLDS& S, int qv, int2 q, int seed, int f0, int f1,
                             BlockStats* st) {
    const int lane = lane_id();
    if (bad_slot(B, seed) || bad_slot(B, f0) || bad_slot(B, f1)) return ST_INTERNAL;
    if (lane == 0) {
        S.cav_slot[0] = seed;
        S.cav_rec[0] = B.tri[seed];
        S.ncav = 1;
        S.nbnd = 0;
    }
    wsync();
    if (bad_tri(B, S.cav_rec[0].v)) return ST_INTERNAL;
    int fs = 0, fe = 1;
    int err = ST_OK;
    int loaded = 1;
    while (fs < fe) {
        const int ncand = 3 * (fe - fs);
        for (int base = 0; base < ncand; base += WAVE) {
            const int j = base + lane;
            const bool act = j < ncand;
            const int ci = fs + j / 3, e = j % 3;
            int nref = 0, ns = -1;
            bool incav = false, conf = false;
            Tri nt;
            Tri ct;
            if (act) {
                ct = S.cav_rec[ci];
                nref = vget(ct.n, e);
                ns = nref >> 2;
                const int nc = S.ncav;
                for (int m = 0; m < nc; ++m)
                    if (S.cav_slot[m] == ns) { incav = true; break; }
                if (!incav) {
                    if (bad_slot(B, ns)) {
                        err = ST_INTERNAL;
                    } else {
                        nt = B.tri[ns];
                        if (bad_tri(B, nt.v)) err = ST_INTERNAL;
                        else conf = conflicts(B, nt, q, qv);
                    }
                }
            }
            if (ballot(err != ST_OK)) { err = ST_INTERNAL; break; }
            const bool c1 = act && !incav && conf;
            const uint64_t mc = ballot(c1);
            loaded += __popcll(ballot(act && !incav));
            if (c1) S.cand[lane] = ns;
            wsync();
            bool dup = false;
            if (c1) {
                uint64_t lower = mc & lanemask_lt();
                while (lower) {
                    int i = __ffsll((long long)lower) - 1;
                    if (S.cand[i] == ns) { dup = true; break; }
                    lower &= lower - 1;
                }
            }
            const bool acc = c1 && !dup;
            const bool bnd = act && !incav && !conf;
            const uint64_t macc = ballot(acc), mb = ballot(bnd);
            const int nc0 = S.ncav, nb0 = S.nbnd;
            const int nacc = __popcll(macc), nbn = __popcll(mb);
            if (nc0 + nacc > CMAX || nb0 + nbn > BMAX) { err = ST_CAPACITY; break; }
            if (acc) {
                int pos = nc0 + lanes_below(macc);
                S.cav_slot[pos] = ns;
                S.cav_rec[pos] = nt;
            }
            if (bnd) {
                int pos = nb0 + lanes_below(mb);
                S.bnd_a[pos] = vget(ct.v, (e + 1) % 3);
                S.bnd_b[pos] = vget(ct.v, (e + 2) % 3);
                S.bnd_out[pos] = nref;
            }
            wsync();
            if (lane == 0) {
                S.ncav = nc0 + nacc;
                S.nbnd = nb0 + nbn;
            }
            wsync();
        }
        if (err) break;
        fs = fe;
        fe = S.ncav;
    }
    const int c = S.ncav, nb = S.nbnd;
    if (!err && nb != c + 2) err = ST_INTERNAL;
    if (err) return err;

    // fan: one triangle (a, b, q) per boundary edge, written into the c
    // cavity slots and the two free ones
    for (int i = lane; i < nb; i += WAVE) {
        const int a = S.bnd_a[i], b = S.bnd_b[i], out = S.bnd_out[i];
        const int slot = i < c ? S.cav_slot[i] : (i == c ? f0 : f1);
        const int3 ph = fan_phys(a, b);
        int jn = -1, jm = -1;  // fan triangles starting at b / ending at a
        for (int m = 0; m < nb; ++m) {
            if (S.bnd_a[m] == b) jn = m;
            if (S.bnd_b[m] == a) jm = m;
        }
        if (jn < 0 || jm < 0) { err = ST_INTERNAL; continue; }
        const int sjn = jn < c ? S.cav_slot[jn] : (jn == c ? f0 : f1);
        const int sjm = jm < c ? S.cav_slot[jm] : (jm == c ? f0 : f1);
        const int3 pjn = fan_phys(S.bnd_a[jn], S.bnd_b[jn]);
        const int3 pjm = fan_phys(S.bnd_a[jm], S.bnd_b[jm]);
        Tri r;
        r.v = make_int4(0, 0, 0, 0);
        r.n = make_int4(0, 0, 0, 0);
        vset(r.v, ph.x, a);
        vset(r.v, ph.y, b);
        vset(r.v, ph.z, qv);
        vset(r.n, ph.z, out);                      // across (a, b)
        vset(r.n, ph.x, sjn * 4 + pjn.y);          // across (b, q): jn's edge (q, b)
        vset(r.n, ph.y, sjm * 4 + pjm.x);          // across (q, a): jm's edge (a, q)
        B.tri[slot] = r;
        reinterpret_cast<int*>(&B.tri[out >> 2].n)[out & 3] = slot * 4 + ph.z;
        if (a != GHOST) B.vtri[a] = slot;
        if (i == 0) B.vtri[qv] = slot;
    }
    const uint64_t bad = ballot(err != ST_OK);
    wsync();
    if (bad) return ST_INTERNAL;
    if (lane == 0 && st) {
        st->cavity_sum += c;
        // records read: cavity + tested neighbours; written: fan; patches c+2;
        // coordinates of tested vertices; vtri writes c+3
        st->tri_touched += loaded + nb;
        st->alg_bytes += 32LL * loaded + 8LL * loaded + 32LL * nb + 4LL * nb + 4LL * (nb + 1);
    }
    return ST_OK;
}

// ---------------------------------------------------------------- delete
__device__ __forceinline__ int pack3(int i, int j, int l) { return (i << 16) | (j << 8) | l; }

// Remove point p from the block's DT* (the Delete step of Fig. 4).
// The hole left by p's star is retriangulated from its link q_0..q_{k-1}
// (counter-clockwise, with the vertex at infinity last when p is on the
// hull): the new triangles are the triples q_i, q_j, q_l (i < j < l) that
// are counter-clockwise and whose (perturbed) circle holds no other link
// vertex -- for a ghost triple (q_i, q_j, inf), no link vertex beyond the
// line q_i q_j.  These are the Delaunay triangles of the link vertices that
// lie in the hole, i.e. exactly DT*(S - p) there.  The k - 2 new triangles
// take the first k - 2 star slots; the last two star slots become free.
// Returns k (> 0) or an error code (< 0) with the block unchanged.
__device__ int remove_vertex(BlockView& B, WaveLDS& S, int p, BlockStats* st) {
    const int lane = lane_id();
    // 1. star of p, counter-clockwise (every lane walks it identically)
    int t = B.vtri[p];
    if (bad_slot(B, t)) return ST_INTERNAL;
    Tri r = B.tri[t];
    if (bad_tri(B, r.v)) return ST_INTERNAL;
    int pi = r.v.x == p ? 0 : (r.v.y == p ? 1 : (r.v.z == p ? 2 : -1));
    if (pi < 0) return ST_INTERNAL;
    const int start = t;
    int k = 0, ghost_at = -1;
    while (true) {
        if (k >= KMAX) return ST_CAPACITY;
        const int a = vget(r.v, (pi + 1) % 3);
        if (lane == k) {
            S.star_slot[k] = t;
            S.link[k] = a;
            S.outref[k] = vget(r.n, pi);
        }
        if (a == GHOST) ghost_at = k;
        const int nr = vget(r.n, (pi + 1) % 3);
        if (bad_slot(B, vget(r.n, pi) >> 2)) return ST_INTERNAL;
        t = nr >> 2;
        pi = ((nr & 3) + 1) % 3;
        ++k;
        if (t == start) break;
        if (bad_slot(B, t) || pi > 2) return ST_INTERNAL;
        r = B.tri[t];
        if (bad_tri(B, r.v) || vget(r.v, pi) != p) return ST_INTERNAL;
    }
    wsync();
    if (k < 3) return ST_INTERNAL;
    if (k > TRIPLE_KMAX) return ST_CAPACITY;
    // 2. rotate so that the vertex at infinity, if any, comes last
    if (ghost_at >= 0 && ghost_at != k - 1) {
        int s0 = 0, s1 = 0, s2 = 0;
        const int src = (lane + ghost_at + 1) % k;
        if (lane < k) { s0 = S.star_slot[src]; s1 = S.link[src]; s2 = S.outref[src]; }
        wsync();
        if (lane < k) { S.star_slot[lane] = s0; S.link[lane] = s1; S.outref[lane] = s2; }
        wsync();
    }
    const int lv = lane < k ? S.link[lane] : GHOST;
    // 3. valid triples; lanes stride over pairs (i, j), each scans l > j
    if (lane == 0) S.nhole = 0;
    if (lane < k) S.edge_tri[lane] = -1;
    wsync();
    const int npairs = k * (k - 1) / 2;
    for (int pidx = lane; pidx < npairs; pidx += WAVE) {
        // decode pidx -> (i, j), i < j, in the order (0,1), (0,2), (1,2), (0,3), ...
        int j = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)pidx)) * 0.5f);
        while (j * (j - 1) / 2 > pidx) --j;
        while ((j + 1) * j / 2 <= pidx) ++j;
        const int i = pidx - j * (j - 1) / 2;
        const int vi = S.link[i], vj = S.link[j];
        if (vi == GHOST || vj == GHOST) continue;
        const int2 pi2 = B.xy[vi], pj2 = B.xy[vj];
        for (int l = j + 1; l < k; ++l) {
            const int vl = S.link[l];
            bool ok = true;
            if (vl == GHOST) {
                for (int m = 0; m < k - 1 && ok; ++m) {
                    if (m == i || m == j) continue;
                    if (ghost_conflict(pi2, pj2, B.xy[S.link[m]])) ok = false;
                }
            } else {
                const int2 pl2 = B.xy[vl];
                if (orient(pi2, pj2, pl2) <= 0) continue;
                for (int m = 0; m < k && ok; ++m) {
                    if (m == i || m == j || m == l) continue;
                    const int vm = S.link[m];
                    if (vm == GHOST) continue;
                    if (incircle_star(pi2, vi, pj2, vj, pl2, vl, B.xy[vm], vm) >= 0) ok = false;
                }
            }
            if (ok) {
                int pos = atomicAdd(&S.nhole, 1);
                if (pos < KMAX) S.hole_key[pos] = pack3(i, j, l);
            }
        }
    }
    wsync();
    const int nh = S.nhole;
    if (nh != k - 2) return ST_INTERNAL;
    // deterministic order: sort hole keys (rank sort, one lane per key)
    int key = lane < nh ? S.hole_key[lane] : 0x7fffffff;
    int rank = 0;
    for (int m = 0; m < nh; ++m) {
        int km = S.hole_key[m];
        rank += km < key;
    }
    wsync();
    if (lane < nh) S.hole_key[rank] = key;
    wsync();
    // 4. adjacency of the hole triangles
    int herr = 0;
    if (lane < nh) {
        const int hk = S.hole_key[lane];
        const int c0 = hk >> 16, c1 = (hk >> 8) & 255, c2 = hk & 255;
        const int cs[3] = {c0, c1, c2};
        Tri h;
        h.v = make_int4(S.link[c0], S.link[c1], S.link[c2], 0);
        h.n = make_int4(0, 0, 0, 0);
        for (int e = 0; e < 3; ++e) {
            const int u = cs[(e + 1) % 3], w = cs[(e + 2) % 3];
            int nref;
            if (w == (u + 1) % k) {  // link edge u: the triangle outside it
                nref = S.outref[u];
                S.edge_tri[u] = lane * 4 + e;
            } else {  // diagonal: the hole triangle with edge (w, u)
                nref = -1;
                for (int m = 0; m < nh && nref < 0; ++m) {
                    if (m == lane) continue;
                    const int mk = S.hole_key[m];
                    const int d[3] = {mk >> 16, (mk >> 8) & 255, mk & 255};
                    for (int f = 0; f < 3; ++f)
                        if (d[(f + 1) % 3] == w && d[(f + 2) % 3] == u) nref = S.star_slot[m] * 4 + f;
                }
                if (nref < 0) herr = 1;
            }
            vset(h.n, e, nref);
        }
        S.hole_rec[lane] = h;
    }
    if (ballot(herr)) return ST_INTERNAL;
    wsync();
    if (ballot(lane < k && S.edge_tri[lane] < 0)) return ST_INTERNAL;
    // 5. write the hole triangles, patch the outside neighbours, vtri
    if (lane < nh) B.tri[S.star_slot[lane]] = S.hole_rec[lane];
    if (lane < k) {
        const int et = S.edge_tri[lane];
        const int hs = S.star_slot[et >> 2];
        const int o = S.outref[lane];
        reinterpret_cast<int*>(&B.tri[o >> 2].n)[o & 3] = hs * 4 + (et & 3);
        if (lv != GHOST) B.vtri[lv] = hs;
    }
    wsync();
    if (lane == 0 && st) {
        st->star_sum += k;
        st->tri_touched += k + nh;
        // star records + link coordinates read; hole records written;
        // k back-pointer patches; k vtri writes
        st->alg_bytes += 32LL * k + 8LL * k + 32LL * nh + 4LL * k + 4LL * k;
    }
    return k;
}

}  // namespace kdt
