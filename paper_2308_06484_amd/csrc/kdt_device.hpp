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
//   tri[s]   64-byte record (one aligned half cache line):
//              v  = {v0, v1, v2, 0}   local point indices; GHOST (-1) is the
//                                     vertex at infinity, kept in v2
//              n  = {n0, n1, n2, 0}   n_e = 4 * slot + e': the triangle across
//                                     the edge opposite v_e, and that edge's
//                                     index e' in it
//              c01 = {x0, y0, x1, y1}, c2 = {x2, y2, 0, 0}: vertex positions
//            A point changes position only by being deleted and inserted
//            again, so the copies of its position in the records of its
//            triangles are always current.  With them a walk step or a
//            conflict test needs one record load and no other.
//            A block of n points always holds exactly 2n - 2 records (real
//            triangles plus one ghost per hull edge).
//   xy[i]    int2 position of local point i
//   vtri[i]  slot of one triangle incident to point i
// Local point order follows global id order, so local indices serve as the
// perturbation order.
//
// Write-back table.  A move reads every record it needs into a small hash
// table in LDS (keyed by slot) and makes every change there; the changed
// records, the incident-triangle updates and the new position go to memory
// in one burst at the end of the move.  On this hardware the vector-memory
// counter covers stores as well as loads, so a load issued after a store
// waits for that store; keeping the stores to the end keeps every load of
// the move free of that wait.  A move that fails leaves memory unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kdt {

constexpr int GHOST = -1;
constexpr int WAVE = 64;
constexpr int KMAX = 64;         // largest degree of a deleted vertex
constexpr int TRIPLE_KMAX = 40;  // link-triple retriangulation limit
constexpr int HT = 256;          // write-back table entries (power of two)
static_assert(HT <= 256, "table entries are listed as bytes");
constexpr int HT_LIMIT = 200;    // entries a move may use (keeps probe chains short)
constexpr int CMAX = 160;        // largest Bowyer-Watson cavity
constexpr int BMAX = CMAX + 2;   // cavity boundary
constexpr int VTMAX = KMAX + BMAX + 1;  // pending incident-triangle updates
constexpr int DRYMAX = 256;     // moves of one block in one step on the rebuild branch
constexpr int EMK = 16;          // links up to this size use the closed-form triple decode and edge matrix
constexpr int WPMAX = 64;        // walk hops a planned move can record
constexpr int SPLIT_K = 10;      // links from this size test candidates in two phases
constexpr int SURV_MAX = 160;    // candidates the second phase holds

constexpr int F_DIRTY = 1;  // table entry changed: write back
constexpr int F_CAV = 2;    // table entry is in the current cavity

// status codes (mirror kdt.h)
constexpr int ST_OK = 0;
constexpr int ST_ARG = -1;
constexpr int ST_DEGEN = -4;
constexpr int ST_CAPACITY = -5;
constexpr int ST_INTERNAL = -8;

struct alignas(64) Tri {
    int4 v;
    int4 n;
    int4 c01;
    int4 c2;
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
    // wall-clock ticks spent by the block's wavefront in each phase of a move
    long long t_star, t_locate, t_hole, t_insert;
    // applied moves by wavefront time, bucket b: [2^b, 2^(b+1)) wall-clock ticks
    long long hist[16];
    long long fast;     // moves done by the star-only path
    long long rebuilt;  // block steps done by the rebuild branch
    long long flipped;  // moves done by move-and-flip
    long long flips;    // edge flips of those moves
};

// per-wavefront scratch in LDS; H write-back table entries (a power of two,
// at most 256)
template <int H>
struct WaveLDST {
    static constexpr int TN = H;                 // table entries
    static constexpr int TLIMIT = H * 25 / 32;   // entries a move may use (keeps probe chains short)
    static_assert(H <= 256 && (H & (H - 1)) == 0, "table entries are listed as bytes, hashed by bits");
    // star of the deleted point, counter-clockwise
    int star_slot[KMAX];
    int link[KMAX];      // link vertex q_s (star triangle s = (p, q_s, q_s+1))
    int2 lxy[KMAX];      // its position
    int outref[KMAX];    // triangle outside link edge (q_s, q_s+1)
    int out_ent[KMAX];   // its table entry
    int edge_tri[KMAX];  // link edge s -> 4 * hole triangle + edge index
    int hole_key[KMAX];  // packed link indices (i, j, l) of hole triangles
    int hole_ent[KMAX];  // table entry of hole triangle h
    // write-back table
    int tkey[H];  // slot, or -1
    int tflag[H];
    Tri trec[H];
    uint8_t tused[H];  // entries in use, in claim order (H <= 256)
    // the directed edges (u, w) of the hole triangles: 4 * triangle + edge
    int emat[EMK * EMK];
    // Bowyer-Watson cavity: table entries, boundary edges (a, b) with the
    // surviving triangle behind them and the positions of a and b
    int cav_ent[CMAX];
    int bnd_a[BMAX], bnd_b[BMAX], bnd_out[BMAX];
    int2 bnd_pa[BMAX], bnd_pb[BMAX];
    // incident-triangle updates: those of the deletion, then those of the
    // insertion (a point in both lists gets the later value)
    int vt_v[VTMAX], vt_s[VTMAX];
    int nvt_del;
    int bnd_slot[BMAX];  // slot of the fan triangle on boundary edge i
    int bnd_ph[BMAX];    // its stored index of a (bits 0-1), b (2-3), q (4-5)
    int nhole, pad[3];
    int wpath[WPMAX];  // slots a planned move's walks read (global mode)
    BlockStats st;  // the block's counters while its wavefront works on it
};
// the step kernels' scratch: a table that holds any move the path's other
// capacities allow
using WaveLDS = WaveLDST<HT>;
static_assert(WaveLDS::TLIMIT == HT_LIMIT, "table limit");
// The rebuild branch does not use the repair scratch (everything before
// `st`) and lays its own arrays over it, so they cost no LDS of their own
// (4 KB less lets five step wavefronts share a compute unit instead of four):
// the dry run's position hash (PH_CAP 8-byte entries) at 0, then the points
// moved this step and their new places; the parallel build's attempts at 0
// (the dry run is over by then) and its counters and deferred points after
// the moved-point arrays.
constexpr int DRY_HASH_BYTES = 2048 * 8;
constexpr int DRY_V_OFF = DRY_HASH_BYTES;
constexpr int DRY_Q_OFF = DRY_V_OFF + 4 * DRYMAX;
constexpr int PB_LDS_OFF = DRY_Q_OFF + 8 * DRYMAX;
constexpr int PB_LDS_INTS = 4 + 256;
static_assert(PB_LDS_OFF + 4 * PB_LDS_INTS <= (int)offsetof(WaveLDS, st), "rebuild arrays overlap the counters");
__device__ __forceinline__ int* dry_v_of(WaveLDS& S) { return reinterpret_cast<int*>(reinterpret_cast<char*>(&S) + DRY_V_OFF); }
__device__ __forceinline__ int2* dry_q_of(WaveLDS& S) { return reinterpret_cast<int2*>(reinterpret_cast<char*>(&S) + DRY_Q_OFF); }
__device__ __forceinline__ int* pb_lds_of(WaveLDS& S) { return reinterpret_cast<int*>(reinterpret_cast<char*>(&S) + PB_LDS_OFF); }

// ---------------------------------------------------------------- wave ops

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }
__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }
__device__ __forceinline__ int lanes_below(uint64_t m) { return __popcll(m & lanemask_lt()); }
__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll((long long)m) - 1; }
// Ordering between the lanes of the wavefront for LDS traffic: LDS
// operations of one wavefront complete in issue order, so only the compiler
// must be kept from moving memory operations across this point.
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
// Full workgroup barrier with fence: global stores of the wavefront are
// complete and visible before any later load (used between two moves).
__device__ __forceinline__ void gsync() { __syncthreads(); }

__device__ __forceinline__ int vget(const int4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : v.z);
}
__device__ __forceinline__ void vset(int4& v, int i, int val) {
    if (i == 0) v.x = val;
    else if (i == 1) v.y = val;
    else v.z = val;
}
__device__ __forceinline__ int2 cget(const Tri& t, int i) {
    return i == 0 ? make_int2(t.c01.x, t.c01.y)
                  : (i == 1 ? make_int2(t.c01.z, t.c01.w) : make_int2(t.c2.x, t.c2.y));
}
__device__ __forceinline__ void cset(Tri& t, int i, int2 p) {
    if (i == 0) { t.c01.x = p.x; t.c01.y = p.y; }
    else if (i == 1) { t.c01.z = p.x; t.c01.w = p.y; }
    else { t.c2.x = p.x; t.c2.y = p.y; }
}
__device__ __forceinline__ bool same(int2 a, int2 b) { return a.x == b.x && a.y == b.y; }

// Every slot and vertex index read from memory is checked against the
// block's ranges before use, so corrupted state ends in an error code,
// never in an access outside the block.
__device__ __forceinline__ bool bad_slot(const BlockView& B, int s) {
    return (unsigned)s >= (unsigned)B.ntri;
}
__device__ __forceinline__ bool bad_tri(const BlockView& B, const int4& v) {
    return (unsigned)v.x >= (unsigned)B.n || (unsigned)v.y >= (unsigned)B.n ||
           (v.z != GHOST && (unsigned)v.z >= (unsigned)B.n);
}

// A record with all four parts requested before any is used.  Left to
// itself the compiler issues the parts that a check's branch does not need
// behind that branch, one memory round trip later; the empty asm takes every
// part as an operand, so all four loads leave together and one wait covers
// them.
__device__ __forceinline__ Tri load_tri(const Tri* p) {
    const int4* q = reinterpret_cast<const int4*>(p);
    Tri t;
    t.v = q[0];
    t.n = q[1];
    t.c01 = q[2];
    t.c2 = q[3];
    asm volatile("" : "+v"(t.v.x), "+v"(t.v.y), "+v"(t.v.z), "+v"(t.n.x), "+v"(t.n.y), "+v"(t.n.z),
                 "+v"(t.c01.x), "+v"(t.c01.y), "+v"(t.c01.z), "+v"(t.c01.w), "+v"(t.c2.x), "+v"(t.c2.y));
    return t;
}
// Two records at once, in one round trip.
__device__ __forceinline__ void load_tri2(const Tri* p, const Tri* r, Tri& a, Tri& b) {
    const int4* q = reinterpret_cast<const int4*>(p);
    const int4* u = reinterpret_cast<const int4*>(r);
    a.v = q[0]; a.n = q[1]; a.c01 = q[2]; a.c2 = q[3];
    b.v = u[0]; b.n = u[1]; b.c01 = u[2]; b.c2 = u[3];
    asm volatile("" : "+v"(a.v.x), "+v"(a.v.y), "+v"(a.v.z), "+v"(a.n.x), "+v"(a.n.y), "+v"(a.n.z),
                 "+v"(a.c01.x), "+v"(a.c01.y), "+v"(a.c01.z), "+v"(a.c01.w), "+v"(a.c2.x), "+v"(a.c2.y),
                 "+v"(b.v.x), "+v"(b.v.y), "+v"(b.v.z), "+v"(b.n.x), "+v"(b.n.y), "+v"(b.n.z),
                 "+v"(b.c01.x), "+v"(b.c01.y), "+v"(b.c01.z), "+v"(b.c01.w), "+v"(b.c2.x), "+v"(b.c2.y));
}

// ---------------------------------------------------------------- predicates
// Every coordinate is in [0, 2^24), so differences are below 2^24 in
// magnitude.

// Twice the signed area of (a, b, c): > 0 counter-clockwise.  Exact in
// doubles: each product is below 2^48 and their difference below 2^49.
__device__ __forceinline__ double orient(int2 a, int2 b, int2 c) {
#pragma clang fp contract(off)
    const double abx = (double)(b.x - a.x), aby = (double)(b.y - a.y);
    const double acx = (double)(c.x - a.x), acy = (double)(c.y - a.y);
    return abx * acy - aby * acx;
}

__device__ __noinline__ int incircle_exact(double al, double bl, double cl, double m_bc, double m_ca,
                                           double m_ab) {
    const __int128 d = (__int128)(long long)al * (long long)m_bc +
                       (__int128)(long long)bl * (long long)m_ca +
                       (__int128)(long long)cl * (long long)m_ab;
    return (d > 0) - (d < 0);
}

// Sign of the incircle determinant (> 0: d strictly inside the circle of the
// counter-clockwise a, b, c).  The lifts |p - d|^2 and the 2x2 minors are
// integers below 2^49, computed exactly in doubles; only the three final
// products and two sums round, so the computed value is within
// 3u(1 + O(u)) * P of the true one, P the sum of the product magnitudes
// (u = 2^-53).  A result larger than 4u * P in magnitude has the right sign;
// otherwise the determinant is recomputed in 128-bit integers from the same
// exact lifts and minors.
__device__ __forceinline__ int incircle(int2 a, int2 b, int2 c, int2 d) {
#pragma clang fp contract(off)
    const double adx = (double)(a.x - d.x), ady = (double)(a.y - d.y);
    const double bdx = (double)(b.x - d.x), bdy = (double)(b.y - d.y);
    const double cdx = (double)(c.x - d.x), cdy = (double)(c.y - d.y);
    const double al = adx * adx + ady * ady;
    const double bl = bdx * bdx + bdy * bdy;
    const double cl = cdx * cdx + cdy * cdy;
    const double m_bc = bdx * cdy - bdy * cdx;
    const double m_ca = cdx * ady - cdy * adx;
    const double m_ab = adx * bdy - ady * bdx;
    const double p1 = al * m_bc;
    const double p2 = bl * m_ca;
    const double p3 = cl * m_ab;
    const double det = (p1 + p2) + p3;
    const double perm = (fabs(p1) + fabs(p2)) + fabs(p3);
    const double bound = perm * 0x1p-51;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return incircle_exact(al, bl, cl, m_bc, m_ca, m_ab);
}

__device__ __forceinline__ int sgn(double v) { return (v > 0) - (v < 0); }

// Exact ties: the point with the largest rank is lifted most and decides
// through the cofactor of its height in the lifted 4x4 determinant
// (rows x, y, x^2+y^2, 1 in the order a, b, c, d).
__device__ __noinline__ int incircle_tie(int2 a, int ra, int2 b, int rb, int2 c, int rc, int2 d,
                                         int rd) {
    if (ra > rb && ra > rc && ra > rd) return sgn(orient(b, c, d));
    if (rb > rc && rb > rd) return -sgn(orient(a, c, d));
    if (rc > rd) return sgn(orient(a, b, d));
    return -sgn(orient(a, b, c));
}

// Incircle with ties on exactly cocircular points broken by the id lift.
__device__ __forceinline__ int incircle_star(int2 a, int ra, int2 b, int rb, int2 c, int rc,
                                             int2 d, int rd) {
    const int s = incircle(a, b, c, d);
    if (s != 0) return s;
    return incircle_tie(a, ra, b, rb, c, rc, d, rd);
}

// Ghost (a, b, inf) covers the open half-plane left of a->b and the open
// segment ab; a new point there destroys it.
__device__ __forceinline__ bool ghost_conflict(int2 a, int2 b, int2 q) {
    const double o = orient(a, b, q);
    if (o != 0) return o > 0;
    const long long t1 = (long long)(q.x - a.x) * (b.x - a.x) + (long long)(q.y - a.y) * (b.y - a.y);
    const long long t2 = (long long)(q.x - b.x) * (a.x - b.x) + (long long)(q.y - b.y) * (a.y - b.y);
    return t1 > 0 && t2 > 0;
}

// Does inserting point q (rank rq) destroy triangle t?
__device__ __forceinline__ bool conflicts(const Tri& t, int2 q, int rq) {
    if (t.v.z == GHOST) return ghost_conflict(cget(t, 0), cget(t, 1), q);
    return incircle_star(cget(t, 0), t.v.x, cget(t, 1), t.v.y, cget(t, 2), t.v.z, q, rq) > 0;
}

// ---------------------------------------------------------------- table

template <int H>
__device__ __forceinline__ int thash(int s) {
    return (int)(((unsigned)s * 0x9E3779B1u) >> (32 - __builtin_ctz(H)));
}

template <class WL>
__device__ __forceinline__ void table_clear(WL& S) {
    for (int h = lane_id(); h < WL::TN; h += WAVE) {
        S.tkey[h] = -1;
        S.tflag[h] = 0;
    }
    wsync();
}

// Per-kernel setup of the wave's scratch: an empty table.
template <class WL>
__device__ __forceinline__ void scratch_init(WL& S) { table_clear(S); }

// The t-th triple i < j < l < 16 in colex order (t < 560): l is the number
// of tetrahedral numbers C(l'+1, 3) <= t, j the number of triangular numbers
// C(j'+1, 2) <= t - C(l, 3); no loops, no tables.
__device__ __forceinline__ void triple_of(int t, int* i, int* j, int* l) {
    int L = 2;
#pragma unroll
    for (int x = 3; x < EMK; ++x) L += t >= x * (x - 1) * (x - 2) / 6;
    const int r = t - L * (L - 1) * (L - 2) / 6;
    int J = 1;
#pragma unroll
    for (int x = 2; x < EMK; ++x) J += r >= x * (x - 1) / 2;
    *l = L;
    *j = J;
    *i = r - J * (J - 1) / 2;
}

// Entry of slot s, or -1.
template <class WL>
__device__ __forceinline__ int tfind(const WL& S, int s) {
    int h = thash<WL::TN>(s);
    for (int i = 0; i < WL::TN; ++i) {
        const int k = S.tkey[h];
        if (k == s) return h;
        if (k == -1) return -1;
        h = (h + 1) & (WL::TN - 1);
    }
    return -1;
}

// Claim the entry of slot s for every lane with want set: found if present,
// else created (linear probing, claimed by compare-and-swap).  *mine tells
// the lane that created it.  -1 if the table is full.
template <class WL>
__device__ __forceinline__ int tclaim(WL& S, bool want, int s, bool* mine) {
    *mine = false;
    if (!want) return -1;
    int h = thash<WL::TN>(s);
    for (int i = 0; i < WL::TN; ++i) {
        const int k = S.tkey[h];
        if (k == s) return h;
        if (k == -1) {
            const int old = atomicCAS(&S.tkey[h], -1, s);
            if (old == -1) { *mine = true; return h; }
            if (old == s) return h;
        }
        h = (h + 1) & (WL::TN - 1);
    }
    return -1;
}

// Table entry of slot s for every lane with want set, reading the record
// from memory if it is not in the table yet.  Called by the whole wave.
// *used counts the entries in use (wave-uniform); returns -1 on a full table.
// Record the entries the lanes with `mine` set just claimed.
template <class WL>
__device__ __forceinline__ void tnote(WL& S, bool mine, int e, int* used) {
    const uint64_t m = ballot(mine);
    if (mine && *used + lanes_below(m) < WL::TN) S.tused[*used + lanes_below(m)] = e;
    *used += __popcll(m);
}

template <class WL>
__device__ __forceinline__ int tget(const BlockView& B, WL& S, bool want, int s, int* used) {
    // The record leaves memory before the claim, so the claim's LDS round
    // trips run while it is in flight; a lane whose slot is in the table
    // already drops what it read.
    int4 r0 = make_int4(0, 0, 0, 0), r1 = r0, r2 = r0, r3 = r0;
    if (want && !bad_slot(B, s)) {
        const int4* src = reinterpret_cast<const int4*>(B.tri + s);
        r0 = src[0];
        r1 = src[1];
        r2 = src[2];
        r3 = src[3];
    }
    bool mine;
    const int e = tclaim(S, want, s, &mine);
    if (mine) {
        int4* dst = reinterpret_cast<int4*>(&S.trec[e]);
        dst[0] = r0;
        dst[1] = r1;
        dst[2] = r2;
        dst[3] = r3;
        S.tflag[e] = 0;
    }
    tnote(S, mine, e, used);
    wsync();
    return e;
}

// Record of slot s as the move sees it (table first, memory else).
template <class WL>
__device__ __forceinline__ Tri tread(const BlockView& B, const WL& S, int s) {
    const int e = tfind(S, s);
    if (e >= 0) return S.trec[e];
    return load_tri(B.tri + s);
}

// ---------------------------------------------------------------- walk
// Visibility walk toward q (every lane runs it identically).  Ends at a
// triangle that q destroys: a real triangle whose closed area holds q, or a
// ghost whose half-plane holds q.  *hit gets the local index of a vertex
// sitting exactly at q (-1 if none).  Returns -1 if the step limit is hit.
// TABLE: read through the move's write-back table (after changes).
template <bool TABLE, class WL>
__device__ __forceinline__ int walk(const BlockView& B, const WL* S, int start, int2 q, int* hit, int* hops,
                    int* path = nullptr, int* npath = nullptr) {
    int cur = start, entry = -1;
    const int limit = 4 * B.ntri + 16;
    *hit = -1;
    for (int h = 0; h < limit; ++h) {
        if (bad_slot(B, cur)) return -1;
        if (path) {  // record the slots read (wave-uniform; lane 0 writes)
            if (*npath < WPMAX && lane_id() == 0) path[*npath] = cur;
            ++*npath;
        }
        const Tri t = TABLE ? tread(B, *S, cur) : load_tri(B.tri + cur);
        if (bad_tri(B, t.v)) return -1;
        const int2 p0 = cget(t, 0), p1 = cget(t, 1);
        if (t.v.z == GHOST) {
            if (ghost_conflict(p0, p1, q)) {
                *hops += h + 1;
                return cur;
            }
            entry = t.n.z & 3;
            cur = t.n.z >> 2;
            continue;
        }
        const int2 p2 = cget(t, 2);
        int next = -1;
        if (entry != 0 && orient(p1, p2, q) < 0) next = 0;
        else if (entry != 1 && orient(p2, p0, q) < 0) next = 1;
        else if (entry != 2 && orient(p0, p1, q) < 0) next = 2;
        if (next < 0) {
            if (same(p0, q)) *hit = t.v.x;
            else if (same(p1, q)) *hit = t.v.y;
            else if (same(p2, q)) *hit = t.v.z;
            *hops += h + 1;
            return cur;
        }
        const int r = vget(t.n, next);
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

// Insert point qv at q into the block's DT* (Bowyer-Watson, Sec. IV), in the
// write-back table.  The cavity starts from the nseed table entries already
// in S.cav_ent (flagged F_CAV) or, when nseed is 0, from `seed`, a triangle
// q destroys; f0, f1 are two free slots that take the two triangles the
// insertion adds.  The cavity grows level by level: the lanes test the
// frontier's neighbours, ballots and prefix counts compact the survivors.
// *used: table entries in use; *nvt: pending incident-triangle updates.
// Returns ST_OK or an error code (the table is then not to be written back).
template <class WL>
__device__ __forceinline__ int insert_vertex(const BlockView& B, WL& S, int qv, int2 q, int seed, int nseed, int f0,
                             int f1, int* used, int* nvt, BlockStats* st) {
    const int lane = lane_id();
    if (bad_slot(B, f0) || bad_slot(B, f1)) return ST_INTERNAL;
    const int fetched0 = *used;
    int ncav = nseed, nbnd = 0;  // wave-uniform counts of S.cav_ent and S.bnd_*
    if (nseed == 0) {
        if (bad_slot(B, seed)) return ST_INTERNAL;
        const int se = tget(B, S, lane == 0, seed, used);
        const int se0 = __shfl(se, 0);
        if (se0 < 0) return ST_CAPACITY;
        if (bad_tri(B, S.trec[se0].v)) return ST_INTERNAL;
        if (lane == 0) {
            S.cav_ent[0] = se0;
            S.tflag[se0] |= F_CAV;
        }
        wsync();
        ncav = 1;
    }
    int fs = 0, fe = ncav;
    while (fs < fe) {
        const int ncand = 3 * (fe - fs);
        for (int base = 0; base < ncand; base += WAVE) {
            const int j = base + lane;
            const bool act = j < ncand;
            const int ci = fs + j / 3, e = j % 3;
            Tri ct;
            int nref = 0, ns = 0;
            if (act) {
                ct = S.trec[S.cav_ent[ci]];
                nref = vget(ct.n, e);
                ns = nref >> 2;
            }
            const bool okslot = act && !bad_slot(B, ns);
            if (ballot(act && !okslot)) return ST_INTERNAL;
            const int ne = tget(B, S, okslot, ns, used);
            if (ballot(okslot && ne < 0) || *used > WL::TLIMIT) return ST_CAPACITY;
            bool incav = false, conf = false, bad = false;
            if (act) {
                incav = (S.tflag[ne] & F_CAV) != 0;
                if (!incav) {
                    const Tri nt = S.trec[ne];
                    bad = bad_tri(B, nt.v);
                    conf = !bad && conflicts(nt, q, qv);
                }
            }
            if (ballot(bad)) return ST_INTERNAL;
            bool acc = false;
            if (act && !incav && conf) acc = (atomicOr(&S.tflag[ne], F_CAV) & F_CAV) == 0;
            const bool bnd = act && !incav && !conf;
            const uint64_t macc = ballot(acc), mb = ballot(bnd);
            const int nacc = __popcll(macc), nbn = __popcll(mb);
            if (ncav + nacc > CMAX || nbnd + nbn > BMAX) return ST_CAPACITY;
            if (acc) S.cav_ent[ncav + lanes_below(macc)] = ne;
            if (bnd) {
                const int pos = nbnd + lanes_below(mb);
                S.bnd_a[pos] = vget(ct.v, (e + 1) % 3);
                S.bnd_b[pos] = vget(ct.v, (e + 2) % 3);
                S.bnd_pa[pos] = cget(ct, (e + 1) % 3);
                S.bnd_pb[pos] = cget(ct, (e + 2) % 3);
                S.bnd_out[pos] = nref;
            }
            wsync();
            ncav += nacc;
            nbnd += nbn;
        }
        fs = fe;
        fe = ncav;
    }
    const int c = ncav, nb = nbnd;
    if (nb != c + 2) return ST_INTERNAL;
    const int fetched = *used - fetched0;

    // table entries of the two extra slots
    bool mine;
    const int fent = tclaim(S, lane < 2, lane == 0 ? f0 : f1, &mine);
    tnote(S, mine, fent, used);
    if (ballot(lane < 2 && fent < 0) || *used > WL::TN) return ST_CAPACITY;
    const int fe0 = __shfl(fent, 0), fe1 = __shfl(fent, 1);
    wsync();

    // fan: one triangle (a, b, q) per boundary edge, into the c cavity
    // entries and the two extra ones
    for (int i = lane; i < nb; i += WAVE) {
        const int3 ph = fan_phys(S.bnd_a[i], S.bnd_b[i]);
        S.bnd_slot[i] = i < c ? S.tkey[S.cav_ent[i]] : (i == c ? f0 : f1);
        S.bnd_ph[i] = ph.x | (ph.y << 2) | (ph.z << 4);
    }
    wsync();
    int err = 0;
    for (int i = lane; i < nb; i += WAVE) {
        const int a = S.bnd_a[i], b = S.bnd_b[i], out = S.bnd_out[i];
        const int ent = i < c ? S.cav_ent[i] : (i == c ? fe0 : fe1);
        const int slot = S.bnd_slot[i];
        const int phi = S.bnd_ph[i];
        const int pa = phi & 3, pb = (phi >> 2) & 3, pq = phi >> 4;
        int jn = -1, jm = -1;  // fan triangles starting at b / ending at a
#pragma unroll 8
        for (int m = 0; m < nb; ++m) {
            jn = S.bnd_a[m] == b ? m : jn;
            jm = S.bnd_b[m] == a ? m : jm;
        }
        const int oe = tfind(S, out >> 2);
        if (jn < 0 || jm < 0 || oe < 0) { err = 1; continue; }
        Tri r;
        r.v = make_int4(0, 0, 0, 0);
        r.n = make_int4(0, 0, 0, 0);
        r.c01 = make_int4(0, 0, 0, 0);
        r.c2 = make_int4(0, 0, 0, 0);
        vset(r.v, pa, a);
        vset(r.v, pb, b);
        vset(r.v, pq, qv);
        if (a != GHOST) cset(r, pa, S.bnd_pa[i]);
        if (b != GHOST) cset(r, pb, S.bnd_pb[i]);
        cset(r, pq, q);
        vset(r.n, pq, out);                                          // across (a, b)
        vset(r.n, pa, S.bnd_slot[jn] * 4 + ((S.bnd_ph[jn] >> 2) & 3));  // across (b, q): jn's edge (q, b)
        vset(r.n, pb, S.bnd_slot[jm] * 4 + (S.bnd_ph[jm] & 3));         // across (q, a): jm's edge (a, q)
        S.trec[ent] = r;
        S.tflag[ent] = F_DIRTY;
        reinterpret_cast<int*>(&S.trec[oe].n)[out & 3] = slot * 4 + pq;
        S.tflag[oe] |= F_DIRTY;
        const int vi = *nvt + i;
        S.vt_v[vi] = a;  // GHOST entries are skipped at write-back
        S.vt_s[vi] = slot;
    }
    if (ballot(err)) return ST_INTERNAL;
    if (lane == 0) {
        S.vt_v[*nvt + nb] = qv;
        S.vt_s[*nvt + nb] = S.tkey[S.cav_ent[0]];
    }
    *nvt += nb + 1;
    wsync();
    if (lane == 0 && st) {
        st->cavity_sum += c;
        // records read: seed, cavity and tested neighbours not already at
        // hand; written: the fan and the c + 2 patched neighbours; c + 3
        // incident-triangle updates
        st->tri_touched += fetched + 2 * nb;
        st->alg_bytes += 64LL * fetched + 128LL * nb + 4LL * (nb + 1);
    }
    return ST_OK;
}

// Write back the move: changed records, then the incident-triangle updates
// of the deletion, then those of the insertion (no point occurs twice in
// one list; stores of one wavefront to one address land in program order,
// so the insertion's value wins), and empty the table.
template <class WL>
__device__ __forceinline__ void commit(const BlockView& B, WL& S, int used, int nvt_del, int nvt) {
    const int lane = lane_id();
    for (int u = lane; u < used; u += WAVE) {
        const int h = S.tused[u];
        if (S.tflag[h] & F_DIRTY) B.tri[S.tkey[h]] = S.trec[h];
    }
    for (int i = lane; i < nvt_del; i += WAVE) {
        const int v = S.vt_v[i];
        if (v != GHOST) B.vtri[v] = S.vt_s[i];
    }
    for (int i = nvt_del + lane; i < nvt; i += WAVE) {
        const int v = S.vt_v[i];
        if (v != GHOST) B.vtri[v] = S.vt_s[i];
    }
    wsync();
    for (int u = lane; u < used; u += WAVE) {
        const int h = S.tused[u];
        S.tkey[h] = -1;
        S.tflag[h] = 0;
    }
    wsync();
}

// Empty the table entries of the tused list without writing anything back
// (a planned move that is not committed).
template <class WL>
__device__ __forceinline__ void table_drop(WL& S, int used) {
    wsync();
    for (int u = lane_id(); u < used; u += WAVE) {
        const int h = S.tused[u];
        S.tkey[h] = -1;
        S.tflag[h] = 0;
    }
    wsync();
}

// ---------------------------------------------------------------- delete

// Gather the star of p counter-clockwise into S: star_slot, link (q_s) and
// its position lxy, outref (the triangle across link edge q_s q_s+1), with
// the vertex at infinity, if p is on the hull, rotated to the last place;
// and the triangles outside the link edges into the table.  Two walkers
// turn around p in opposite directions and meet halfway.
// t0: p's incident triangle.  Returns the degree k (>= 3) or an error code.
template <class WL>
__device__ __forceinline__ int gather_star(const BlockView& B, WL& S, int p, int t0, int* used, BlockStats* st) {
    const int lane = lane_id();
    if (bad_slot(B, t0)) return ST_INTERNAL;
    const Tri r0 = load_tri(B.tri + t0);
    if (bad_tri(B, r0.v)) return ST_INTERNAL;
    const int pi0 = r0.v.x == p ? 0 : (r0.v.y == p ? 1 : (r0.v.z == p ? 2 : -1));
    if (pi0 < 0) return ST_INTERNAL;
    // counter-clockwise entries at 0, 1, ...; clockwise ones at KMAX-1,
    // KMAX-2, ...
    if (lane == 0) {
        S.star_slot[0] = t0;
        S.link[0] = vget(r0.v, (pi0 + 1) % 3);
        S.lxy[0] = cget(r0, (pi0 + 1) % 3);
        S.outref[0] = vget(r0.n, pi0);
    }
    int na = 1, nc = 0;
    int ccw_ref = vget(r0.n, (pi0 + 1) % 3), cw_ref = vget(r0.n, (pi0 + 2) % 3);
    int last_ccw = t0, last_cw = t0;
    while (true) {
        if (na + nc + 2 > KMAX) return ST_CAPACITY;
        const int cs = ccw_ref >> 2, ws = cw_ref >> 2;
        if (cs == last_cw) break;
        if (bad_slot(B, cs) || bad_slot(B, ws)) return ST_INTERNAL;
        Tri rc, rw;
        load_tri2(B.tri + cs, B.tri + ws, rc, rw);
        const int pc = ((ccw_ref & 3) + 1) % 3, pw = ((cw_ref & 3) + 2) % 3;
        if (bad_tri(B, rc.v) || bad_tri(B, rw.v) || vget(rc.v, pc) != p || vget(rw.v, pw) != p)
            return ST_INTERNAL;
        if (lane == 0) {
            S.star_slot[na] = cs;
            S.link[na] = vget(rc.v, (pc + 1) % 3);
            S.lxy[na] = cget(rc, (pc + 1) % 3);
            S.outref[na] = vget(rc.n, pc);
        }
        ++na;
        last_ccw = cs;
        if (ws == cs) break;
        if (lane == 0) {
            const int d = KMAX - 1 - nc;
            S.star_slot[d] = ws;
            S.link[d] = vget(rw.v, (pw + 1) % 3);
            S.lxy[d] = cget(rw, (pw + 1) % 3);
            S.outref[d] = vget(rw.n, pw);
        }
        ++nc;
        last_cw = ws;
        ccw_ref = vget(rc.n, (pc + 1) % 3);
        cw_ref = vget(rw.n, (pw + 2) % 3);
        if ((cw_ref >> 2) == last_ccw) break;
    }
    const int k = na + nc;
    wsync();
    // move the clockwise entries next to the counter-clockwise ones and, if
    // p is on the hull, rotate the vertex at infinity to the end
    int slot = 0, link = 0, outr = 0;
    int2 lxy = make_int2(0, 0);
    if (lane < k) {
        const int src = lane < na ? lane : KMAX - 1 - (k - 1 - lane);
        slot = S.star_slot[src];
        link = S.link[src];
        lxy = S.lxy[src];
        outr = S.outref[src];
    }
    const uint64_t gm = ballot(lane < k && link == GHOST);
    const int rot = gm ? first_lane(gm) + 1 : 0;  // new index = old - rot (mod k)
    if (ballot(lane < k && bad_slot(B, outr >> 2))) return ST_INTERNAL;
    wsync();
    // the triangles around the star, one per lane, in one round trip
    const int oe = tget(B, S, lane < k, outr >> 2, used);
    if (ballot(lane < k && oe < 0)) return ST_CAPACITY;
    if (lane < k) {
        const int d = (lane - rot + k) % k;
        S.star_slot[d] = slot;
        S.link[d] = link;
        S.lxy[d] = lxy;
        S.outref[d] = outr;
        S.out_ent[d] = oe;
    }
    wsync();
    if (lane == 0 && st) {
        st->star_sum += k;
        st->tri_touched += k + *used;
        st->alg_bytes += 64LL * (k + *used) + 4;  // star and surrounding records, vtri[p]
    }
    return k;
}

// Is q inside the closed region of p's star (p at position pp), and does it
// sit on a link vertex?  Star triangle s is (p, q_s, q_s+1); a ghost one is
// tested as the half-plane it stands for.
template <class WL>
__device__ __forceinline__ void locate_in_star(const WL& S, int k, int2 pp, int2 q,
                                               bool* in_star, bool* on_vertex) {
    const int lane = lane_id();
    bool in = false, on = false;
    if (lane < k) {
        const int a = S.link[lane], b = S.link[(lane + 1) % k];
        const int2 pa = S.lxy[lane], pb = S.lxy[(lane + 1) % k];
        if (b == GHOST) in = ghost_conflict(pp, pa, q);       // (p, q_s, inf)
        else if (a == GHOST) in = ghost_conflict(pb, pp, q);  // (q_s+1, p, inf)
        else in = orient(pp, pa, q) >= 0 && orient(pa, pb, q) >= 0 && orient(pb, pp, q) >= 0;
        on = a != GHOST && same(pa, q);
    }
    *in_star = ballot(in) != 0;
    *on_vertex = ballot(on) != 0;
}

// After the hole of p is filled (q inside the star): every triangle of the
// table that q destroys -- hole triangles, then triangles around the star,
// each once -- goes into S.cav_ent, flagged F_CAV.  The triangles a point
// destroys form one connected region, so the cavity grows from these
// without a walk.  Returns their number.
template <class WL>
__device__ __forceinline__ int seed_cavity(WL& S, int k, int2 q, int qv) {
    const int lane = lane_id();
    const int he = lane < k - 2 ? S.hole_ent[lane] : -1;
    const bool ch = he >= 0 && conflicts(S.trec[he], q, qv);
    const uint64_t mh = ballot(ch);
    if (ch) {
        S.cav_ent[lanes_below(mh)] = he;
        S.tflag[he] |= F_CAV;
    }
    const int nh = __popcll(mh);
    wsync();
    const int oe = lane < k ? S.out_ent[lane] : -1;
    bool co = oe >= 0 && conflicts(S.trec[oe], q, qv);
    // a triangle outside two link edges is taken once
    if (co) co = (atomicOr(&S.tflag[oe], F_CAV) & F_CAV) == 0;
    const uint64_t mo = ballot(co);
    if (co) S.cav_ent[nh + lanes_below(mo)] = oe;
    wsync();
    return nh + __popcll(mo);
}

// Widen the star region by the triangles q destroys around it, level by
// level, so that the star-only path covers them as well: a destroyed
// triangle T outside boundary edge (a, b) is (r, b, a), and the boundary
// then runs a, r, b there; the triangles across (a, r) and (r, b) are read
// and tested in turn.  Taken only if every grown T is a real triangle whose
// r is not on the boundary yet, the r of one level are distinct (the region
// stays a simple polygon with no vertex inside), the polygon keeps at most
// EMK - 1 vertices and, at the end, no triangle across the boundary is
// destroyed by q (the triangles q destroys are connected, so its cavity
// then lies in the region).  The region is then retriangulated like a star:
// DT*(boundary + q) inside it.  cm: link edges whose outside triangle q
// destroys.  q_out: q lies outside the star, and the region must come to
// hold it (in a grown triangle, not at its corner).  Returns the new vertex
// count -- the polygon arrays rewritten, the grown triangles' slots after
// the star's in S.star_slot -- or 0 with the star's polygon as it was.
template <class WL>
__device__ __forceinline__ int grow_region(const BlockView& B, WL& S, int k, int2 q, int qv, uint64_t cm,
                                           int* used, bool q_out) {
    const int lane = lane_id();
    // the star's polygon, put back if the growth stops short
    int lv0 = GHOST, orf0 = 0, oen0 = 0;
    int2 lp0 = make_int2(0, 0);
    if (lane < k) {
        lv0 = S.link[lane];
        lp0 = S.lxy[lane];
        orf0 = S.outref[lane];
        oen0 = S.out_ent[lane];
    }
    int kr = k, nslot = k;
    bool ok = true, q_in = !q_out;
    while (cm) {
        const int k2 = kr + __popcll(cm);
        if (k2 + 1 > EMK) {
            ok = false;
            break;
        }
        const bool c = lane < kr && ((cm >> lane) & 1ull);
        int lv = GHOST, orf = 0, oen = 0, r = GHOST, u1 = 0, u2 = 0;
        int2 lp = make_int2(0, 0), pr = make_int2(0, 0);
        bool ghost = false;
        if (lane < kr) {
            lv = S.link[lane];
            lp = S.lxy[lane];
            orf = S.outref[lane];
            oen = S.out_ent[lane];
        }
        if (c) {
            const Tri t = S.trec[oen];
            const int e = orf & 3;
            ghost = t.v.z == GHOST;
            r = vget(t.v, e);
            pr = cget(t, e);
            u1 = vget(t.n, (e + 1) % 3);  // across (a, r)
            u2 = vget(t.n, (e + 2) % 3);  // across (r, b)
        }
        // grown triangle (r, b, a) on boundary edge (a, b): does it hold q?
        const int nb = lane + 1 < kr ? lane + 1 : 0;
        const int2 pb = make_int2(__shfl(lp.x, nb), __shfl(lp.y, nb));
        const bool qt = c && !ghost && orient(pr, pb, q) >= 0 && orient(pb, lp, q) >= 0 && orient(lp, pr, q) >= 0;
        q_in = q_in || ballot(qt) != 0;
        bool clash = (c && ghost) || (qt && same(pr, q));  // the hull changes beyond the region, or q is held
        for (int m = 0; m < kr; ++m) {
            const int lm = __builtin_amdgcn_readlane(lv, m), rm = __builtin_amdgcn_readlane(r, m);
            clash = clash || (c && (lm == r || (m != lane && ((cm >> m) & 1ull) && rm == r)));
        }
        if (ballot(clash)) {
            ok = false;
            break;
        }
        // the triangles across the new boundary edges: lanes 0..31 the first
        // edge of each grown triangle, lanes 32..63 the second (kr < 32); both
        // shuffles by every lane (a lane-dependent choice between them would
        // run each with half the lanes off, and a read from a lane that is off
        // does not return its value)
        const int src = lane & 31;
        const bool want = src < kr && ((cm >> src) & 1ull);
        const int s1 = __shfl(u1, src), s2 = __shfl(u2, src);
        const int uref = lane < 32 ? s1 : s2;
        if (ballot(want && bad_slot(B, uref >> 2))) {
            ok = false;
            break;
        }
        const int ue = tget(B, S, want, uref >> 2, used);
        if (ballot(want && ue < 0)) {
            ok = false;
            break;
        }
        const bool uc = want && conflicts(S.trec[ue], q, qv);
        const int ue1 = __shfl(ue, src), ue2 = __shfl(ue, src + 32);
        const int uc1 = __shfl((int)uc, src), uc2 = __shfl((int)uc, src + 32);
        // a moves to a + (grown edges before it), r right after it
        const int at = lane + lanes_below(cm);
        wsync();
        if (lane < kr) {
            S.link[at] = lv;
            S.lxy[at] = lp;
            S.outref[at] = c ? u1 : orf;
            S.out_ent[at] = c ? ue1 : oen;
            S.cav_ent[at] = c ? uc1 : 0;  // the next level's edges
        }
        if (c) {
            S.link[at + 1] = r;
            S.lxy[at + 1] = pr;
            S.outref[at + 1] = u2;
            S.out_ent[at + 1] = ue2;
            S.cav_ent[at + 1] = uc2;
            S.star_slot[nslot + lanes_below(cm)] = orf >> 2;
        }
        wsync();
        nslot += __popcll(cm);
        kr = k2;
        cm = ballot(lane < kr && S.cav_ent[lane] != 0);
    }
    ok = ok && q_in;
    if (!ok) {
        if (lane < k) {
            S.link[lane] = lv0;
            S.lxy[lane] = lp0;
            S.outref[lane] = orf0;
            S.out_ent[lane] = oen0;
        }
        wsync();
        return 0;
    }
    return kr;
}

__device__ __forceinline__ int pack3(int i, int j, int l) { return (i << 16) | (j << 8) | l; }

// The u-th pair i < j < 16 in colex order (u < 120), without loops.
__device__ __forceinline__ void pair_of(int u, int* i, int* j) {
    int J = 1;
#pragma unroll
    for (int x = 2; x < EMK; ++x) J += u >= x * (x - 1) / 2;
    *j = J;
    *i = u - J * (J - 1) / 2;
}

// Retriangulate p's star polygon, its star already gathered by gather_star,
// in the write-back table.  Vertices: the link q_0..q_{k-1} (counter-
// clockwise, the vertex at infinity last when p is on the hull) and, when
// with_q, the new point qv at q as vertex k.
//
//  * Without q -- the Delete step of Fig. 4: the new triangles are the link
//    triples q_i, q_j, q_l (i < j < l) that are counter-clockwise and whose
//    perturbed circle holds no other link vertex -- for a ghost triple
//    (q_i, q_j, inf), no link vertex beyond the line q_i q_j.  These are the
//    Delaunay triangles of the link vertices inside the hole, i.e. exactly
//    DT*(S - p) there; k - 2 of them take the first k - 2 star slots and the
//    last two star slots become free.
//  * With q -- Delete and Insert at once, used when q lies inside the star
//    (a ghost's half-plane included) and destroys none of the triangles
//    around it: then every link edge stays Delaunay, nothing outside the
//    star changes, and the star region holds DT*(link + q) restricted to
//    it: the link triples above that also keep q out of their circle or
//    half-plane, the counter-clockwise triangles (q_i, q_j, q) whose circle
//    holds no link vertex and, when p is on the hull, the ghosts
//    (q_i, q, inf) and (q, q_i, inf) with no link vertex beyond their edge
//    (q on the hull: every face around q lies in the star region, whose
//    boundary edges are Delaunay).  There are k of them, one per star slot.
//
// Lanes stride over the candidate triangles, each rejected at its first
// violating vertex.  *nvt: pending incident-triangle updates.  Returns ST_OK
// or an error code.
//
// A candidate triangle by polygon index in stored order: link indices
// 0..k-1, index k for q; only the last stored vertex can be the vertex at
// infinity.
struct TriCand {
    int i, j, l, vi, vj, vl;
    int2 pi, pj, pl;
    bool ghost, ok;
};

// The candidate with the given indices (already oriented).
template <class WL>
__device__ __forceinline__ TriCand tri_cand_of(const WL& S, int k, int i, int j, int l, int qv, int2 q) {
    TriCand c;
    c.i = i; c.j = j; c.l = l;
    c.vi = i == k ? qv : S.link[i];
    c.vj = j == k ? qv : S.link[j];
    c.vl = l == k ? qv : S.link[l];
    c.pi = i == k ? q : S.lxy[i];
    c.pj = j == k ? q : S.lxy[j];
    c.pl = l == k ? q : S.lxy[l];
    c.ghost = c.vl == GHOST;
    c.ok = true;
    return c;
}

// Candidate t: the link triples first, then the pairs (q_i, q_j) with q,
// then (p on the hull) the ghosts with q; ok tells whether it passes
// orientation and, with q, keeps q out of its circle or half-plane.
template <class WL>
__device__ __forceinline__ TriCand tri_cand(const WL& S, int k, int t, int ntrip, int npair, int ncand,
                                            int qv, int2 q, bool with_q) {
    int i = 0, j = 1, l = 2, kind = 0;  // 0 link triple, 1 (q_i, q_j, q), 2 ghost with q
    bool ok = t < ncand;
    if (ok) {
        if (t >= ntrip + npair) {
            const int u = t - ntrip - npair, a = u >> 1;
            i = (u & 1) ? k : a;
            j = (u & 1) ? a : k;
            l = k - 1;
            kind = 2;
        } else if (t >= ntrip) {
            pair_of(t - ntrip, &i, &j);
            l = k;
            kind = 1;
        } else if (k <= EMK) {
            triple_of(t, &i, &j, &l);
        } else {
            l = (int)cbrtf(6.0f * (float)t) + 1;
            while (l * (l - 1) * (l - 2) / 6 > t) --l;
            while ((l + 1) * l * (l - 1) / 6 <= t) ++l;
            const int r = t - l * (l - 1) * (l - 2) / 6;
            j = (int)sqrtf(2.0f * (float)r) + 1;
            while (j * (j - 1) / 2 > r) --j;
            while ((j + 1) * j / 2 <= r) ++j;
            i = r - j * (j - 1) / 2;
        }
    }
    TriCand c = tri_cand_of(S, k, i, j, l, qv, q);
    ok = ok && c.vi != GHOST && c.vj != GHOST;
    if (kind == 1 && ok) {  // orient (q_i, q_j, q) counter-clockwise
        const double o = orient(c.pi, c.pj, q);
        if (o < 0) c = tri_cand_of(S, k, j, i, l, qv, q);
        ok = o != 0;
    } else if (kind == 0) {
        ok = ok && (c.ghost || orient(c.pi, c.pj, c.pl) > 0);
        // a link triple must also keep q out of its circle or half-plane
        if (ok && with_q)
            ok = c.ghost ? !ghost_conflict(c.pi, c.pj, q)
                         : incircle_star(c.pi, c.vi, c.pj, c.vj, c.pl, c.vl, q, qv) < 0;
    }
    c.ok = ok;
    return c;
}

// Does link vertex m (id vm at pm) rule the candidate out: inside its
// perturbed circle, or inside the half-plane of a ghost?
__device__ __forceinline__ bool cand_killed_by(const TriCand& c, int m, int vm, int2 pm) {
    if (vm == GHOST || m == c.i || m == c.j || m == c.l) return false;
    return c.ghost ? ghost_conflict(c.pi, c.pj, pm)
                   : incircle_star(c.pi, c.vi, c.pj, c.vj, c.pl, c.vl, pm, vm) >= 0;
}

// Lawson flips inside the polygon q_0..q_{k-1} + q (index k), from the fan
// (q_s, q_s+1, q), with q in the polygon's kernel; see fill_star.  The
// triangles live in S.emat (idle here): 8 ints each, vertices at 0..2
// counter-clockwise, at 4 + e the triangle across the edge opposite vertex
// e (-1 on the polygon's boundary).  On success writes the k triangles'
// keys to S.hole_key in candidate order and k to S.nhole; false when the
// flips hit the cap (S.hole_key untouched).
constexpr int LAWSON_MAX_FLIPS = 32;
template <class WL>
__device__ __forceinline__ bool lawson_from_fan(WL& S, int k, int qv, int2 q, int ntrip) {
    const int lane = lane_id();
    int* T = S.emat;
    static_assert(EMK * EMK >= 8 * (EMK - 1), "the flip triangles fit the edge matrix");
    if (lane < k) {
        const int s1 = lane + 1 < k ? lane + 1 : 0, sp = lane > 0 ? lane - 1 : k - 1;
        T[lane * 8 + 0] = lane;
        T[lane * 8 + 1] = s1;
        T[lane * 8 + 2] = k;
        T[lane * 8 + 4] = s1;  // across (s+1, q)
        T[lane * 8 + 5] = sp;  // across (q, s)
        T[lane * 8 + 6] = -1;  // link edge
    }
    wsync();
    bool settled = false;
    for (int it = 0; it <= LAWSON_MAX_FLIPS; ++it) {
        // one lane per (triangle, edge); each inner edge tested once, from
        // its lower-numbered triangle: t = (c, a, b) and u = (d, b, a)
        // share edge (a, b), and a flip makes them t = (c, a, d) and u =
        // (c, d, b), sharing (c, d)
        const int t = lane >> 2, e = lane & 3;
        bool flip = false;
        int u = -1, c = 0, a = 0, b = 0, d = 0, n_bc = -1, n_ca = -1, n_ad = -1, n_db = -1;
        if (t < k && e < 3) {
            const int e1 = e == 2 ? 0 : e + 1, e2 = e == 0 ? 2 : e - 1;
            u = T[t * 8 + 4 + e];
            c = T[t * 8 + e];
            a = T[t * 8 + e1];
            b = T[t * 8 + e2];
            n_bc = T[t * 8 + 4 + e1];
            n_ca = T[t * 8 + 4 + e2];
            if (u > t) {
                const int u0 = T[u * 8 + 0], u1 = T[u * 8 + 1];
                const int f = u0 != a && u0 != b ? 0 : (u1 != a && u1 != b ? 1 : 2);
                const int f1 = f == 2 ? 0 : f + 1, f2 = f == 0 ? 2 : f - 1;
                d = T[u * 8 + f];
                n_ad = T[u * 8 + 4 + f1];
                n_db = T[u * 8 + 4 + f2];
                const int2 pc = c < k ? S.lxy[c] : q, pa = a < k ? S.lxy[a] : q;
                const int2 pb = b < k ? S.lxy[b] : q, pd = d < k ? S.lxy[d] : q;
                const int vc = c < k ? S.link[c] : qv, va = a < k ? S.link[a] : qv;
                const int vb = b < k ? S.link[b] : qv, vd = d < k ? S.link[d] : qv;
                flip = incircle_star(pc, vc, pa, va, pb, vb, pd, vd) > 0;
            }
        }
        const uint64_t m = ballot(flip);
        if (!m) {
            settled = true;
            break;
        }
        if (it == LAWSON_MAX_FLIPS) break;
        if (lane == first_lane(m)) {  // the first edge that fails flips
            T[t * 8 + 0] = c; T[t * 8 + 1] = a; T[t * 8 + 2] = d;
            T[t * 8 + 4] = n_ad; T[t * 8 + 5] = u; T[t * 8 + 6] = n_ca;
            T[u * 8 + 0] = c; T[u * 8 + 1] = d; T[u * 8 + 2] = b;
            T[u * 8 + 4] = n_db; T[u * 8 + 5] = n_bc; T[u * 8 + 6] = t;
            if (n_ad >= 0)
                for (int g = 4; g < 7; ++g)
                    if (T[n_ad * 8 + g] == u) T[n_ad * 8 + g] = t;
            if (n_bc >= 0)
                for (int g = 4; g < 7; ++g)
                    if (T[n_bc * 8 + g] == t) T[n_bc * 8 + g] = u;
        }
        wsync();
    }
    if (!settled) return false;
    // keys and candidate indices as the search forms them: a triangle with
    // q is the pair candidate (i, j, q), counter-clockwise; one without is
    // the link triple in increasing order
    int key = 0, cidx = 0x7fffffff;
    if (lane < k) {
        const int v0 = T[lane * 8 + 0], v1 = T[lane * 8 + 1], v2 = T[lane * 8 + 2];
        if (v0 == k || v1 == k || v2 == k) {
            const int i = v2 == k ? v0 : (v0 == k ? v1 : v2);
            const int j = v2 == k ? v1 : (v0 == k ? v2 : v0);
            const int lo = min(i, j), hi = max(i, j);
            key = pack3(i, j, k);
            cidx = ntrip + hi * (hi - 1) / 2 + lo;
        } else {
            const int a = min(v0, min(v1, v2)), c = max(v0, max(v1, v2)), b = v0 + v1 + v2 - a - c;
            key = pack3(a, b, c);
            cidx = c * (c - 1) * (c - 2) / 6 + b * (b - 1) / 2 + a;
        }
    }
    int rank = 0;
    for (int u = 0; u < k; ++u) rank += __builtin_amdgcn_readlane(cidx, u) < cidx ? 1 : 0;
    wsync();
    if (lane < k) S.hole_key[rank] = key;
    if (lane == 0) S.nhole = k;
    return true;
}

template <class WL>
__device__ __forceinline__ int fill_star(const BlockView& B, WL& S, int k, int qv, int2 q, bool with_q, int* used,
                         int* nvt, BlockStats* st, bool direct = false) {
    const int lane = lane_id();
    if (k < 3) return ST_INTERNAL;
    if (k > TRIPLE_KMAX || (with_q && k + 1 > EMK)) return ST_CAPACITY;
    if (lane == 0) S.nhole = 0;
    if (lane < k) S.edge_tri[lane] = -1;
    wsync();
    const int lv = lane < k ? S.link[lane] : GHOST;
    const int2 lp = lane < k ? S.lxy[lane] : make_int2(0, 0);
    const int ntrip = k * (k - 1) * (k - 2) / 6;
    const int npair = with_q ? k * (k - 1) / 2 : 0;
    const int nqg = with_q && S.link[k - 1] == GHOST ? 2 * (k - 1) : 0;
    const int ncand = ntrip + npair + nqg;
    bool done = false, fan = false;
    // The common case first (a short move keeps the star's shape): with q
    // strictly left of every link edge and no link vertex inside the
    // perturbed circle of any fan triangle (q_s, q_s+1, q), the fan is the
    // whole retriangulation.  Its k triangles are Delaunay among the link
    // vertices and q and tile the polygon; any other triple that passed
    // every test would lie outside the polygon, in a pocket behind a
    // concave chain, and a pocket triangle is clockwise in link order, so
    // the search below would find exactly the fan.  The fan's records are
    // then built straight from the link (below), in the order that search
    // lists them: pairs (i < j) by j, then i, so t_s = (s, s+1, q) comes
    // at s for s < k-2, then t_k-1 = (k-1, 0, q), then t_k-2.  Same
    // predicates, same argument order.
    if (with_q && !ballot(lane < k && S.link[lane] == GHOST)) {
        const int sh = k <= 8 ? 3 : 4;  // lanes per link edge (k <= EMK - 1 here)
        bool bad = false, side = false;
        for (int x = lane; x < (k << sh); x += WAVE) {
            const int s = x >> sh, m = x & ((1 << sh) - 1);
            const int s1 = s + 1 < k ? s + 1 : 0;
            if (m >= k || m == s1) continue;
            const int2 a = S.lxy[s], b = S.lxy[s1];
            if (m == s) side = side || !(orient(a, b, q) > 0);
            else bad = bad || incircle_star(a, S.link[s], b, S.link[s1], q, qv, S.lxy[m], S.link[m]) >= 0;
        }
        const bool kernel = !ballot(side);  // q strictly left of every link edge
        done = fan = kernel && !ballot(bad);
        // Not the fan but q in the polygon's kernel (most of the rest): the
        // fan is still a triangulation of the polygon, and Lawson flips of
        // its edges that fail the perturbed test reach the triangulation
        // whose inner edges all pass it.  No triangle outside the region is
        // destroyed, so that is the part of DT*(S - p + q) inside the
        // region: the triangles the search would find.  Each flip lowers
        // the lifted surface, so the flips end; they are capped all the
        // same, and a capped run leaves the work to the search.  The
        // triangles are then listed in the search's order (by candidate
        // index), so everything after this point is the same either way.
        if (kernel && !fan) done = lawson_from_fan(S, k, qv, q, ntrip);
    }
    // Two phases: the candidates that pass orientation (and keep q out)
    // are compacted into S.emat, their verdicts in S.cav_ent (both idle
    // here), and then tested against every link vertex, one (candidate,
    // vertex) pair per lane.  Large links first test each candidate against
    // the link neighbours of its vertices, which reject most non-Delaunay
    // triples.  Too many survivors: every lane tests its candidate against
    // every vertex.
    if (!done) {
        int nsurv = 0;
        for (int t0 = 0; t0 < ncand; t0 += WAVE) {
            TriCand c = tri_cand(S, k, t0 + lane, ntrip, npair, ncand, qv, q, with_q);
            if (k >= SPLIT_K) {
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const int base = f < 2 ? c.i : (f < 4 ? c.j : c.l);
                    if (base == k) continue;  // q has no link neighbours
                    const int m = (base + ((f & 1) ? 1 : k - 1)) % k;
                    if (c.ok && cand_killed_by(c, m, S.link[m], S.lxy[m])) c.ok = false;
                }
            }
            const uint64_t sm = ballot(c.ok);
            if (c.ok && nsurv + lanes_below(sm) < SURV_MAX) S.emat[nsurv + lanes_below(sm)] = pack3(c.i, c.j, c.l);
            nsurv += __popcll(sm);
        }
        if (nsurv <= SURV_MAX) {
            for (int x = lane; x < nsurv; x += WAVE) S.cav_ent[x] = 1;
            wsync();
            for (int x = lane; x < nsurv * k; x += WAVE) {
                const int si = x / k, m = x - si * k;
                const int key = S.emat[si];
                const TriCand c = tri_cand_of(S, k, key >> 16, (key >> 8) & 255, key & 255, qv, q);
                if (cand_killed_by(c, m, S.link[m], S.lxy[m])) S.cav_ent[si] = 0;
            }
            wsync();
            int nh = 0;
            for (int x0 = 0; x0 < nsurv; x0 += WAVE) {
                const int x = x0 + lane;
                const bool keep = x < nsurv && S.cav_ent[x];
                const uint64_t km = ballot(keep);
                if (keep && nh + lanes_below(km) < KMAX) S.hole_key[nh + lanes_below(km)] = S.emat[x];
                nh += __popcll(km);
            }
            if (lane == 0) S.nhole = nh;
            done = true;
        }
    }
    if (!done) {
        int nh = 0;
        for (int t0 = 0; t0 < ncand; t0 += WAVE) {
            TriCand c = tri_cand(S, k, t0 + lane, ntrip, npair, ncand, qv, q, with_q);
            // link vertex m's id and position sit in lane m's registers
            for (int m = 0; m < k; ++m) {
                if (!ballot(c.ok)) break;
                const int vm = __builtin_amdgcn_readlane(lv, m);
                const int2 pm = make_int2(__builtin_amdgcn_readlane(lp.x, m), __builtin_amdgcn_readlane(lp.y, m));
                if (c.ok && cand_killed_by(c, m, vm, pm)) c.ok = false;
            }
            const uint64_t km = ballot(c.ok);
            if (c.ok && nh + lanes_below(km) < KMAX) S.hole_key[nh + lanes_below(km)] = pack3(c.i, c.j, c.l);
            nh += __popcll(km);
        }
        if (lane == 0) S.nhole = nh;
    }
    wsync();
    // the new triangles in the order the candidates were found (the same on
    // every run: compaction by ballot and prefix count)
    const int nh = fan ? k : S.nhole;
    if (nh != (with_q ? k : k - 2)) return ST_INTERNAL;
    const int nv = with_q ? k + 1 : k;  // vertices of the polygon (+ q)
    const bool small = nv <= EMK;
    if (small && !fan)
        for (int x = lane; x < nv * EMK; x += WAVE) S.emat[x] = -1;
    wsync();
    if (small && !fan && lane < nh) {
        const int hk = S.hole_key[lane];
        const int d0 = hk >> 16, d1 = (hk >> 8) & 255, d2 = hk & 255;
        S.emat[d1 * EMK + d2] = lane * 4 + 0;
        S.emat[d2 * EMK + d0] = lane * 4 + 1;
        S.emat[d0 * EMK + d1] = lane * 4 + 2;
    }
    wsync();
    // adjacency of the new triangles
    int herr = 0;
    Tri h;
    bool has_q = false;
    if (fan) {
        // fan triangle t_s = (s, s+1, q) at s (s < k-2), k-2 (s = k-1) or
        // k-1 (s = k-2): its edge 0, (s+1, q), borders t_s+1 at that one's
        // edge 1; its edge 1, (q, s), borders t_s-1 at that one's edge 0;
        // its edge 2 is link edge s
        if (lane < nh) {
            const int s = lane < k - 2 ? lane : (lane == k - 2 ? k - 1 : k - 2);
            const int s1 = s + 1 < k ? s + 1 : 0, sp = s > 0 ? s - 1 : k - 1;
            const int a1 = s1 < k - 2 ? s1 : (s1 == k - 1 ? k - 2 : k - 1);
            const int a2 = sp < k - 2 ? sp : (sp == k - 1 ? k - 2 : k - 1);
            const int2 p0 = S.lxy[s], p1 = S.lxy[s1];
            h.v = make_int4(S.link[s], S.link[s1], qv, 0);
            h.n = make_int4(S.star_slot[a1] * 4 + 1, S.star_slot[a2] * 4 + 0, S.outref[s], 0);
            h.c01 = make_int4(p0.x, p0.y, p1.x, p1.y);
            h.c2 = make_int4(q.x, q.y, 0, 0);
            S.edge_tri[s] = lane * 4 + 2;
            has_q = true;
        }
    } else if (lane < nh) {
        const int hk = S.hole_key[lane];
        const int cs[3] = {hk >> 16, (hk >> 8) & 255, hk & 255};
        const TriCand c = tri_cand_of(S, k, cs[0], cs[1], cs[2], qv, q);
        const int2 c0 = c.pi, c1 = c.pj, c2 = c.pl;
        const int v2 = c.vl;
        has_q = cs[0] == k || cs[1] == k || cs[2] == k;
        h.v = make_int4(c.vi, c.vj, v2, 0);
        h.n = make_int4(0, 0, 0, 0);
        h.c01 = make_int4(c0.x, c0.y, c1.x, c1.y);
        h.c2 = v2 != GHOST ? make_int4(c2.x, c2.y, 0, 0) : make_int4(0, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int u = cs[(e + 1) % 3], w = cs[(e + 2) % 3];
            int nref;
            if (u < k && w < k && w == (u + 1) % k) {  // link edge u: the triangle outside it
                nref = S.outref[u];
                S.edge_tri[u] = lane * 4 + e;
            } else if (small) {  // inner edge: the new triangle with edge (w, u)
                nref = S.emat[w * EMK + u];
                if (nref < 0) herr = 1;
                else nref = S.star_slot[nref >> 2] * 4 + (nref & 3);
            } else {
                nref = -1;
#pragma unroll 8
                for (int m = 0; m < nh; ++m) {
                    const int mk = S.hole_key[m];
                    const int d0 = mk >> 16, d1 = (mk >> 8) & 255, d2 = mk & 255;
                    // edge f of triangle m is (d[f+1], d[f+2])
                    const int f = (d1 == w && d2 == u) ? 0 : (d2 == w && d0 == u) ? 1 : (d0 == w && d1 == u) ? 2 : -1;
                    nref = (m != lane && f >= 0) ? m * 4 + f : nref;
                }
                if (nref < 0) herr = 1;
                else nref = S.star_slot[nref >> 2] * 4 + (nref & 3);
            }
            vset(h.n, e, nref);
        }
    }
    if (ballot(herr)) return ST_INTERNAL;
    wsync();
    if (!fan && ballot(lane < k && S.edge_tri[lane] < 0)) return ST_INTERNAL;
    if (with_q && !ballot(has_q)) return ST_INTERNAL;
    if (direct) {
        // every check passed: the region's new records, the outside
        // neighbours' links into it and the incident triangles go straight
        // to memory (the move ends here; its table holds only records read)
        if (lane < nh) B.tri[S.star_slot[lane]] = h;
        if (lane < k) {
            const int et = S.edge_tri[lane];
            const int hs = S.star_slot[et >> 2];
            const int o = S.outref[lane];
            reinterpret_cast<int*>(&B.tri[o >> 2].n)[o & 3] = hs * 4 + (et & 3);
            const int v = S.link[lane];
            if (v != GHOST) B.vtri[v] = hs;
        }
        const uint64_t mq = ballot(has_q);
        if (lane == first_lane(mq)) B.vtri[qv] = S.star_slot[lane];
        if (lane == 0 && st) {
            st->tri_touched += nh;
            st->alg_bytes += 64LL * nh + 4LL * (k + 1);
        }
        return ST_OK;
    }
    // the new triangles into the table, the outside neighbours patched there,
    // incident triangles of the link vertices (and q) queued
    bool mine;
    const int he = tclaim(S, lane < nh, S.star_slot[lane < nh ? lane : 0], &mine);
    tnote(S, mine, he, used);
    if (ballot(lane < nh && he < 0)) return ST_CAPACITY;
    if (lane < nh) {
        S.trec[he] = h;
        S.tflag[he] = F_DIRTY;
        S.hole_ent[lane] = he;
    }
    wsync();
    if (lane < k) {
        const int et = S.edge_tri[lane];
        const int hs = S.star_slot[et >> 2];
        const int o = S.outref[lane];
        const int oe = S.out_ent[lane];
        reinterpret_cast<int*>(&S.trec[oe].n)[o & 3] = hs * 4 + (et & 3);
        S.tflag[oe] = F_DIRTY;
        S.vt_v[*nvt + lane] = S.link[lane];
        S.vt_s[*nvt + lane] = hs;
    }
    *nvt += k;
    if (with_q) {
        const uint64_t mq = ballot(has_q);
        if (!mq) return ST_INTERNAL;
        if (lane == 0) {
            S.vt_v[*nvt] = qv;
            S.vt_s[*nvt] = S.star_slot[first_lane(mq)];
        }
        *nvt += 1;
    }
    wsync();
    if (lane == 0 && st) {
        st->tri_touched += nh;
        // new records written, incident-triangle updates
        st->alg_bytes += 64LL * nh + 4LL * (k + (with_q ? 1 : 0));
    }
    return ST_OK;
}

// ---------------------------------------------------------------- move and flip
// The move-and-flip repair, the other way to update a triangulation of
// points moved in discrete steps beside delete + insert (De Berg et al.;
// Sec. II).  When the new place q lies strictly inside the kernel of p's
// star -- p not on the hull, every star triangle (p, q_s, q_s+1) still
// counter-clockwise with p at q -- p moves there in place: the
// triangulation stays valid and the hull is unchanged.  Lawson flips then
// restore the Delaunay property: an edge whose opposite vertex lies inside
// the perturbed circle of a triangle is flipped, and the four edges around
// the flipped pair are checked again.  Only edges whose two triangles hold
// p can fail at first: the spokes and the link edges.  Flipping ends (each
// flip lowers the lifted surface) at a triangulation every edge of which is
// locally Delaunay under the perturbed test, i.e. DT*, the result of delete
// + insert.  All of it happens in the write-back table; commit() writes it.
// Returns 1 when taken, 0 when q is not inside the kernel (nothing read or
// changed), or ST_CAPACITY (too many flips, or the table is full; memory
// unchanged).
constexpr int FLIP_MAX = (VTMAX - 1) / 2;  // flips one move may do: two incident-triangle updates each
template <class WL>
__device__ __forceinline__ int move_and_flip(const BlockView& B, WL& S, int k, int p, int2 q, int* used,
                                             int* nvt, int* nflips) {
    const int lane = lane_id();
    *nflips = 0;
    *nvt = 0;
    bool ok = true;
    if (lane < k) {
        const int a = S.link[lane], b = S.link[(lane + 1) % k];
        ok = a != GHOST && b != GHOST && orient(S.lxy[lane], S.lxy[(lane + 1) % k], q) > 0;
    }
    if (k < 3 || ballot(!ok)) return 0;
    // the star triangles into the table with p's position copies at q; the
    // queue of edges to check (4 * slot + index of the opposite vertex): the
    // link edge opposite p and the spoke (q_s+1, p) opposite q_s of each
    const int se = tget(B, S, lane < k, S.star_slot[lane < k ? lane : 0], used);
    if (ballot(lane < k && se < 0)) return ST_CAPACITY;
    int* queue = S.cav_ent;  // a ring of CMAX edges (the cavity arrays are unused here)
    if (lane < k) {
        Tri& t = S.trec[se];
        const int pi = t.v.x == p ? 0 : (t.v.y == p ? 1 : 2);
        cset(t, pi, q);
        S.tflag[se] |= F_DIRTY;
        const int ss = S.star_slot[lane];
        queue[2 * lane] = 4 * ss + pi;
        queue[2 * lane + 1] = 4 * ss + (pi + 1) % 3;
    }
    wsync();
    int head = 0, tail = 2 * k;
    while (head < tail) {
        const int ref = queue[head % CMAX];
        ++head;
        const int ts = ref >> 2, te = ref & 3;
        if (bad_slot(B, ts)) return ST_INTERNAL;
        const int et = tget(B, S, true, ts, used);
        if (et < 0) return ST_CAPACITY;
        const Tri t = S.trec[et];
        if (t.v.z == GHOST) continue;
        const int nref = vget(t.n, te);
        const int us = nref >> 2, ue = nref & 3;
        if (bad_slot(B, us)) return ST_INTERNAL;
        const int eu = tget(B, S, true, us, used);
        if (eu < 0) return ST_CAPACITY;
        const Tri u = S.trec[eu];
        if (u.v.z == GHOST) continue;  // a hull edge: never flipped
        // t = (A, B, C) from te, u = (D, C, B) from ue; the shared edge is BC
        const int iA = te, iB = (te + 1) % 3, iC = (te + 2) % 3;
        const int vA = vget(t.v, iA), vB = vget(t.v, iB), vC = vget(t.v, iC), vD = vget(u.v, ue);
        const int2 pA = cget(t, iA), pB = cget(t, iB), pC = cget(t, iC), pD = cget(u, ue);
        if (incircle_star(pA, vA, pB, vB, pC, vC, pD, vD) <= 0) continue;
        if (++*nflips > FLIP_MAX || tail - head + 4 > CMAX) return ST_CAPACITY;
        const int rAB = vget(t.n, iC), rCA = vget(t.n, iB);
        const int rBD = vget(u.n, (ue + 1) % 3), rDC = vget(u.n, (ue + 2) % 3);
        // t becomes (A, B, D), u becomes (A, D, C); their shared edge AD
        if (lane == 0) {
            Tri nt, nu;
            nt.v = make_int4(vA, vB, vD, 0);
            nt.n = make_int4(rBD, 4 * us + 2, rAB, 0);
            nt.c01 = make_int4(pA.x, pA.y, pB.x, pB.y);
            nt.c2 = make_int4(pD.x, pD.y, 0, 0);
            nu.v = make_int4(vA, vD, vC, 0);
            nu.n = make_int4(rDC, rCA, 4 * ts + 1, 0);
            nu.c01 = make_int4(pA.x, pA.y, pD.x, pD.y);
            nu.c2 = make_int4(pC.x, pC.y, 0, 0);
            S.trec[et] = nt;
            S.trec[eu] = nu;
            S.tflag[et] |= F_DIRTY;
            S.tflag[eu] |= F_DIRTY;
            // B left u and C left t: their incident triangles are found again
            // at the end
            S.vt_v[*nvt] = vB;
            S.vt_v[*nvt + 1] = vC;
            queue[tail % CMAX] = 4 * ts + 0;      // BD
            queue[(tail + 1) % CMAX] = 4 * ts + 2;  // AB
            queue[(tail + 2) % CMAX] = 4 * us + 0;  // DC
            queue[(tail + 3) % CMAX] = 4 * us + 1;  // CA
        }
        *nvt += 2;
        tail += 4;
        wsync();
        // the four outside neighbours point into the new pair
        const int oref = lane == 0 ? rBD : (lane == 1 ? rAB : (lane == 2 ? rDC : rCA));
        const int oval = lane == 0 ? 4 * ts + 0 : (lane == 1 ? 4 * ts + 2 : (lane == 2 ? 4 * us + 0 : 4 * us + 1));
        if (ballot(lane < 4 && bad_slot(B, oref >> 2))) return ST_INTERNAL;
        const int eo = tget(B, S, lane < 4, oref >> 2, used);
        if (ballot(lane < 4 && eo < 0)) return ST_CAPACITY;
        if (lane < 4) {
            reinterpret_cast<int*>(&S.trec[eo].n)[oref & 3] = oval;
            S.tflag[eo] |= F_DIRTY;
        }
        wsync();
    }
    // an incident triangle for every vertex that lost one (the same answer
    // for a vertex listed twice): the first changed real record holding it
    for (int i = lane; i < *nvt; i += WAVE) {
        const int v = S.vt_v[i];
        int found = -1;
        for (int u2 = 0; u2 < *used && found < 0; ++u2) {
            const int h = S.tused[u2];
            const Tri& r = S.trec[h];
            if ((S.tflag[h] & F_DIRTY) && r.v.z != GHOST && (r.v.x == v || r.v.y == v || r.v.z == v)) found = S.tkey[h];
        }
        S.vt_s[i] = found;
        if (found < 0) S.vt_v[i] = GHOST;  // cannot happen: v is in a changed triangle
    }
    wsync();
    return 1;
}

}  // namespace kdt
