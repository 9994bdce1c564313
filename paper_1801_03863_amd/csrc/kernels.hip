// kernels.hip -- fused stream-and-collide kernels of MinxEnt-LBM for gfx950.
//
// One thread owns one node per row it visits.  Each time step it pulls the
// nine (or three) populations that stream into its node from the previous
// post-collision state (Sec. II.A: f_a(x + v_a, t+1) = post-collision f_a(x, t),
// read here as f_a(x) <- f*_a(x - v_a)), applies the node's role -- the
// collision rule on fluid nodes, full-way bounce-back on walls, the
// equilibrium of the lid's density and velocity on the lid (Sec. IV.E) -- and
// writes its nine post-collision populations to the other buffer.
//
// Layout: structure of arrays, one plane per direction of ny rows of nx
// values, x fastest, each row starting a 128-byte line (rows `pitch`
// elements apart, nx rounded up to whole lines; the padding is never read),
// so every plane read is a unit-stride row shifted by at most one element and
// every write is aligned and unit-stride.  Planes follow each other at a
// stride of ny * pitch rounded up to 64 elements, plus, for a
// large single lattice, a tuned pad that is a multiple of 256 bytes, so every
// plane starts 256-byte aligned.  The single-step kernels read and write
// every population exactly once per step; they are bound by HBM bandwidth in
// the FP64, FP32 and FP32-storage/FP64-compute forms, and by VALU issue (the
// logarithms, reciprocals and 4 x 4 solve of the Newton step) when the
// populations are FP16 deviations.  The multi-step kernels further down (two
// D2Q9 steps, or up to 256 D1Q3 steps, per launch) keep the steps between in
// LDS and read and write every population once per launch; HBM then no
// longer bounds them.
//
// Slots of boundary nodes whose upstream node lies outside the lattice read a
// clamped (in-bounds) location; their values are bounced outward and never
// reach a fluid node.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "collide.hpp"
#include "kernels.hpp"

namespace lbm {

// --------------------------------------------------------------------------
// Storage forms
// --------------------------------------------------------------------------

template <int ST> struct Form;
template <> struct Form<ST_F64> { using T = double; using C = double; };
template <> struct Form<ST_F32N64> { using T = float; using C = double; };
template <> struct Form<ST_F32> { using T = float; using C = float; };
template <> struct Form<ST_F16DEV> { using T = _Float16; using C = float; };

template <int ST>
__device__ __forceinline__ typename Form<ST>::C load(const typename Form<ST>::T *p, typename Form<ST>::C ref,
                                                     float iscale)
{
    using C = typename Form<ST>::C;
    if constexpr (ST == ST_F16DEV) return ref + C(*p) * iscale;
    else return C(*p);
}

// Raw load of one stored population; NT marks it non-temporal (streamed:
// every population is read once per step).
template <class T, bool NT>
__device__ __forceinline__ T ldraw(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// FP16 deviation of v from ref, scaled by the power of two `scale`: the
// fused form v*scale - ref*scale rounds once, straight to binary16 (one
// mixed-precision fma); ref*scale is exact and uniform across the wave.
__device__ __forceinline__ _Float16 enc16(float v, float ref, float scale)
{
    return (_Float16)__builtin_fmaf(v, scale, -(ref * scale));
}

// A population in its storage form (rounded to the storage type, or the
// scaled FP16 deviation).
template <int ST>
__device__ __forceinline__ typename Form<ST>::T to_storage(typename Form<ST>::C v, typename Form<ST>::C ref,
                                                           float scale)
{
    using T = typename Form<ST>::T;
    if constexpr (ST == ST_F16DEV) return enc16(v, ref, scale);
    else return T(v);
}

template <int ST, bool NT = false>
__device__ __forceinline__ void store(typename Form<ST>::T *p, typename Form<ST>::C v, typename Form<ST>::C ref,
                                      float scale)
{
    const typename Form<ST>::T t = to_storage<ST>(v, ref, scale);
    if constexpr (NT) __builtin_nontemporal_store(t, p);
    else *p = t;
}

template <class C>
__device__ __forceinline__ void ref9(C rho0, C (&r)[9])
{
    r[0] = W9<C>::rest * rho0;
#pragma unroll
    for (int a = 1; a < 5; ++a) r[a] = W9<C>::axis * rho0;
#pragma unroll
    for (int a = 5; a < 9; ++a) r[a] = W9<C>::diag * rho0;
}

// D2Q9 direction table (pull offsets are the negated velocities).
__device__ __forceinline__ int cx9(int a) { return (a == 1 || a == 5 || a == 8) ? 1 : (a == 3 || a == 6 || a == 7) ? -1 : 0; }
__device__ __forceinline__ int cy9(int a) { return (a == 2 || a == 5 || a == 6) ? 1 : (a == 4 || a == 7 || a == 8) ? -1 : 0; }

// Neighbour rows and columns of (x, y): wrapped on periodic axes, clamped
// otherwise.
struct Nb {
    int xm, xp, ym, yp;
};

__device__ __forceinline__ Nb neighbours(int x, int y, int nx, int ny, int bc)
{
    const bool xw = bc == BC_PERIODIC;
    const bool yw = bc == BC_PERIODIC || bc == BC_TUBE;
    Nb n;
    n.xm = x > 0 ? x - 1 : (xw ? nx - 1 : 0);
    n.xp = x < nx - 1 ? x + 1 : (xw ? 0 : nx - 1);
    n.ym = y > 0 ? y - 1 : (yw ? ny - 1 : 0);
    n.yp = y < ny - 1 ? y + 1 : (yw ? 0 : ny - 1);
    return n;
}

enum Role { R_FLUID = 0, R_WALL = 1, R_LID = 2 };

__device__ __forceinline__ int role9(int x, int y, int nx, int ny, int bc)
{
    switch (bc) {
    case BC_CAVITY:
        if (y == ny - 1) return R_LID;
        return (x == 0 || x == nx - 1 || y == 0) ? R_WALL : R_FLUID;
    case BC_BOX:
        return (x == 0 || x == nx - 1 || y == 0 || y == ny - 1) ? R_WALL : R_FLUID;
    case BC_TUBE:
        return (x == 0 || x == nx - 1) ? R_WALL : R_FLUID;
    default:
        return R_FLUID;
    }
}

// Pull the nine raw populations of node (x, y) given the column byte offsets
// of x and of its two neighbours.  Row bases are uniform when the rows are
// (scalar registers), so the loads take the scalar-base + 32-bit
// vector-offset form.
// NL selects non-temporal loads: 0 none, 1 every plane, 2 only the three
// planes without a horizontal shift (rest, N, S), whose cache lines no other
// tile reads; the six x-shifted planes then keep regular loads, so the line a
// tile shares with its horizontal neighbour can still be found in cache.
template <int ST, int NL = 0>
__device__ __forceinline__ void pull9_cols(const typename Form<ST>::T *__restrict__ s, int64_t P, int y, int ym,
                                           int yp, int pitch, uint32_t cc, uint32_t cm, uint32_t cp,
                                           typename Form<ST>::T (&r)[9])
{
    using T = typename Form<ST>::T;
    constexpr bool A = NL == 1, U = NL != 0;
    const int64_t PB = P * (int64_t)sizeof(T);
    const int64_t RB = (int64_t)pitch * (int64_t)sizeof(T);
    const char *bc_ = (const char *)s + (int64_t)y * RB;
    const char *bm_ = (const char *)s + (int64_t)ym * RB;
    const char *bp_ = (const char *)s + (int64_t)yp * RB;
    r[0] = ldraw<T, U>((const T *)(bc_ + cc));
    r[1] = ldraw<T, A>((const T *)((bc_ + PB) + cm));
    r[2] = ldraw<T, U>((const T *)((bm_ + 2 * PB) + cc));
    r[3] = ldraw<T, A>((const T *)((bc_ + 3 * PB) + cp));
    r[4] = ldraw<T, U>((const T *)((bp_ + 4 * PB) + cc));
    r[5] = ldraw<T, A>((const T *)((bm_ + 5 * PB) + cm));
    r[6] = ldraw<T, A>((const T *)((bm_ + 6 * PB) + cp));
    r[7] = ldraw<T, A>((const T *)((bp_ + 7 * PB) + cp));
    r[8] = ldraw<T, A>((const T *)((bp_ + 8 * PB) + cm));
}

// Non-temporal load mode of a launch-shape bit mask NT: bit 0 every plane,
// bit 2 the unshifted planes only (bit 1 is the stores; bit 3, in the
// single-lattice D2Q9 kernel, raises the wave's issue priority while it
// issues its loads).
constexpr int nl_mode(int nt) { return (nt & 1) ? 1 : ((nt & 4) ? 2 : 0); }

// Column byte offsets of a node's own column and its two neighbours.  In a
// tile that touches neither side of the lattice the neighbours are x -+ 1
// for every boundary kind, so only the two edge tiles of a row (a uniform
// test) evaluate the wrap/clamp rule.
struct Cols {
    uint32_t cc, cm, cp;
};

__device__ __forceinline__ Cols columns(int xs, bool edge_tile, int nx, int bc, uint32_t E)
{
    Cols c;
    c.cc = (uint32_t)xs * E;
    c.cm = c.cc - E;
    c.cp = c.cc + E;
    if (edge_tile) {
        const Nb n = neighbours(xs, 0, nx, 1, bc);
        c.cm = (uint32_t)n.xm * E;
        c.cp = (uint32_t)n.xp * E;
    }
    return c;
}

// Pull the nine raw stored populations that stream into node (x, y) (rows
// `pitch` elements apart).
template <int ST, int NL = 0>
__device__ __forceinline__ void pull9_raw(const typename Form<ST>::T *__restrict__ s, int64_t P, int x, int y,
                                          int pitch, const Nb &n, typename Form<ST>::T (&r)[9])
{
    const uint32_t E = sizeof(typename Form<ST>::T);
    pull9_cols<ST, NL>(s, P, y, n.ym, n.yp, pitch, (uint32_t)x * E, (uint32_t)n.xm * E, (uint32_t)n.xp * E, r);
}

// Pull and widen the nine populations that stream into node (x, y) (NL as
// for pull9_cols).
template <int ST, int NL = 0>
__device__ __forceinline__ void pull9(const typename Form<ST>::T *__restrict__ s, int64_t P, int x, int y,
                                      int pitch, const Nb &n, const typename Form<ST>::C (&ref)[9], float iscale,
                                      typename Form<ST>::C (&f)[9])
{
    typename Form<ST>::T r[9];
    pull9_raw<ST, NL>(s, P, x, y, pitch, n, r);
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = load<ST>(&r[q], ref[q], iscale);
}

// Write the nine populations of node (x, y), already in their storage form,
// of a row that is uniform across the wave.  The row base is read from the
// first lane so that it lives in scalar registers, and each store takes the
// scalar-base + 32-bit vector-offset form of a global store.
template <int ST, bool NT = false>
__device__ __forceinline__ void push9_xy_st(typename Form<ST>::T *__restrict__ d, int64_t P, int x, int y,
                                            int pitch, const typename Form<ST>::T (&v)[9])
{
    using T = typename Form<ST>::T;
    using GT = __attribute__((address_space(1))) T;
    const uint64_t a = (uint64_t)d + (uint64_t)((int64_t)y * pitch * (int64_t)sizeof(T));
    // readfirstlane returns a signed int: each half goes through uint32_t so
    // that widening zero-extends it.
    const uint32_t ahi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
    const uint32_t alo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    const uint64_t b = ((uint64_t)ahi << 32) | (uint64_t)alo;
    const uint64_t PB = (uint64_t)P * sizeof(T);
    // The empty asm statements keep the lane offset and each plane base
    // opaque, so the compiler can neither share a widened offset with the
    // loads nor fold it into a 64-bit vector address.
    uint32_t o = (uint32_t)x * (uint32_t)sizeof(T);
    asm volatile("" : "+v"(o));
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        uint64_t bq = b + q * PB;
        asm volatile("" : "+s"(bq));
        GT *p = (GT *)(bq + (uint64_t)o);
        if constexpr (NT) __builtin_nontemporal_store(v[q], p);
        else *p = v[q];
    }
}

// The same from populations in compute precision.
template <int ST, bool NT = false>
__device__ __forceinline__ void push9_xy(typename Form<ST>::T *__restrict__ d, int64_t P, int x, int y,
                                         int pitch, const typename Form<ST>::C (&f)[9],
                                         const typename Form<ST>::C (&ref)[9], float scale)
{
    typename Form<ST>::T v[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) v[q] = to_storage<ST>(f[q], ref[q], scale);
    push9_xy_st<ST, NT>(d, P, x, y, pitch, v);
}

// Address of a block-uniform pointer, read from the first lane so that it
// lives in scalar registers (each half through uint32_t: readfirstlane
// returns a signed int, and widening must zero-extend it).
__device__ __forceinline__ uint64_t uniform_addr(const void *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

// Batched D2Q9: pull the nine raw populations of a node of one instance,
// whose planes start at the block-uniform address s (stride P elements),
// from byte offsets of rows (rc own, rm below, rp above) and columns (cc
// own, cm left, cp right).  An instance holds fewer than 2^22 nodes and
// pads each row by fewer than 64 elements, so its plane spans fewer than
// 2^28 elements (2^31 bytes) and every offset fits 32 bits: each load takes
// the scalar-base + 32-bit vector-offset form.  NL as for pull9_cols.
template <int ST, int NL>
__device__ __forceinline__ void pull9_inst(uint64_t s, int64_t P, uint32_t rc, uint32_t rm, uint32_t rp,
                                           uint32_t cc, uint32_t cm, uint32_t cp, typename Form<ST>::T (&r)[9])
{
    using T = typename Form<ST>::T;
    using GT = const __attribute__((address_space(1))) T;
    constexpr bool A = NL == 1, U = NL != 0;
    constexpr bool nt[9] = {U, A, U, A, U, A, A, A, A};
    const uint32_t o[9] = {rc + cc, rc + cm, rm + cc, rc + cp, rp + cc, rm + cm, rm + cp, rp + cp, rp + cm};
    const uint64_t PB = (uint64_t)P * sizeof(T);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        uint64_t bq = s + q * PB;
        asm volatile("" : "+s"(bq));
        uint32_t oq = o[q];
        asm volatile("" : "+v"(oq));
        GT *p = (GT *)(bq + (uint64_t)oq);
        if (nt[q]) r[q] = __builtin_nontemporal_load(p);
        else r[q] = *p;
    }
}

// Pull of a row that is uniform across the block (the two-step kernel's
// window rows): rows y (own), ym (below), yp (above), columns as byte
// offsets cc, cm, cp.  Each row and plane base lives in scalar registers and
// each load takes the scalar-base + 32-bit vector-offset form, so no lane
// forms a 64-bit address.  NL as for pull9_cols.
template <int ST, int NL>
__device__ __forceinline__ void pull9_row_u(const typename Form<ST>::T *__restrict__ s, int64_t P, int y, int ym,
                                            int yp, int pitch, uint32_t cc, uint32_t cm, uint32_t cp,
                                            typename Form<ST>::T (&r)[9])
{
    using T = typename Form<ST>::T;
    using GT = const __attribute__((address_space(1))) T;
    constexpr bool A = NL == 1, U = NL != 0;
    constexpr bool nt[9] = {U, A, U, A, U, A, A, A, A};
    constexpr int row[9] = {0, 0, 1, 0, 2, 1, 1, 2, 2};  // own, below, above
    constexpr int col[9] = {0, 1, 0, 2, 0, 1, 2, 2, 1};  // own, left, right
    const uint64_t s0 = uniform_addr(s);
    const uint64_t RB = (uint64_t)pitch * sizeof(T), PB = (uint64_t)P * sizeof(T);
    const uint64_t rb[3] = {s0 + (uint64_t)y * RB, s0 + (uint64_t)ym * RB, s0 + (uint64_t)yp * RB};
    uint32_t co[3] = {cc, cm, cp};
    asm volatile("" : "+v"(co[0]), "+v"(co[1]), "+v"(co[2]));
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        uint64_t bq = rb[row[q]] + q * PB;
        asm volatile("" : "+s"(bq));
        GT *p = (GT *)(bq + (uint64_t)co[col[q]]);
        if (nt[q]) r[q] = __builtin_nontemporal_load(p);
        else r[q] = *p;
    }
}

// Batched D2Q9: write the nine populations of the node at byte offset o of
// the instance whose planes start at the block-uniform address d.
template <int ST, bool NT = false>
__device__ __forceinline__ void push9_inst(uint64_t d, int64_t P, uint32_t o, const typename Form<ST>::C (&f)[9],
                                           const typename Form<ST>::C (&ref)[9], float scale)
{
    using T = typename Form<ST>::T;
    using GT = __attribute__((address_space(1))) T;
    const uint64_t PB = (uint64_t)P * sizeof(T);
    asm volatile("" : "+v"(o));
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        uint64_t bq = d + q * PB;
        asm volatile("" : "+s"(bq));
        GT *p = (GT *)(bq + (uint64_t)o);
        T t;
        if constexpr (ST == ST_F16DEV) t = enc16(f[q], ref[q], scale);
        else t = T(f[q]);
        if constexpr (NT) __builtin_nontemporal_store(t, p);
        else *p = t;
    }
}

// Write the nine post-collision populations of node index i.
template <int ST, bool NT = false>
__device__ __forceinline__ void push9(typename Form<ST>::T *__restrict__ d, int64_t P, int i,
                                      const typename Form<ST>::C (&f)[9], const typename Form<ST>::C (&ref)[9],
                                      float scale)
{
    using T = typename Form<ST>::T;
    char *b = (char *)d;
    const int64_t PB = P * (int64_t)sizeof(T);
    const uint32_t o = (uint32_t)i * (uint32_t)sizeof(T);
#pragma unroll
    for (int q = 0; q < 9; ++q) store<ST, NT>((T *)(b + q * PB + o), f[q], ref[q], scale);
}

// Role collision of one D2Q9 node.  Returns bit 0 = unstable, bit 1 = guarded.
template <int ST, int CO>
__device__ __forceinline__ int node9(typename Form<ST>::C (&f)[9], int role, const Inst &in)
{
    using C = typename Form<ST>::C;
    if (role == R_LID) {
#pragma unroll
        for (int a = 0; a < 9; ++a) f[a] = C(in.lid[a]);
        return 0;
    }
    if constexpr (ST == ST_F16DEV && (CO == CO_MINXENT4 || CO == CO_MINXENT2)) {
        // FP16 deviations: the collision runs on the fluid lanes only, then
        // the wall lanes, whose f still holds the pulled populations, swap
        // them.  The same results as the order below; in this form the
        // compiler then keeps fewer values live across the collision (69
        // instead of 77 VGPRs in the tuned two-step shape, 7 waves per SIMD
        // instead of 6).  In the double-precision forms this order costs
        // registers instead.
        int r = 0;
        if (role != R_WALL) {
            bool ok = true;
            const bool g = collide_minxent<C, CO == CO_MINXENT2, true, false>(f, C(in.omega), C(in.omega2), ok);
            r = (g ? 2 : 0) | (ok ? 0 : 1);
        }
        if (role == R_WALL) {
            C t;
            t = f[1]; f[1] = f[3]; f[3] = t;
            t = f[2]; f[2] = f[4]; f[4] = t;
            t = f[5]; f[5] = f[7]; f[7] = t;
            t = f[6]; f[6] = f[8]; f[8] = t;
        }
        return r;
    }
    if (role == R_WALL) {
        C t;
        t = f[1]; f[1] = f[3]; f[3] = t;
        t = f[2]; f[2] = f[4]; f[4] = t;
        t = f[5]; f[5] = f[7]; f[7] = t;
        t = f[6]; f[6] = f[8]; f[8] = t;
        return 0;
    }
    // Stable iff every population is >= 0 and finite (Sec. IV.G): the
    // minimum catches negatives; inf and NaN are caught by the Newton
    // increments (MinxEnt) or by the sum (the other rules).
    if constexpr (CO == CO_MINXENT4 || CO == CO_MINXENT2) {
        bool ok = true;
        const bool g = collide_minxent<C, CO == CO_MINXENT2, ST == ST_F16DEV, ST == ST_F32N64>(f, C(in.omega), C(in.omega2), ok);
        return (g ? 2 : 0) | (ok ? 0 : 1);
    } else {
        if constexpr (CO == CO_SRT) {
            collide_srt<C>(f, C(in.omega));
        } else if constexpr (CO == CO_TRT) {
            collide_mrt<C>(f, C(in.omega), C(in.omega), C(in.omega2), C(in.omega));
        } else {
            collide_mrt<C>(f, C(1.64), C(1.54), C(in.omega2), C(in.omega));
        }
        C mn = f[0], sm = f[0];
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            mn = __builtin_fmin(mn, f[a]);
            sm += f[a];
        }
        const bool ok = mn >= C(0) && sm < C(__builtin_huge_valf());
        return ok ? 0 : 1;
    }
}

// Role collision of one node of a non-lid row that is uniform across the
// wave: only the two side-wall lanes diverge.
template <int ST, int CO>
__device__ __forceinline__ int node9_row(typename Form<ST>::C (&f)[9], int x, int y, int nx, int ny, int bc,
                                         const Inst &in)
{
    const bool wall_row = (bc == BC_CAVITY && y == 0) || (bc == BC_BOX && (y == 0 || y == ny - 1));
    const bool wall = wall_row || (bc != BC_PERIODIC && (x == 0 || x == nx - 1));
    return node9<ST, CO>(f, wall ? R_WALL : R_FLUID, in);
}

// The cavity's lid row (uniform across the wave): every node takes the lid
// equilibrium, which needs no loads.
template <int ST, bool NT = false>
__device__ __forceinline__ void push_lid(typename Form<ST>::T *__restrict__ d, int64_t P, int x, int y, int pitch,
                                         const Inst &in, const typename Form<ST>::C (&ref)[9], float scale)
{
    using C = typename Form<ST>::C;
    C f[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = C(in.lid[a]);
    push9_xy<ST, NT>(d, P, x, y, pitch, f, ref, scale);
}

// Wave-level status update: one atomic per wave and kind.
// Key of an unstable event: the step in the high word (saturating at 2^32 -
// 1), the node index (x + y nx within its instance) in the low word, so that
// the smallest key is the first step's smallest node.
__device__ __forceinline__ uint64_t event_key(int64_t step, int node)
{
    const uint64_t s = step < 0xffffffffll ? (uint64_t)step : 0xffffffffull;
    return (s << 32) | (uint32_t)node;
}

// Sentinel of a lane's unstable-node record: no unstable node.
constexpr int kNoNode = 0x7fffffff;

// bad_node: the smallest unstable node index of this lane in this launch, or
// kNoNode.  One atomic per wave and kind; the wave's smallest unstable node
// is found by a butterfly minimum only in waves that have one.
__device__ __forceinline__ void report(DevStatus *st, int bad_node, int guarded_in_wave, int64_t step,
                                       const int64_t *step_base)
{
    const unsigned long long m = __ballot(bad_node != kNoNode);
    if (m != 0ull) {
        int v = bad_node;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
        if (__lane_id() == 0) {
            const int64_t s = step + (step_base ? *step_base : 0);
            atomicOr(&st->flags, 1u);
            atomicMin((unsigned long long *)&st->first, (unsigned long long)event_key(s, v));
        }
    }
    if (guarded_in_wave != 0 && __lane_id() == 0) {
        atomicOr(&st->flags, 2u);
        atomicAdd((unsigned long long *)&st->guarded, (unsigned long long)guarded_in_wave);
    }
}

// Batched instances with a step limit: once the step index reaches the
// instance's `stop`, its launches carry the state over unchanged (the two
// buffers alternate for the whole batch).
__device__ __forceinline__ bool instance_stopped(const StepArgs &a, const Inst &in)
{
    return in.stop <= a.step + (a.step_base ? *a.step_base : 0);
}

template <class T>
__device__ __forceinline__ void carry_node(const T *__restrict__ s, T *__restrict__ d, int64_t P, int planes, int node)
{
    for (int q = 0; q < planes; ++q) d[q * P + node] = s[q * P + node];
}

// Map block b of a grid of nb blocks so that the blocks the hardware sends to
// one XCD (b, b+8, b+16, ...) cover a contiguous range of tiles.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, k = b & 7;
    return k * q + (k < r ? k : r) + (b >> 3);
}

// Tile (tx, ty) of this block.  The grid is (tiles_x, tiles_y), or one
// dimension of tiles_x * tiles_y blocks when tiles_y exceeds the grid's y
// limit.  In dispatch order (x fastest) the hardware deals blocks
// round-robin to the eight XCDs, each with its own L2; with the swizzle the
// linear block index is remapped so that each XCD works on a contiguous band
// of rows.
__device__ __forceinline__ void tile_of_block(int swizzle, int tiles_x, int &tx, int &ty)
{
    if (!swizzle && (int)gridDim.x == tiles_x) {
        tx = blockIdx.x;
        ty = blockIdx.y;
        return;
    }
    int b = blockIdx.y * gridDim.x + blockIdx.x;
    if (swizzle) b = xcd_remap(b, gridDim.x * gridDim.y);
    ty = b / tiles_x;
    tx = b - ty * tiles_x;
}

// --------------------------------------------------------------------------
// D2Q9, one lattice.  Block = BX x BY threads (BX a multiple of 64, so a wave
// never spans two rows); it covers BX columns and BY*RPT rows.
// --------------------------------------------------------------------------

// WPE > 0 asks the compiler for at least WPE waves per SIMD (a register
// budget of 512/WPE VGPRs), trading registers for occupancy.
template <int ST, int CO, int BX, int BY, int RPT, int NT = 0, int WPE = 0>
__global__ __launch_bounds__(BX *BY) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void k_d2q9(const typename Form<ST>::T *__restrict__ src, typename Form<ST>::T *__restrict__ dst, StepArgs a)
{
    using C = typename Form<ST>::C;
    // NT bit 3: the wave runs at raised issue priority until its loads are
    // in flight, so a new wave gets its memory requests out ahead of the
    // arithmetic of older waves.
    if constexpr ((NT & 8) != 0) __builtin_amdgcn_s_setprio(2);
    const Inst &in = a.one;
    const int nx = in.nx, ny = in.ny, pitch = in.pitch;
    const int64_t P = in.plane;
    int tx, ty;
    tile_of_block(a.xcd_swizzle, a.tiles_x, tx, ty);
    const int x = tx * BX + (int)threadIdx.x;
    const bool xin = x < nx;
    const int xs = xin ? x : nx - 1;
    const Cols cols = columns(xs, tx == 0 || tx == a.tiles_x - 1, nx, a.bc, sizeof(typename Form<ST>::T));
    C ref[9];
    ref9<C>(C(in.rho0), ref);
    int bad = kNoNode;
    int guarded = 0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        // A wave never spans two rows (BX is a multiple of 64), so y is
        // wave-uniform; saying so keeps all row logic in scalar registers.
        const int y = __builtin_amdgcn_readfirstlane((ty * RPT + k) * BY + (int)threadIdx.y);
        if (y >= ny) break;
        if (a.bc == BC_CAVITY && y == ny - 1) {
            if (xin) push_lid<ST, (NT & 2) != 0>(dst, P, x, y, pitch, in, ref, a.fp16_scale);
            continue;
        }
        const Nb n = neighbours(0, y, 1, ny, a.bc);  // rows only
        C f[9];
        {
            typename Form<ST>::T raw[9];
            pull9_cols<ST, nl_mode(NT)>(src, P, y, n.ym, n.yp, pitch, cols.cc, cols.cm, cols.cp, raw);
            if constexpr ((NT & 8) != 0) __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int q = 0; q < 9; ++q) f[q] = load<ST>(&raw[q], ref[q], a.fp16_iscale);
        }
        const int fl = node9_row<ST, CO>(f, xs, y, nx, ny, a.bc, in);
        if (xin && (fl & 1)) bad = min(bad, y * nx + x);
        guarded += __popcll(__ballot(xin && (fl & 2)));
        if (xin) push9_xy<ST, (NT & 2) != 0>(dst, P, x, y, pitch, f, ref, a.fp16_scale);
    }
    report(a.status, bad, guarded, a.step, a.step_base);
}

// Sixteen bytes of stored populations, moved as one vector access.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// LDS-staged form.  A block of BX threads covers BX columns of RY rows, one
// row at a time.  For each of the nine planes it stages the source row
// window [x0 - 1, x0 + BX] that the row's nodes pull from (row shifted by the
// plane's vertical velocity, columns by at most one) in LDS: the aligned
// BX-wide middle with 16-byte vector loads when every row start is 16-byte
// aligned (the row pitch a multiple of the vector width), element by element otherwise,
// and the two edge columns by single loads.  Window columns outside the
// lattice hold the wrap/clamp source of the edge nodes, so every node reads
// exactly what the direct forms read and results are bitwise equal.
template <int ST, int CO, int BX, int RY, int NT = 0>
__global__ __launch_bounds__(BX) void k_d2q9_stage(const typename Form<ST>::T *__restrict__ src,
                                                   typename Form<ST>::T *__restrict__ dst, StepArgs a)
{
    using C = typename Form<ST>::C;
    using T = typename Form<ST>::T;
    constexpr int V = 16 / sizeof(T);  // elements per vector
    // LDS row: [V-1] left edge, [V, V+BX) middle (16-byte aligned), [V+BX]
    // right edge; the row stride is a multiple of 16 bytes.
    constexpr int W = BX + 2 * V;
    __shared__ __align__(16) T win[9][W];
    const Inst &in = a.one;
    const int nx = in.nx, ny = in.ny, pitch = in.pitch;
    const int64_t P = in.plane;
    const bool xw = a.bc == BC_PERIODIC;
    int tx, ty;
    tile_of_block(a.xcd_swizzle, a.tiles_x, tx, ty);
    const int t = (int)threadIdx.x;
    const int x0 = tx * BX;
    const int x = x0 + t;
    const bool xin = x < nx;
    const int xs = xin ? x : nx - 1;
    const bool vec = (pitch % V) == 0;
    C ref[9];
    ref9<C>(C(in.rho0), ref);
    int bad = kNoNode;
    int guarded = 0;
    for (int r = 0; r < RY; ++r) {
        const int y = ty * RY + r;  // uniform across the block
        if (y >= ny) break;
        if (a.bc == BC_CAVITY && y == ny - 1) {
            if (xin) push_lid<ST, (NT & 2) != 0>(dst, P, x, y, pitch, in, ref, a.fp16_scale);
            continue;
        }
        const Nb n = neighbours(0, y, 1, ny, a.bc);  // rows only
        // Stage the nine windows.
        for (int i = t; i < 9 * (BX / V); i += BX) {
            const int q = i / (BX / V), k = i - q * (BX / V);
            const int vy = cy9(q);
            const int ys = vy > 0 ? n.ym : (vy < 0 ? n.yp : y);
            const T *row = src + (int64_t)q * P + (int64_t)ys * pitch;
            const int c0 = x0 + k * V;
            if (vec && c0 + V <= nx) {
                const u32x4 *p = (const u32x4 *)(row + c0);
                u32x4 w;
                if constexpr ((NT & 1) != 0) w = __builtin_nontemporal_load(p);
                else w = *p;
                *(u32x4 *)&win[q][V + k * V] = w;
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int c = c0 + e;
                    const int ce = c < nx ? c : ((c == nx && xw) ? 0 : nx - 1);
                    win[q][V + k * V + e] = ldraw<T, (NT & 1) != 0>(row + ce);
                }
            }
        }
        if (t < 18) {
            const int q = t >> 1;
            const int vy = cy9(q);
            const int ys = vy > 0 ? n.ym : (vy < 0 ? n.yp : y);
            const int c = (t & 1) ? x0 + BX : x0 - 1;
            const int ce = c < 0 ? (xw ? nx - 1 : 0) : (c >= nx ? ((c == nx && xw) ? 0 : nx - 1) : c);
            win[q][(t & 1) ? V + BX : V - 1] =
                ldraw<T, (NT & 1) != 0>(src + (int64_t)q * P + (int64_t)ys * pitch + ce);
        }
        __syncthreads();
        C f[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q] = load<ST>(&win[q][t + V - cx9(q)], ref[q], a.fp16_iscale);
        __syncthreads();  // the windows are restaged for the next row
        const int fl = node9_row<ST, CO>(f, xs, y, nx, ny, a.bc, in);
        if (xin && (fl & 1)) bad = min(bad, y * nx + x);
        guarded += __popcll(__ballot(xin && (fl & 2)));
        if (xin) push9_xy<ST, (NT & 2) != 0>(dst, P, x, y, pitch, f, ref, a.fp16_scale);
    }
    report(a.status, bad, guarded, a.step, a.step_base);
}

// Software-pipelined form: a block of BX threads walks RPT consecutive rows;
// each thread issues the raw loads of its next row before computing the
// current one, so nine loads per thread are always in flight while the VALU
// works.  Same per-node arithmetic as k_d2q9 (bitwise identical results).
template <int ST, int CO, int BX, int RPT, int NT = 0, int WPE = 0>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1))) void k_d2q9_pf(const typename Form<ST>::T *__restrict__ src,
                                                typename Form<ST>::T *__restrict__ dst, StepArgs a)
{
    using C = typename Form<ST>::C;
    using T = typename Form<ST>::T;
    const Inst &in = a.one;
    const int nx = in.nx, ny = in.ny, pitch = in.pitch;
    const int64_t P = in.plane;
    int tx, ty;
    tile_of_block(a.xcd_swizzle, a.tiles_x, tx, ty);
    const int x = tx * BX + (int)threadIdx.x;
    const bool xin = x < nx;
    const int xs = xin ? x : nx - 1;
    const int y0 = ty * RPT;
    const Cols cols = columns(xs, tx == 0 || tx == a.tiles_x - 1, nx, a.bc, sizeof(T));
    C ref[9];
    ref9<C>(C(in.rho0), ref);
    int bad = kNoNode;
    int guarded = 0;
    T raw[9];
    {
        const Nb n = neighbours(0, y0, 1, ny, a.bc);  // rows only
        pull9_cols<ST, nl_mode(NT)>(src, P, y0, n.ym, n.yp, pitch, cols.cc, cols.cm, cols.cp, raw);
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int y = y0 + k;
        if (y >= ny) break;  // uniform across the block
        C f[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q] = load<ST>(&raw[q], ref[q], a.fp16_iscale);
        if (k + 1 < RPT && y + 1 < ny) {
            const Nb n = neighbours(0, y + 1, 1, ny, a.bc);  // rows only
            pull9_cols<ST, nl_mode(NT)>(src, P, y + 1, n.ym, n.yp, pitch, cols.cc, cols.cm, cols.cp, raw);
        }
        if (a.bc == BC_CAVITY && y == ny - 1) {
            if (xin) push_lid<ST, (NT & 2) != 0>(dst, P, x, y, pitch, in, ref, a.fp16_scale);
            continue;
        }
        const int fl = node9_row<ST, CO>(f, xs, y, nx, ny, a.bc, in);
        if (xin && (fl & 1)) bad = min(bad, y * nx + x);
        guarded += __popcll(__ballot(xin && (fl & 2)));
        if (xin) push9_xy<ST, (NT & 2) != 0>(dst, P, x, y, pitch, f, ref, a.fp16_scale);
    }
    report(a.status, bad, guarded, a.step, a.step_base);
}

// --------------------------------------------------------------------------
// D2Q9, one lattice, two steps per launch (temporal blocking).
//
// A block of BX threads owns an output tile of BX columns and H rows (in a
// batch, of the instance's tile width tw <= BX, below).  It walks a window
// that is one node wider on every side: window column i is
// lattice column x0 - 1 + i and window row j is lattice row y0 - 1 + j, each
// mapped into the lattice by the neighbour rule (wrapped on periodic axes,
// clamped otherwise).  The first step computes every window node exactly as
// the single-step kernels compute that lattice node, and rounds it to the
// storage type into LDS; the second step computes the tile's own nodes from
// those values and writes them to HBM.  Because the window rows and columns
// around a node are precisely its neighbour rows and columns, every result
// is bitwise equal to two single-step launches, while HBM sees one read and
// one write of each population per two steps.
//
// The first step runs row by row (thread t: column x0 + t) and the second
// step trails it by one row.  RS = 4 or 3 keeps all nine planes of a window
// row in a ring of RS rows: with four slots one barrier per row suffices (the
// row written in iteration j + 1 was last read in iteration j - 1); three
// take less LDS and a second barrier.  RS = 0 splits the planes by how long
// they are needed: the second step reads the unshifted planes 0, 2 and 4 only
// in the thread's own column, so they stay in registers (plane 4 of the row
// just computed, plane 0 of the row before, plane 2 of the row before that);
// planes 7 and 8 are read in the iteration that writes them (two slots),
// 1 and 3 one iteration later (three), 5 and 6 two iterations later (four).
// That is 18 plane-rows of LDS instead of 36, with one barrier per row.  The
// two halo columns of every window row are computed first, by the first
// 2 (H + 2) threads, into their own LDS array, and copied into the ring as
// each row is written.  The second step reads a halo column only in the three
// planes that stream in from that side (1, 5, 8 from the left; 3, 6, 7 from
// the right), so the array keeps those six values per row.  Each first-step row's loads are
// issued one iteration ahead, before the barrier, and complete during the
// second step of the row before.
// Only nodes inside the tile report status (first step at a.step, second at
// a.step + 1), so every node reports once per step.
// --------------------------------------------------------------------------

// Plane-rows of LDS the ring of the two-step kernel holds (RS as there).
constexpr int t2_plane_rows(int rs) { return rs == 0 ? 18 : 9 * rs; }

// LDS of the two-step kernel: the ring (plane-rows of bx + 2 columns) and
// the three planes the second step reads in each halo column of every window
// row.
template <class T>
constexpr size_t t2_lds_bytes(int bx, int h, int rs)
{
    return sizeof(T) * (size_t)(t2_plane_rows(rs) * (bx + 2) + 6 * (h + 2));
}

// Plane of the k-th value (k < 3) kept for a halo column: the left column
// (side 0) feeds planes 1, 5 and 8 of the tile's first column, the right one
// planes 3, 6 and 7 of its last.
__device__ __forceinline__ int t2_halo_plane(int side, int k)
{
    return side ? (k == 0 ? 3 : (k == 1 ? 6 : 7)) : (k == 0 ? 1 : (k == 1 ? 5 : 8));
}

// Lattice coordinate of window coordinate g on an axis of n nodes: the
// neighbour rule one node beyond either edge (wrap or clamp); coordinates
// further out (ragged last tiles) are clamped, and those nodes are computed
// but never read.
__device__ __forceinline__ int t2_map(int g, int n, bool wrap)
{
    if (g < 0) return wrap ? n - 1 : 0;
    if (g >= n) return (wrap && g == n) ? 0 : n - 1;
    return g;
}

// Workgroup barrier that orders LDS accesses only, so global loads issued
// before it stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The same ordering within one wave, for tiles a single wave owns: LDS
// writes before it are visible to every lane of the wave after it.
__device__ __forceinline__ void lds_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// LDS bytes of one wave's tile in the wave-tiled mode (64 columns), rounded
// to 16 bytes.
template <class T>
constexpr size_t t2_wave_lds_bytes(int h, int rs)
{
    return (t2_lds_bytes<T>(64, h, rs) + 15) / 16 * 16;
}

// WT > 0 (batches): wave-tiled mode.  Each of the block's WT waves owns a
// tile of 64 columns (BX = 64) from the tile table, with an LDS region of its
// own; the waves never wait for each other, and a wave without a tile leaves
// at once.
template <int ST, int CO, int BX, int H, int RS, int NT = 0, int WPE = 0, bool BATCH = false, int WT = 0>
__global__ __launch_bounds__(WT > 0 ? 64 * WT : BX) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void k_d2q9_t2(const typename Form<ST>::T *__restrict__ src_all, typename Form<ST>::T *__restrict__ dst_all,
               StepArgs a)
{
    using C = typename Form<ST>::C;
    using T = typename Form<ST>::T;
    constexpr int W = BX + 2;     // window columns
    extern __shared__ __align__(16) unsigned char t2_lds[];
    static_assert(RS == 0 || RS == 3 || RS == 4, "ring of three or four window rows, or split rings");
    static_assert(WT == 0 || (BATCH && BX == 64), "wave-tiled mode: batches, 64-column tiles");
    // Barrier between a row's LDS writes and their reads: the block's, or in
    // the wave-tiled mode the wave's own.
    auto sync = [] {
        if constexpr (WT > 0) lds_wave_sync();
        else lds_barrier();
    };
    // Tile-table entry of this block (or of this wave in the wave-tiled mode).
    // (The wave index is read from the first lane so that the compiler knows
    // it, and everything derived from the tile, to be wave-uniform.)
    const int wave = WT > 0 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
    const int tile = WT > 0 ? (int)blockIdx.x * WT + wave
                            : (BATCH && a.xcd_swizzle ? xcd_remap((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x);
    if constexpr (WT > 0) {
        if (tile >= a.ntiles) return;  // wave-uniform; no block barrier in this mode
    }
    T *ring = (T *)(t2_lds + (size_t)wave * (WT > 0 ? t2_wave_lds_bytes<T>(H, RS) : 0));
    // RS > 0: [RS][9][W]; RS = 0: planes 7,8 [2][2][W], 1,3 [3][2][W], 5,6 [4][2][W]
    T *halo = ring + t2_plane_rows(RS) * W;  // [H + 2][2][3]
    // Plane q of window row j in the ring (q and the ring layout are
    // compile-time, j is uniform).
    auto plane = [&](int q, int j) -> T * {
        if constexpr (RS != 0) {
            return ring + ((j % RS) * 9 + q) * W;
        } else {
            if (q == 7 || q == 8) return ring + ((j & 1) * 2 + (q - 7)) * W;
            if (q == 1 || q == 3) return ring + (4 + (j % 3) * 2 + (q == 3)) * W;
            return ring + (10 + (j & 3) * 2 + (q - 5)) * W;  // q = 5, 6
        }
    };
    // Instance and tile of this block: a single lattice's grid of tiles, or a
    // batch's tile table (instance, tile index within the instance).
    const int ii = BATCH ? a.tile_inst[tile] : 0;
    const Inst &in = BATCH ? a.inst[ii] : a.one;
    const int nx = in.nx, ny = in.ny, pitch = in.pitch;
    const int64_t P = in.plane;
    const int tiles_x = BATCH ? (nx + BX - 1) / BX : a.tiles_x;
    int tx, ty;
    if constexpr (BATCH) {
        const int k = a.tile_first[tile];
        ty = k / tiles_x;
        tx = k - ty * tiles_x;
    } else {
        tile_of_block(a.xcd_swizzle, a.tiles_x, tx, ty);
    }
    const T *src = src_all + (BATCH ? in.offset : 0);
    T *dst = dst_all + (BATCH ? in.offset : 0);
    DevStatus *status = a.status + ii;
    const bool xw = a.bc == BC_PERIODIC;
    const bool yw = a.bc == BC_PERIODIC || a.bc == BC_TUBE;
    const bool cavity = a.bc == BC_CAVITY;
    const int t = WT > 0 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
    // Tile width: BX, or in a batch the instance's columns spread evenly over
    // its tiles_x tiles, rounded up to whole waves (an instance 300 wide
    // takes two tiles of 192 columns instead of two of 256).  The waves of a
    // block that hold no needed column, beyond the tile's width or beyond the
    // column just past the instance's edge, skip the arithmetic and keep
    // every barrier.
    constexpr bool BAL = BATCH && WT == 0;
    int tw = BX;
    if constexpr (BAL) tw = min(BX, ((nx + tiles_x - 1) / tiles_x + 63) & ~63);
    const int x0 = tx * tw, y0 = ty * H;
    const int hn = min(H, ny - y0);  // output rows of this tile (block-uniform)
    const int x = x0 + t;
    const bool xin = (!BAL || t < tw) && x < nx;
    const int xs = t2_map(x, nx, xw);  // lattice column of this thread's window column
    bool wave_on = true;
    if constexpr (BAL) {
        const int t0 = __builtin_amdgcn_readfirstlane(t & ~63);
        wave_on = t0 < tw && t0 <= nx - x0;
    }

    // Steps this launch takes here (block-uniform): two; one for an odd step
    // count's last step, or for a batch instance whose step limit falls
    // between the two (the first step's own nodes then go straight to HBM);
    // none for a stopped instance, which carries its state over.
    int kdo = a.max_steps;
    if constexpr (BATCH) {
        const int64_t s0 = a.step + (a.step_base ? *a.step_base : 0);
        kdo = (int)max((int64_t)0, min((int64_t)kdo, in.stop - s0));
    }
    if (kdo <= 0) {
        if (xin)
            for (int r = 0; r < hn; ++r) carry_node(src, dst, P, 9, (y0 + r) * pitch + x);
        return;
    }
    const Cols cols = columns(xs, tx == 0 || tx == tiles_x - 1, nx, a.bc, sizeof(T));
    C ref[9];
    ref9<C>(C(in.rho0), ref);

    // The first window row's loads are issued first, so that they are in
    // flight during the halo columns' first step.
    const int nj = hn + 2;
    auto row_of = [&](int j) { return t2_map(y0 - 1 + j, ny, yw); };
    auto pull_row = [&](int j, T (&r)[9]) {
        const int gy = row_of(j);
        if (cavity && gy == ny - 1) return;  // the lid row loads nothing
        const Nb n = neighbours(0, gy, 1, ny, a.bc);  // rows only
        pull9_row_u<ST, nl_mode(NT)>(src, P, gy, n.ym, n.yp, pitch, cols.cc, cols.cm, cols.cp, r);
    };
    T raw[9];
    if (wave_on) pull_row(0, raw);

    // Halo columns (x0 - 1 and x0 + tw) of every window row, first step.
    for (int k = t; k < 2 * (hn + 2); k += BX) {
        const int side = k & 1, j = k >> 1;
        const int gx = t2_map(side ? x0 + tw : x0 - 1, nx, xw);
        const int gy = row_of(j);
        C f[9];
        const Nb n = neighbours(gx, gy, nx, ny, a.bc);
        pull9<ST>(src, P, gx, gy, pitch, n, ref, a.fp16_iscale, f);
        (void)node9<ST, CO>(f, role9(gx, gy, nx, ny, a.bc), in);
        // The three planes the second step reads in this column (t2_halo_plane;
        // ref is the same within the axis and within the diagonal directions).
        T *h = halo + (j * 2 + side) * 3;
        store<ST>(h + 0, side ? f[3] : f[1], ref[1], a.fp16_scale);
        store<ST>(h + 1, side ? f[6] : f[5], ref[5], a.fp16_scale);
        store<ST>(h + 2, side ? f[7] : f[8], ref[5], a.fp16_scale);
    }

    int bad1 = kNoNode, bad2 = kNoNode;
    int guarded = 0;
    if constexpr (BAL) {
        if (!wave_on) {
            // A wave without a needed column takes only the block's barriers,
            // as many and in the order the row loop below takes them.
            sync();  // halo array complete
            for (int j = 0; j < nj; ++j) {
                if constexpr (RS == 3) {
                    if (j > 0) sync();
                }
                sync();
            }
            return;
        }
    }
    T lid_st[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) lid_st[q] = to_storage<ST>(C(in.lid[q]), ref[q], a.fp16_scale);
    sync();  // halo array complete

    // Iteration j: first step of window row j from raw (loaded in the
    // iteration before), loads of row j + 1 into raw, barrier, second step of
    // lattice row y0 + j - 2.
    constexpr int kShifted[6] = {1, 3, 5, 6, 7, 8};  // planes read in a neighbour column
    T u0 = T(0), u2a = T(0), u2b = T(0);  // RS = 0: plane 0 of row j - 1, plane 2 of rows j - 1 and j - 2
    for (int j = 0; j < nj; ++j) {
        // Three slots: the slot written now was read by the last second step.
        if constexpr (RS == 3) {
            if (j > 0) sync();
        }
        T v0 = T(0), v2 = T(0), v4 = T(0);  // RS = 0: the unshifted planes of row j
        {
            const int gy = row_of(j);
            // The row's populations in storage form, converted once for the
            // ring and the direct write: the lid row's are the lid
            // equilibrium's (uniform), any other row's its first step's.
            T sv[9];
            int fl = 0;
            if (cavity && gy == ny - 1) {
                // (An empty statement gives this path a block of its own, so
                // that the copies below are not hoisted onto every row.)
                asm volatile("");
#pragma unroll
                for (int q = 0; q < 9; ++q) sv[q] = lid_st[q];
            } else {
                C f[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) f[q] = load<ST>(&raw[q], ref[q], a.fp16_iscale);
                fl = node9_row<ST, CO>(f, xs, gy, nx, ny, a.bc, in);
#pragma unroll
                for (int q = 0; q < 9; ++q) sv[q] = to_storage<ST>(f[q], ref[q], a.fp16_scale);
            }
            const bool own = j >= 1 && j <= hn && xin;
            if (own && (fl & 1)) bad1 = min(bad1, gy * nx + x);
            guarded += __popcll(__ballot(own && (fl & 2)));
            if (kdo == 1 && own) push9_xy_st<ST, (NT & 2) != 0>(dst, P, x, gy, pitch, sv);
            if constexpr (RS != 0) {
#pragma unroll
                for (int q = 0; q < 9; ++q) plane(q, j)[t + 1] = sv[q];
                if (t < 6) {
                    const int side = t >= 3, k = t - 3 * side;
                    plane(t2_halo_plane(side, k), j)[side ? tw + 1 : 0] = halo[(j * 2 + side) * 3 + k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const int q = kShifted[k];
                    plane(q, j)[t + 1] = sv[q];
                }
                v0 = sv[0];
                v2 = sv[2];
                v4 = sv[4];
                if (t < 6) {
                    const int side = t >= 3, k = t - 3 * side;
                    plane(t2_halo_plane(side, k), j)[side ? tw + 1 : 0] = halo[(j * 2 + side) * 3 + k];
                }
            }
        }
        if (j + 1 < nj) pull_row(j + 1, raw);  // completes during this second step
        sync();
        // Unshifted planes this second step reads from registers (rows j - 1
        // and j - 2), then the delay line moves on by one row.
        const T s0 = u0, s2 = u2b;
        u0 = v0;
        u2b = u2a;
        u2a = v2;
        if (j < 2 || kdo == 1) continue;
        // Second step, lattice row y = y0 + j - 2 (window row j - 1): window
        // rows j - 2 and j hold its neighbour rows, window columns t and
        // t + 2 its neighbour columns.
        const int y = y0 + j - 2;
        if (cavity && y == ny - 1) {
            if (xin) push_lid<ST, (NT & 2) != 0>(dst, P, x, y, pitch, in, ref, a.fp16_scale);
            continue;
        }
        C f[9];
        if constexpr (RS != 0) {
            f[0] = load<ST>(plane(0, j - 1) + t + 1, ref[0], a.fp16_iscale);
            f[2] = load<ST>(plane(2, j - 2) + t + 1, ref[2], a.fp16_iscale);
            f[4] = load<ST>(plane(4, j) + t + 1, ref[4], a.fp16_iscale);
        } else {
            f[0] = load<ST>(&s0, ref[0], a.fp16_iscale);
            f[2] = load<ST>(&s2, ref[2], a.fp16_iscale);
            f[4] = load<ST>(&v4, ref[4], a.fp16_iscale);
        }
        f[1] = load<ST>(plane(1, j - 1) + t, ref[1], a.fp16_iscale);
        f[3] = load<ST>(plane(3, j - 1) + t + 2, ref[3], a.fp16_iscale);
        f[5] = load<ST>(plane(5, j - 2) + t, ref[5], a.fp16_iscale);
        f[6] = load<ST>(plane(6, j - 2) + t + 2, ref[6], a.fp16_iscale);
        f[7] = load<ST>(plane(7, j) + t + 2, ref[7], a.fp16_iscale);
        f[8] = load<ST>(plane(8, j) + t, ref[8], a.fp16_iscale);
        const int fl = node9_row<ST, CO>(f, xs, y, nx, ny, a.bc, in);
        if (xin && (fl & 1)) bad2 = min(bad2, y * nx + x);
        guarded += __popcll(__ballot(xin && (fl & 2)));
        if (xin) push9_xy<ST, (NT & 2) != 0>(dst, P, x, y, pitch, f, ref, a.fp16_scale);
    }
    report(status, bad1, guarded, a.step, a.step_base);
    report(status, bad2, 0, a.step + 1, a.step_base);
}

// --------------------------------------------------------------------------
// D2Q9, batch of lattices.  A tile is BLK consecutive nodes (row-major) of
// one instance; tile tables give its instance and first node.
// --------------------------------------------------------------------------

template <int ST, int CO, int BLK, int NT = 0>
__global__ __launch_bounds__(BLK) void k_d2q9_batch(const typename Form<ST>::T *__restrict__ src,
                                                    typename Form<ST>::T *__restrict__ dst, StepArgs a)
{
    using C = typename Form<ST>::C;
    if constexpr ((NT & 8) != 0) __builtin_amdgcn_s_setprio(2);  // until the loads are issued
    int t = blockIdx.x;
    if (a.xcd_swizzle) t = xcd_remap(t, gridDim.x);
    const int i = a.tile_inst[t];
    const Inst &in = a.inst[i];
    const int nx = in.nx, ny = in.ny;
    const int64_t P = in.plane;
    const int nodes = nx * ny;
    int node = a.tile_first[t] + (int)threadIdx.x;
    const bool valid = node < nodes;
    if (!valid) node = nodes - 1;
    // node -> (x, y): float estimate, exact after one correction (node < 2^24).
    int y = (int)((float)node * __builtin_amdgcn_rcpf((float)nx));
    int x = node - y * nx;
    if (x < 0) { --y; x += nx; }
    if (x >= nx) { ++y; x -= nx; }
    constexpr uint32_t E = sizeof(typename Form<ST>::T);
    // Byte offsets of the node's row and its rows below and above (rows are
    // `pitch` elements apart; the neighbours are one row away unless the
    // wrap/clamp rule applies).
    const uint32_t rb = (uint32_t)in.pitch * E, rc = (uint32_t)y * rb;
    if (instance_stopped(a, in)) {  // uniform across the block
        if (valid) carry_node(src + in.offset, dst + in.offset, P, 9, y * in.pitch + x);
        return;
    }
    C ref[9];
    ref9<C>(C(in.rho0), ref);
    const Nb n = neighbours(x, y, nx, ny, a.bc);
    const uint32_t rm = n.ym == y - 1 ? rc - rb : (uint32_t)n.ym * rb;
    const uint32_t rp = n.yp == y + 1 ? rc + rb : (uint32_t)n.yp * rb;
    C f[9];
    {
        typename Form<ST>::T raw[9];
        pull9_inst<ST, nl_mode(NT)>(uniform_addr(src + in.offset), P, rc, rm, rp, (uint32_t)x * E,
                                    (uint32_t)n.xm * E, (uint32_t)n.xp * E, raw);
        if constexpr ((NT & 8) != 0) __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q] = load<ST>(&raw[q], ref[q], a.fp16_iscale);
    }
    const int role = role9(x, y, nx, ny, a.bc);
    const int fl = node9<ST, CO>(f, role, in);
    if (valid)
        push9_inst<ST, (NT & 2) != 0>(uniform_addr(dst + in.offset), P, rc + (uint32_t)x * E, f, ref,
                                      a.fp16_scale);
    const int guarded = __popcll(__ballot(valid && (fl & 2)));
    report(a.status + i, valid && (fl & 1) ? node : kNoNode, guarded, a.step, a.step_base);
}

// --------------------------------------------------------------------------
// D2Q9, batch of small lattices resident in LDS: one workgroup per instance
// runs `nsteps` steps inside one launch.  Both population buffers live in
// LDS at storage precision (so every step rounds exactly as the per-step
// kernels do and results are bitwise identical); a workgroup barrier
// separates the steps.  The state is read from `src` once and the final
// state written to `dst` once (they may be the same buffer: every read
// happens before the first write).
// --------------------------------------------------------------------------

template <int ST, int CO>
__global__ __launch_bounds__(1024) void k_d2q9_lds(const typename Form<ST>::T *src, typename Form<ST>::T *dst,
                                                   StepArgs a, int nsteps)
{
    using C = typename Form<ST>::C;
    using T = typename Form<ST>::T;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int i = blockIdx.x;
    const Inst &in = a.inst[i];
    const int nx = in.nx, ny = in.ny;
    const int nodes = nx * ny;
    T *L0 = (T *)lds_raw;
    T *L1 = L0 + 9 * nodes;
    const T *g = src + in.offset;
    // LDS holds the nodes without the row padding: node j of plane q at
    // q * nodes + j.
    for (int idx = threadIdx.x; idx < 9 * nodes; idx += blockDim.x) {
        const int q = idx / nodes, j = idx - q * nodes, jy = j / nx;
        L0[idx] = g[q * in.plane + jy * in.pitch + (j - jy * nx)];
    }
    __syncthreads();
    C ref[9];
    ref9<C>(C(in.rho0), ref);
    const float inx = __builtin_amdgcn_rcpf((float)nx);
    const int64_t s0 = a.step + (a.step_base ? *a.step_base : 0);
    uint64_t first_bad = ~0ull;
    int64_t guarded = 0;
    // Steps this instance takes in this launch (its step limit may end them
    // early; the break below is uniform across the block).
    const int kdone = (int)max((int64_t)0, min((int64_t)nsteps, in.stop - s0));
    for (int k = 0; k < nsteps; ++k) {
        if (k >= kdone) break;
        const T *sin = (k & 1) ? L1 : L0;
        T *sout = (k & 1) ? L0 : L1;
        for (int node = threadIdx.x; node < nodes; node += blockDim.x) {
            int y = (int)((float)node * inx);
            int x = node - y * nx;
            if (x < 0) { --y; x += nx; }
            if (x >= nx) { ++y; x -= nx; }
            const Nb n = neighbours(x, y, nx, ny, a.bc);
            C f[9];
            pull9<ST>(sin, nodes, x, y, nx, n, ref, a.fp16_iscale, f);
            const int fl = node9<ST, CO>(f, role9(x, y, nx, ny, a.bc), in);
            if ((fl & 1) && first_bad == ~0ull) first_bad = event_key(s0 + k, node);  // first step, smallest node of this thread
            guarded += (fl >> 1) & 1;
            push9<ST>(sout, nodes, node, f, ref, a.fp16_scale);
        }
        __syncthreads();
    }
    const T *fin = (kdone & 1) ? L1 : L0;
    T *o = dst + in.offset;
    for (int idx = threadIdx.x; idx < 9 * nodes; idx += blockDim.x) {
        const int q = idx / nodes, j = idx - q * nodes, jy = j / nx;
        o[q * in.plane + jy * in.pitch + (j - jy * nx)] = fin[idx];
    }
    // Status: rare events, one atomic per reporting lane.
    DevStatus *st = a.status + i;
    if (first_bad != ~0ull) {
        atomicOr(&st->flags, 1u);
        atomicMin((unsigned long long *)&st->first, (unsigned long long)first_bad);
    }
    if (guarded != 0) {
        atomicOr(&st->flags, 2u);
        atomicAdd((unsigned long long *)&st->guarded, (unsigned long long)guarded);
    }
}

// --------------------------------------------------------------------------
// D1Q3 (rest, +1, -1): SRT, the exact form of the method on this lattice.
// --------------------------------------------------------------------------

template <class C>
__device__ __forceinline__ int node3(C &f0, C &fp, C &fm, int role, C omega)
{
    if (role == R_WALL) {
        const C t = fp;
        fp = fm;
        fm = t;
        return 0;
    }
    const C rho = (f0 + fp) + fm;
    const C u = (fp - fm) * rcp(rho);
    const C uu = u * u;
    const C e0 = C(2.0 / 3.0) * rho * (C(1) - C(1.5) * uu);
    const C es = C(1.0 / 6.0) * rho * (C(1) + C(3) * uu);
    const C eu = C(1.0 / 6.0) * rho * (C(3) * u);
    f0 = f0 + omega * (e0 - f0);
    fp = fp + omega * ((es + eu) - fp);
    fm = fm + omega * ((es - eu) - fm);
    return (nonneg_finite(f0) && nonneg_finite(fp) && nonneg_finite(fm)) ? 0 : 1;
}

template <int ST, int NT = 0>
__device__ __forceinline__ int step3_node(const typename Form<ST>::T *__restrict__ s,
                                          typename Form<ST>::T *__restrict__ d, int64_t P, int x, int nx,
                                          int bc, typename Form<ST>::C omega, typename Form<ST>::C rho0,
                                          const StepArgs &a, bool valid)
{
    using C = typename Form<ST>::C;
    const bool wrap = bc == BC_PERIODIC;
    const int xm = x > 0 ? x - 1 : (wrap ? nx - 1 : 0);
    const int xp = x < nx - 1 ? x + 1 : (wrap ? 0 : nx - 1);
    const C r0 = C(2.0 / 3.0) * rho0, r1 = C(1.0 / 6.0) * rho0;
    using T = typename Form<ST>::T;
    const T l0 = ldraw<T, (NT & 1) != 0>(s + x), l1 = ldraw<T, (NT & 1) != 0>(s + P + xm),
            l2 = ldraw<T, (NT & 1) != 0>(s + 2 * P + xp);
    C f0 = load<ST>(&l0, r0, a.fp16_iscale);
    C fp = load<ST>(&l1, r1, a.fp16_iscale);
    C fm = load<ST>(&l2, r1, a.fp16_iscale);
    const int role = (bc != BC_PERIODIC && (x == 0 || x == nx - 1)) ? R_WALL : R_FLUID;
    const int fl = node3<C>(f0, fp, fm, role, omega);
    if (valid) {
        store<ST, (NT & 2) != 0>(d + x, f0, r0, a.fp16_scale);
        store<ST, (NT & 2) != 0>(d + P + x, fp, r1, a.fp16_scale);
        store<ST, (NT & 2) != 0>(d + 2 * P + x, fm, r1, a.fp16_scale);
    }
    return fl;
}

// Sixteen bytes of stored populations viewed as elements, and eight
// consecutive populations moved as one or more 16-byte vector accesses.
template <class T>
struct Chunk {
    T e[16 / sizeof(T)];
};

template <class T, bool NT>
__device__ __forceinline__ void ld8(const T *p, T (&v)[8])
{
    constexpr int per = 16 / sizeof(T);
#pragma unroll
    for (int c = 0; c < 8 / per; ++c) {
        const u32x4 *q = (const u32x4 *)(p + c * per);
        u32x4 w;
        if constexpr (NT) w = __builtin_nontemporal_load(q);
        else w = *q;
        const Chunk<T> b = __builtin_bit_cast(Chunk<T>, w);
#pragma unroll
        for (int e = 0; e < per; ++e) v[c * per + e] = b.e[e];
    }
}

template <class T, bool NT>
__device__ __forceinline__ void st8(T *p, const T (&v)[8])
{
    constexpr int per = 16 / sizeof(T);
#pragma unroll
    for (int c = 0; c < 8 / per; ++c) {
        Chunk<T> b;
#pragma unroll
        for (int e = 0; e < per; ++e) b.e[e] = v[c * per + e];
        const u32x4 w = __builtin_bit_cast(u32x4, b);
        u32x4 *q = (u32x4 *)(p + c * per);
        if constexpr (NT) __builtin_nontemporal_store(w, q);
        else *q = w;
    }
}

// Eight consecutive nodes x0 .. x0+7 of one D1Q3 lattice (x0 a multiple of 8,
// x0 < nx; plane bases 256-byte aligned and plane lengths rounded up to 64
// elements, so each group is 16-byte aligned and inside its plane).  Every plane moves as
// 16-byte vectors; the two values shifted in from outside the group (plane 1
// from the left, plane 2 from the right) take one scalar load each, with the
// same wrap/clamp rule as the one-node form, so results are bitwise equal to
// it.  Nodes beyond nx in the last group are computed but neither stored nor
// counted.  Returns the smallest unstable valid node of the group, or kNoNode.
template <int ST, int NT = 0>
__device__ __forceinline__ int step3_group8(const typename Form<ST>::T *__restrict__ s,
                                             typename Form<ST>::T *__restrict__ d, int64_t P, int x0, int nx,
                                             int bc, typename Form<ST>::C omega, typename Form<ST>::C rho0,
                                             const StepArgs &a)
{
    using C = typename Form<ST>::C;
    using T = typename Form<ST>::T;
    constexpr bool NL = (NT & 1) != 0, NS = (NT & 2) != 0;
    T v0[8], v1[8], v2[8];
    ld8<T, NL>(s + x0, v0);
    ld8<T, NL>(s + P + x0, v1);
    ld8<T, NL>(s + 2 * P + x0, v2);
    const bool wrap = bc == BC_PERIODIC;
    const int jl = nx - 1 - x0 < 7 ? nx - 1 - x0 : 7;  // last valid node of the group
    const int xl = x0 + jl;
    const int xm = x0 > 0 ? x0 - 1 : (wrap ? nx - 1 : 0);
    const int xp = xl < nx - 1 ? xl + 1 : (wrap ? 0 : nx - 1);
    const T s1 = ldraw<T, NL>(s + P + xm), s2 = ldraw<T, NL>(s + 2 * P + xp);
    const C r0 = C(2.0 / 3.0) * rho0, r1 = C(1.0 / 6.0) * rho0;
    int bad = kNoNode;
    // Results go back into v0 and v2 in place (node j reads only v0[j] and
    // v2[j+1], not yet overwritten when walking upwards) but into o1 for
    // plane 1, whose node j reads v1[j-1].
    T o1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int x = x0 + j;
        const T rp = j == 0 ? s1 : v1[j > 0 ? j - 1 : 0];
        const T rm = j < jl ? v2[j < 7 ? j + 1 : 7] : s2;
        C f0 = load<ST>(&v0[j], r0, a.fp16_iscale);
        C fp = load<ST>(&rp, r1, a.fp16_iscale);
        C fm = load<ST>(&rm, r1, a.fp16_iscale);
        const int role = (bc != BC_PERIODIC && (x == 0 || x == nx - 1)) ? R_WALL : R_FLUID;
        const int fl = node3<C>(f0, fp, fm, role, omega);
        if (bad == kNoNode && j <= jl && fl) bad = x;
        if constexpr (ST == ST_F16DEV) {
            v0[j] = enc16(f0, r0, a.fp16_scale);
            o1[j] = enc16(fp, r1, a.fp16_scale);
            v2[j] = enc16(fm, r1, a.fp16_scale);
        } else {
            v0[j] = T(f0);
            o1[j] = T(fp);
            v2[j] = T(fm);
        }
    }
    if (jl == 7) {
        st8<T, NS>(d + x0, v0);
        st8<T, NS>(d + P + x0, o1);
        st8<T, NS>(d + 2 * P + x0, v2);
    } else {
        for (int j = 0; j <= jl; ++j) {
            d[x0 + j] = v0[j];
            d[P + x0 + j] = o1[j];
            d[2 * P + x0 + j] = v2[j];
        }
    }
    return bad;
}

template <int ST, int BX, int NT = 0>
__global__ __launch_bounds__(BX) void k_d1q3_v8(const typename Form<ST>::T *__restrict__ src,
                                                typename Form<ST>::T *__restrict__ dst, StepArgs a)
{
    using C = typename Form<ST>::C;
    const Inst &in = a.one;
    const int x0 = (blockIdx.x * BX + (int)threadIdx.x) * 8;
    int bad = kNoNode;
    if (x0 < in.nx) bad = step3_group8<ST, NT>(src, dst, in.plane, x0, in.nx, a.bc, C(in.omega), C(in.rho0), a);
    report(a.status, bad, 0, a.step, a.step_base);
}

template <int ST, int BLK, int NT = 0>
__global__ __launch_bounds__(BLK) void k_d1q3_batch_v8(const typename Form<ST>::T *__restrict__ src,
                                                       typename Form<ST>::T *__restrict__ dst, StepArgs a)
{
    using C = typename Form<ST>::C;
    int t = blockIdx.x;
    if (a.xcd_swizzle) t = xcd_remap(t, gridDim.x);
    const int i = a.tile_inst[t];
    const Inst &in = a.inst[i];
    const int x0 = a.tile_first[t] + (int)threadIdx.x * 8;
    if (instance_stopped(a, in)) {  // uniform across the block
        for (int j = 0; j < 8 && x0 + j < in.nx; ++j)
            carry_node(src + in.offset, dst + in.offset, in.plane, 3, x0 + j);
        return;
    }
    int bad = kNoNode;
    if (x0 < in.nx)
        bad = step3_group8<ST, NT>(src + in.offset, dst + in.offset, in.plane, x0, in.nx, a.bc, C(in.omega),
                                   C(in.rho0), a);
    report(a.status + i, bad, 0, a.step, a.step_base);
}

template <int ST, int BX, int NPT, int NT = 0>
__global__ __launch_bounds__(BX) void k_d1q3(const typename Form<ST>::T *__restrict__ src,
                                             typename Form<ST>::T *__restrict__ dst, StepArgs a)
{
    using C = typename Form<ST>::C;
    const Inst &in = a.one;
    const int nx = in.nx;
    int bad = kNoNode;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int x = (blockIdx.x * NPT + k) * BX + (int)threadIdx.x;
        const bool valid = x < nx;
        const int fl = step3_node<ST, NT>(src, dst, in.plane, valid ? x : nx - 1, nx, a.bc, C(in.omega),
                                      C(in.rho0), a, valid);
        if (valid && fl) bad = min(bad, x);
    }
    report(a.status, bad, 0, a.step, a.step_base);
}

template <int ST, int BLK, int NPT, int NT = 0>
__global__ __launch_bounds__(BLK) void k_d1q3_batch(const typename Form<ST>::T *__restrict__ src,
                                                    typename Form<ST>::T *__restrict__ dst, StepArgs a)
{
    using C = typename Form<ST>::C;
    int t = blockIdx.x;
    if (a.xcd_swizzle) t = xcd_remap(t, gridDim.x);
    const int i = a.tile_inst[t];
    const Inst &in = a.inst[i];
    const int nx = in.nx;
    if (instance_stopped(a, in)) {  // uniform across the block
        for (int k = 0; k < NPT; ++k) {
            const int x = a.tile_first[t] + k * BLK + (int)threadIdx.x;
            if (x < nx) carry_node(src + in.offset, dst + in.offset, in.plane, 3, x);
        }
        return;
    }
    int bad = kNoNode;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int x = a.tile_first[t] + k * BLK + (int)threadIdx.x;
        const bool valid = x < nx;
        const int fl = step3_node<ST, NT>(src + in.offset, dst + in.offset, in.plane, valid ? x : nx - 1, nx, a.bc,
                                      C(in.omega), C(in.rho0), a, valid);
        if (valid && fl) bad = min(bad, x);
    }
    report(a.status + i, bad, 0, a.step, a.step_base);
}

// --------------------------------------------------------------------------
// State set-up and read-back (off the hot loop; FP64 in and out).
// --------------------------------------------------------------------------

// Storage node (x, y) receives, for each direction a, the value that node
// (x, y) + v_a must pull at the next step: the equilibrium of that node's
// fields (or the given populations).  Destinations outside the lattice take
// the node's own value.
template <int ST, int B>
__global__ void k_init(Inst in, int bc, const double *__restrict__ rho, const double *__restrict__ ux,
                       const double *__restrict__ uy, const double *__restrict__ fin, typename Form<ST>::T *buf,
                       float scale)
{
    using C = typename Form<ST>::C;
    const int nx = in.nx, ny = in.ny;
    const int n = nx * ny;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = i % nx, y = i / nx;
    const bool xw = bc == BC_PERIODIC;
    const bool yw = (bc == BC_PERIODIC || bc == BC_TUBE) && B == 9;
    typename Form<ST>::T *d = buf + in.offset;
    for (int a = 0; a < B; ++a) {
        const int vx = (B == 9) ? cx9(a) : (a == 1 ? 1 : (a == 2 ? -1 : 0));
        const int vy = (B == 9) ? cy9(a) : 0;
        int tx = x + vx, ty = y + vy;
        if (tx < 0 || tx >= nx) tx = xw ? (tx + nx) % nx : x;
        if (ty < 0 || ty >= ny) ty = yw ? (ty + ny) % ny : y;
        if ((tx == x && vx != 0 && !xw) || (ty == y && vy != 0 && !yw)) { tx = x; ty = y; }
        const int j = ty * nx + tx;
        double v;
        if (fin) {
            v = fin[(int64_t)a * n + j];
        } else if (B == 9 && bc == BC_CAVITY && ty == ny - 1) {
            v = in.lid[a];
        } else {
            const double r = rho[j], u = ux[j], w = (B == 9) ? uy[j] : 0.0;
            const double cu = vx * u + vy * w;
            const double wa = (B == 9) ? ((a == 0) ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0))
                                       : (a == 0 ? 2.0 / 3.0 : 1.0 / 6.0);
            v = wa * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (u * u + w * w));
        }
        C ref;
        if (B == 9) {
            ref = (a == 0 ? W9<C>::rest : (a < 5 ? W9<C>::axis : W9<C>::diag)) * C(in.rho0);
        } else {
            ref = (a == 0 ? C(2.0 / 3.0) : C(1.0 / 6.0)) * C(in.rho0);
        }
        store<ST>(d + (int64_t)a * in.plane + (int64_t)y * in.pitch + x, C(v), ref, scale);
    }
}

template <int ST, int B>
__global__ void k_gather(Inst in, int bc, const typename Form<ST>::T *__restrict__ buf, double *rho, double *ux,
                         double *uy, double *fout, float iscale)
{
    using C = typename Form<ST>::C;
    const int nx = in.nx, ny = in.ny;
    const int n = nx * ny;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = i % nx, y = i / nx;
    const int pitch = in.pitch;
    const typename Form<ST>::T *s = buf + in.offset;
    double f[9];
    if (B == 9) {
        C ref[9];
        ref9<C>(C(in.rho0), ref);
        C g[9];
        pull9<ST>(s, in.plane, x, y, pitch, neighbours(x, y, nx, ny, bc), ref, iscale, g);
        for (int a = 0; a < 9; ++a) f[a] = double(g[a]);
    } else {
        const bool wrap = bc == BC_PERIODIC;
        const int xm = x > 0 ? x - 1 : (wrap ? nx - 1 : 0);
        const int xp = x < nx - 1 ? x + 1 : (wrap ? 0 : nx - 1);
        const C r0 = C(2.0 / 3.0) * C(in.rho0), r1 = C(1.0 / 6.0) * C(in.rho0);
        f[0] = double(load<ST>(s + x, r0, iscale));
        f[1] = double(load<ST>(s + in.plane + xm, r1, iscale));
        f[2] = double(load<ST>(s + 2 * in.plane + xp, r1, iscale));
    }
    if (fout) {
        for (int a = 0; a < B; ++a) fout[(int64_t)a * n + i] = f[a];
        return;
    }
    double r, jx, jy;
    if (B == 9) {
        r = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
        jx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
        jy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
    } else {
        r = f[0] + f[1] + f[2];
        jx = f[1] - f[2];
        jy = 0.0;
    }
    if (rho) rho[i] = r;
    if (ux) ux[i] = jx / r;
    if (uy) uy[i] = jy / r;
}

// Each thread moves kCopyVec 16-byte vectors, one block-width apart, so every
// load instruction of a wave covers 1 KiB of contiguous memory and a thread
// has kCopyVec loads in flight before its first store.
constexpr int kCopyVec = 4;

__global__ __launch_bounds__(256) void k_copy(u32x4 *__restrict__ d, const u32x4 *__restrict__ s, size_t n)
{
    const size_t b0 = (size_t)blockIdx.x * (256 * kCopyVec);
    const size_t i0 = b0 + threadIdx.x;
    u32x4 v[kCopyVec];
    if (b0 + 256 * kCopyVec <= n) {  // whole block: no per-vector test, loads all in flight
#pragma unroll
        for (int j = 0; j < kCopyVec; ++j) v[j] = __builtin_nontemporal_load(s + i0 + (size_t)j * 256);
#pragma unroll
        for (int j = 0; j < kCopyVec; ++j) __builtin_nontemporal_store(v[j], d + i0 + (size_t)j * 256);
        return;
    }
#pragma unroll
    for (int j = 0; j < kCopyVec; ++j) {
        const size_t i = i0 + (size_t)j * 256;
        if (i < n) v[j] = __builtin_nontemporal_load(s + i);
    }
#pragma unroll
    for (int j = 0; j < kCopyVec; ++j) {
        const size_t i = i0 + (size_t)j * 256;
        if (i < n) __builtin_nontemporal_store(v[j], d + i);
    }
}

__global__ void k_step_base(int64_t *b, int64_t v, int add)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *b = add ? *b + v : v;
}

__global__ void k_clear_status(DevStatus *st, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        st[i].flags = 0;
        st[i].pad = 0;
        st[i].first = ~0ull;
        st[i].guarded = 0;
    }
}

// --------------------------------------------------------------------------
// D1Q3, up to K steps per launch (temporal blocking).
//
// A block owns S = BX * NPT consecutive nodes of one lattice (a tile-table
// entry in a batch) and loads the stored populations of a window reaching
// KMAX nodes further on each side into LDS: on a periodic axis the window
// wraps (window node w is lattice node (x0 - KMAX + w) mod n, as often as the
// window needs it); otherwise it is cut at the lattice ends.  Step s then
// recomputes every window node that still has both neighbours from step
// s - 1: each step the valid part shrinks by one node at every window end
// that is not a lattice end, while at a lattice end the wall pulls from
// itself exactly as the single-step kernels do (neighbour rule).  After k
// steps (k <= KMAX) the block's own nodes are still valid and go to HBM.
// Every window node is computed with the same arithmetic and rounded to the
// storage type after every step, so results are bitwise equal to k
// single-step launches, while HBM sees one read (plus the 2 KMAX halo) and
// one write of every population per k steps.
// --------------------------------------------------------------------------

template <class T>
constexpr size_t tk_lds_bytes(int s, int kmax)
{
    return sizeof(T) * (size_t)2 * 3 * (size_t)(s + 2 * kmax);
}

// Wave-level minimum of a 64-bit event key and one atomic for the wave.
__device__ __forceinline__ void report_key(DevStatus *st, uint64_t key)
{
    if (__ballot(key != ~0ull) == 0ull) return;
    uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t l2 = (uint32_t)__shfl_xor((int)lo, o), h2 = (uint32_t)__shfl_xor((int)hi, o);
        if (h2 < hi || (h2 == hi && l2 < lo)) {
            hi = h2;
            lo = l2;
        }
    }
    if (__lane_id() == 0) {
        atomicOr(&st->flags, 1u);
        atomicMin((unsigned long long *)&st->first, ((unsigned long long)hi << 32) | lo);
    }
}

template <int ST, int BX, int NPT, int KMAX, int NT = 0, bool BATCH = false>
__global__ __launch_bounds__(BX) void k_d1q3_tk(const typename Form<ST>::T *__restrict__ src_all,
                                                typename Form<ST>::T *__restrict__ dst_all, StepArgs a)
{
    using C = typename Form<ST>::C;
    using T = typename Form<ST>::T;
    constexpr int S = BX * NPT;
    constexpr int W = S + 2 * KMAX;
    extern __shared__ __align__(16) unsigned char tk_lds[];
    T *b0 = (T *)tk_lds;  // two buffers of [3][W]
    T *b1 = b0 + 3 * W;
    const int tile = (int)blockIdx.x;
    const int ii = BATCH ? a.tile_inst[tile] : 0;
    const Inst &in = BATCH ? a.inst[ii] : a.one;
    const int n = in.nx;
    const int64_t P = in.plane;
    const int x0 = BATCH ? a.tile_first[tile] : tile * S;  // first own node
    const T *src = src_all + (BATCH ? in.offset : 0);
    T *dst = dst_all + (BATCH ? in.offset : 0);
    DevStatus *status = a.status + ii;
    const bool wrap = a.bc == BC_PERIODIC;
    const int t = (int)threadIdx.x;
    const int sn = min(S, n - x0);  // own nodes (block-uniform)

    // Steps this launch takes here (block-uniform): a.max_steps (<= KMAX),
    // fewer for a batch instance that reaches its step limit, none for one
    // that has (it carries its nodes over).
    const int64_t s0 = a.step + (a.step_base ? *a.step_base : 0);
    int kdo = min(a.max_steps, KMAX);  // the window holds KMAX steps
    if constexpr (BATCH) kdo = (int)max((int64_t)0, min((int64_t)kdo, in.stop - s0));
    if (kdo <= 0) {
        for (int k = t; k < sn; k += BX) carry_node(src, dst, P, 3, x0 + k);
        return;
    }

    // Window [wl, wl + L) in lattice coordinates (mod n when periodic).
    const int wl = wrap ? x0 - KMAX : max(0, x0 - KMAX);
    const int wr = wrap ? x0 + sn + KMAX : min(n, x0 + sn + KMAX);
    const int L = wr - wl;
    const bool lend = !wrap && wl == 0;  // the window's left end is the lattice's
    const bool rend = !wrap && wr == n;
    auto lattice_x = [&](int w) {
        int x = wl + w;
        if (wrap) x = ((x % n) + n) % n;
        return x;
    };
    for (int w = t; w < L; w += BX) {
        const int x = lattice_x(w);
#pragma unroll
        for (int q = 0; q < 3; ++q) b0[q * W + w] = ldraw<T, (NT & 1) != 0>(src + q * P + x);
    }
    const C r0 = C(2.0 / 3.0) * C(in.rho0), r1 = C(1.0 / 6.0) * C(in.rho0);
    const C omega = C(in.omega);
    const int own0 = x0 - wl;  // window index of the first own node
    uint64_t first_bad = ~0ull;
    T *cur = b0, *nxt = b1;
    for (int s = 1; s <= kdo; ++s) {
        lds_barrier();
        const int lo = lend ? 0 : s, hi = rend ? L : L - s;
        for (int w = lo + t; w < hi; w += BX) {
            const int wm = (lend && w == 0) ? w : w - 1;
            const int wp = (rend && w == L - 1) ? w : w + 1;
            C f0 = load<ST>(&cur[w], r0, a.fp16_iscale);
            C fp = load<ST>(&cur[W + wm], r1, a.fp16_iscale);
            C fm = load<ST>(&cur[2 * W + wp], r1, a.fp16_iscale);
            // Walls exist only without wrap, where lattice x = wl + w.
            const int role = (!wrap && (wl + w == 0 || wl + w == n - 1)) ? R_WALL : R_FLUID;
            const int fl = node3<C>(f0, fp, fm, role, omega);
            if (fl && w >= own0 && w < own0 + sn) {
                const uint64_t key = event_key(s0 + s - 1, x0 + (w - own0));
                first_bad = key < first_bad ? key : first_bad;
            }
            nxt[w] = to_storage<ST>(f0, r0, a.fp16_scale);
            nxt[W + w] = to_storage<ST>(fp, r1, a.fp16_scale);
            nxt[2 * W + w] = to_storage<ST>(fm, r1, a.fp16_scale);
        }
        T *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    lds_barrier();
    for (int k = t; k < sn; k += BX) {
        const int w = own0 + k;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if constexpr ((NT & 2) != 0) __builtin_nontemporal_store(cur[q * W + w], dst + q * P + x0 + k);
            else dst[q * P + x0 + k] = cur[q * W + w];
        }
    }
    report_key(status, first_bad);
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------

namespace {

struct Shape {
    int bx, by, rpt, swz;
    const char *name;
    int steps = 1;  // steps per launch
};

// Launch shapes of the single-lattice D2Q9 kernel.  Every shape computes the
// same per-node arithmetic, so results are bitwise identical.
constexpr Shape kShapes[] = {
    {256, 1, 1, 0, "256x1 rows=1 linear"},
    {256, 1, 1, 1, "256x1 rows=1 xcd"},
    {64, 4, 1, 1, "64x4 rows=1 xcd"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load nt-store"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-store"},
    {256, 1, 1, 1, "256x1 rows=1 xcd nt-load nt-store"},
    {256, -1, 4, 1, "256 rows=4 pipelined xcd nt-load nt-store"},
    {64, 4, 2, 1, "64x4 rows=2 xcd nt-load nt-store"},
    {256, -1, 2, 1, "256 rows=2 pipelined xcd nt-load"},
    {128, -1, 4, 1, "128 rows=4 pipelined xcd nt-store"},
    {256, 1, 2, 1, "256x1 rows=2 xcd nt-load nt-store"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load nt-store waves>=6"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load nt-store waves>=8"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-store waves>=6"},
    {256, 1, 1, 1, "256x1 rows=1 xcd nt-load nt-store waves>=6"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load nt-store waves>=7"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load"},
    {128, 1, 1, 0, "128x1 rows=1 linear nt-load nt-store"},
    {512, 1, 1, 0, "512x1 rows=1 linear nt-load nt-store"},
    {256, -2, 1, 0, "256 LDS-staged rows=1 linear nt-store"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load(unshifted planes) nt-store"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load(unshifted planes) nt-store waves>=6"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load(unshifted planes) nt-store waves>=8"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load(unshifted planes) nt-store prio"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load(unshifted planes) nt-store waves>=6 prio"},
    {256, 1, 1, 0, "256x1 rows=1 linear nt-load(unshifted planes) nt-store waves>=8 prio"},
    {256, 32, 1, 0, "two steps per launch, 256x32 tiles, nt-load(unshifted planes) nt-store", 2},
    {256, 16, 1, 0, "two steps per launch, 256x16 tiles, nt-load(unshifted planes) nt-store", 2},
    {256, 64, 1, 0, "two steps per launch, 256x64 tiles, nt-load(unshifted planes) nt-store", 2},
    {128, 32, 1, 0, "two steps per launch, 128x32 tiles, nt-load(unshifted planes) nt-store", 2},
    {512, 32, 1, 0, "two steps per launch, 512x32 tiles, nt-load(unshifted planes) nt-store", 2},
    {256, 32, 1, 0, "two steps per launch, 256x32 tiles, nt-store", 2},
    {256, 16, 1, 0, "two steps per launch, 256x16 tiles, 3-row ring, nt-load(unshifted planes) nt-store", 2},
    {256, 16, 1, 0, "two steps per launch, 256x16 tiles, 3-row ring, nt-load(unshifted planes) nt-store waves>=5", 2},
    {128, 16, 1, 0, "two steps per launch, 128x16 tiles, 3-row ring, nt-load(unshifted planes) nt-store waves>=5", 2},
    {256, 24, 1, 0, "two steps per launch, 256x24 tiles, 3-row ring, nt-load(unshifted planes) nt-store waves>=5", 2},
    {512, 16, 1, 0, "two steps per launch, 512x16 tiles, nt-load(unshifted planes) nt-store", 2},
    {256, 16, 1, 0, "two steps per launch, 256x16 tiles, split rings, nt-load(unshifted planes) nt-store", 2},
    {256, 32, 1, 0, "two steps per launch, 256x32 tiles, split rings, nt-load(unshifted planes) nt-store", 2},
    {256, 16, 1, 0, "two steps per launch, 256x16 tiles, split rings, nt-load(unshifted planes) nt-store waves>=4", 2},
    {256, 32, 1, 0, "two steps per launch, 256x32 tiles, split rings, nt-load(unshifted planes) nt-store waves>=4", 2},
    {512, 32, 1, 0, "two steps per launch, 512x32 tiles, split rings, nt-load(unshifted planes) nt-store waves>=4", 2},
    {1024, 32, 1, 0, "two steps per launch, 1024x32 tiles, split rings, nt-load(unshifted planes) nt-store waves>=4", 2},
};

constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
constexpr int kMaxGridY = 65535;  // grid y limit; larger tile counts use a 1D grid
constexpr int kNumShapesOther = 3;  // the other collision rules instantiate the first three

template <int ST, int CO, int BX, int BY, int RPT, int NT = 0, int WPE = 0>
hipError_t go9(const void *src, void *dst, StepArgs a, int swz, hipStream_t s)
{
    using T = typename Form<ST>::T;
    const int tiles_x = (a.one.nx + BX - 1) / BX;
    const int tiles_y = (a.one.ny + BY * RPT - 1) / (BY * RPT);
    a.tiles_x = tiles_x;
    a.xcd_swizzle = swz;
    const dim3 grid = tiles_y <= kMaxGridY ? dim3(tiles_x, tiles_y) : dim3(tiles_x * tiles_y);
    hipLaunchKernelGGL((k_d2q9<ST, CO, BX, BY, RPT, NT, WPE>), grid, dim3(BX, BY), 0, s,
                       (const T *)src, (T *)dst, a);
    return hipGetLastError();
}

template <int ST, int CO, int BX, int RY, int NT = 0>
hipError_t go9st(const void *src, void *dst, StepArgs a, int swz, hipStream_t s)
{
    using T = typename Form<ST>::T;
    const int tiles_x = (a.one.nx + BX - 1) / BX;
    const int tiles_y = (a.one.ny + RY - 1) / RY;
    a.tiles_x = tiles_x;
    a.xcd_swizzle = swz;
    const dim3 grid = tiles_y <= kMaxGridY ? dim3(tiles_x, tiles_y) : dim3(tiles_x * tiles_y);
    hipLaunchKernelGGL((k_d2q9_stage<ST, CO, BX, RY, NT>), grid, dim3(BX), 0, s, (const T *)src, (T *)dst, a);
    return hipGetLastError();
}

template <int ST, int CO, int BX, int RPT, int NT = 0, int WPE = 0>
hipError_t go9pf(const void *src, void *dst, StepArgs a, int swz, hipStream_t s)
{
    using T = typename Form<ST>::T;
    const int tiles_x = (a.one.nx + BX - 1) / BX;
    const int tiles_y = (a.one.ny + RPT - 1) / RPT;
    a.tiles_x = tiles_x;
    a.xcd_swizzle = swz;
    const dim3 grid = tiles_y <= kMaxGridY ? dim3(tiles_x, tiles_y) : dim3(tiles_x * tiles_y);
    hipLaunchKernelGGL((k_d2q9_pf<ST, CO, BX, RPT, NT, WPE>), grid, dim3(BX), 0, s,
                       (const T *)src, (T *)dst, a);
    return hipGetLastError();
}

template <int ST, int CO, int BX, int H, int RS, int NT = 0, int WPE = 0>
hipError_t go9t2(const void *src, void *dst, StepArgs a, int swz, hipStream_t s)
{
    using T = typename Form<ST>::T;
    const int tiles_x = (a.one.nx + BX - 1) / BX;
    const int tiles_y = (a.one.ny + H - 1) / H;
    a.tiles_x = tiles_x;
    a.xcd_swizzle = swz;
    const dim3 grid = tiles_y <= kMaxGridY ? dim3(tiles_x, tiles_y) : dim3(tiles_x * tiles_y);
    hipLaunchKernelGGL((k_d2q9_t2<ST, CO, BX, H, RS, NT, WPE>), grid, dim3(BX), t2_lds_bytes<T>(BX, H, RS), s,
                       (const T *)src, (T *)dst, a);
    return hipGetLastError();
}

// LDS beyond the default 64 KiB must be allowed per kernel before launch
// (outside any stream capture): the FP64 two-step tiles need it.
template <int ST, int CO, int BX, int H, int RS, int NT = 0, int WPE = 0>
hipError_t prep9t2()
{
    using T = typename Form<ST>::T;
    constexpr size_t b = t2_lds_bytes<T>(BX, H, RS);
    if (b <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k_d2q9_t2<ST, CO, BX, H, RS, NT, WPE>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
}

// Two-step shapes of the single-lattice kernel (MinxEnt4): launch, or with
// `prep` only set the kernel's LDS limit.
template <int ST, int CO>
hipError_t dispatch9t2(int v, bool prep, const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
#define LBM_T2(BX, H, RS, NT, WPE)                                                            \
    return prep ? prep9t2<ST, CO, BX, H, RS, NT, WPE>()                                       \
                : go9t2<ST, CO, BX, H, RS, NT, WPE>(src, dst, a, kShapes[v].swz, s)
    switch (v) {
    case 26: LBM_T2(256, 32, 4, 6, 0);
    case 27: LBM_T2(256, 16, 4, 6, 0);
    case 28: LBM_T2(256, 64, 4, 6, 0);
    case 29: LBM_T2(128, 32, 4, 6, 0);
    case 30: LBM_T2(512, 32, 4, 6, 0);
    case 31: LBM_T2(256, 32, 4, 2, 0);
    case 32: LBM_T2(256, 16, 3, 6, 0);
    case 33: LBM_T2(256, 16, 3, 6, 5);
    case 34: LBM_T2(128, 16, 3, 6, 5);
    case 35: LBM_T2(256, 24, 3, 6, 5);
    case 36: LBM_T2(512, 16, 4, 6, 0);
    case 37: LBM_T2(256, 16, 0, 6, 0);
    case 38: LBM_T2(256, 32, 0, 6, 0);
    case 39: LBM_T2(256, 16, 0, 6, 4);
    case 40: LBM_T2(256, 32, 0, 6, 4);
    case 41: LBM_T2(512, 32, 0, 6, 4);
    case 42: LBM_T2(1024, 32, 0, 6, 4);
    default: return hipErrorInvalidValue;
    }
#undef LBM_T2
}

template <int ST, int CO>
hipError_t dispatch9(int v, const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    const int swz = kShapes[v].swz;
    switch (v) {
    case 0: return go9<ST, CO, 256, 1, 1>(src, dst, a, swz, s);
    case 1: return go9<ST, CO, 256, 1, 1>(src, dst, a, swz, s);
    case 2: return go9<ST, CO, 64, 4, 1>(src, dst, a, swz, s);
    default: break;
    }
    if constexpr (CO == CO_MINXENT4) {
        switch (v) {
        case 3: return go9<ST, CO, 256, 1, 1, 3>(src, dst, a, swz, s);
        case 4: return go9<ST, CO, 256, 1, 1, 2>(src, dst, a, swz, s);
        case 5: return go9<ST, CO, 256, 1, 1, 3>(src, dst, a, swz, s);
        case 6: return go9pf<ST, CO, 256, 4, 3>(src, dst, a, swz, s);
        case 7: return go9<ST, CO, 64, 4, 2, 3>(src, dst, a, swz, s);
        case 8: return go9pf<ST, CO, 256, 2, 1>(src, dst, a, swz, s);
        case 9: return go9pf<ST, CO, 128, 4, 2>(src, dst, a, swz, s);
        case 10: return go9<ST, CO, 256, 1, 2, 3>(src, dst, a, swz, s);
        case 11: return go9<ST, CO, 256, 1, 1, 3, 6>(src, dst, a, swz, s);
        case 12: return go9<ST, CO, 256, 1, 1, 3, 8>(src, dst, a, swz, s);
        case 13: return go9<ST, CO, 256, 1, 1, 2, 6>(src, dst, a, swz, s);
        case 14: return go9<ST, CO, 256, 1, 1, 3, 6>(src, dst, a, swz, s);
        case 15: return go9<ST, CO, 256, 1, 1, 3, 7>(src, dst, a, swz, s);
        case 16: return go9<ST, CO, 256, 1, 1, 1>(src, dst, a, swz, s);
        case 17: return go9<ST, CO, 128, 1, 1, 3>(src, dst, a, swz, s);
        case 18: return go9<ST, CO, 512, 1, 1, 3>(src, dst, a, swz, s);
        case 19: return go9st<ST, CO, 256, 1, 2>(src, dst, a, swz, s);
        case 20: return go9<ST, CO, 256, 1, 1, 6>(src, dst, a, swz, s);
        case 21: return go9<ST, CO, 256, 1, 1, 6, 6>(src, dst, a, swz, s);
        case 22: return go9<ST, CO, 256, 1, 1, 6, 8>(src, dst, a, swz, s);
        case 23: return go9<ST, CO, 256, 1, 1, 14>(src, dst, a, swz, s);
        case 24: return go9<ST, CO, 256, 1, 1, 14, 6>(src, dst, a, swz, s);
        case 25: return go9<ST, CO, 256, 1, 1, 14, 8>(src, dst, a, swz, s);
        default: return dispatch9t2<ST, CO>(v, false, src, dst, a, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int ST>
hipError_t dispatch9c(int coll, int v, const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    switch (coll) {
    case CO_MINXENT4: return dispatch9<ST, CO_MINXENT4>(v, src, dst, a, s);
    case CO_MINXENT2: return dispatch9<ST, CO_MINXENT2>(v, src, dst, a, s);
    case CO_SRT: return dispatch9<ST, CO_SRT>(v, src, dst, a, s);
    case CO_TRT: return dispatch9<ST, CO_TRT>(v, src, dst, a, s);
    case CO_MRT: return dispatch9<ST, CO_MRT>(v, src, dst, a, s);
    default: return hipErrorInvalidValue;
    }
}


// Two-step batch shapes: one block per tile of the tile table (a.ntiles).
template <int ST, int CO, int BX, int H, int RS, int NT = 0, int WPE = 0>
hipError_t go9bt2(const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    using T = typename Form<ST>::T;
    hipLaunchKernelGGL((k_d2q9_t2<ST, CO, BX, H, RS, NT, WPE, true>), dim3(a.ntiles), dim3(BX),
                       t2_lds_bytes<T>(BX, H, RS), s, (const T *)src, (T *)dst, a);
    return hipGetLastError();
}

template <int ST, int CO, int BX, int H, int RS, int NT = 0, int WPE = 0>
hipError_t prep9bt2()
{
    using T = typename Form<ST>::T;
    constexpr size_t b = t2_lds_bytes<T>(BX, H, RS);
    if (b <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k_d2q9_t2<ST, CO, BX, H, RS, NT, WPE, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
}

// Wave-tiled two-step batch shapes: WT waves per block, one 64-column tile
// each.
template <int ST, int CO, int H, int RS, int NT, int WT>
hipError_t go9bt2w(const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    using T = typename Form<ST>::T;
    const int blocks = (a.ntiles + WT - 1) / WT;
    hipLaunchKernelGGL((k_d2q9_t2<ST, CO, 64, H, RS, NT, 0, true, WT>), dim3(blocks), dim3(64 * WT),
                       WT * t2_wave_lds_bytes<T>(H, RS), s, (const T *)src, (T *)dst, a);
    return hipGetLastError();
}

template <int ST, int CO, int H, int RS, int NT, int WT>
hipError_t prep9bt2w()
{
    using T = typename Form<ST>::T;
    constexpr size_t b = WT * t2_wave_lds_bytes<T>(H, RS);
    if (b <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k_d2q9_t2<ST, CO, 64, H, RS, NT, 0, true, WT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
}

// Two-step batch shapes 17-20 are 9, 14, 15 and 10 with the tile table read
// in XCD-banded order: block b takes the tile xcd_remap(b), so each XCD works
// through a contiguous band of the table and horizontally adjacent tiles (and,
// in narrow instances, vertically adjacent ones) share its L2, which serves
// the window lines they have in common.
constexpr int banded_base(int v) { return v == 17 ? 9 : v == 18 ? 14 : v == 19 ? 15 : v == 20 ? 10 : v; }

template <int ST, int CO>
hipError_t dispatch9bt2(int v, bool prep, const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    v = banded_base(v);
#define LBM_BT2W(H, RS, NT, WT) return prep ? prep9bt2w<ST, CO, H, RS, NT, WT>() : go9bt2w<ST, CO, H, RS, NT, WT>(src, dst, a, s)
    switch (v) {
    case 12: LBM_BT2W(16, 3, 6, 4);
    case 13: LBM_BT2W(16, 0, 6, 4);
    default: break;
    }
#undef LBM_BT2W
#define LBM_BT2(BX, H, RS, NT) return prep ? prep9bt2<ST, CO, BX, H, RS, NT>() : go9bt2<ST, CO, BX, H, RS, NT>(src, dst, a, s)
#define LBM_BT2B(BX, H, RS, NT, WPE) \
    return prep ? prep9bt2<ST, CO, BX, H, RS, NT, WPE>() : go9bt2<ST, CO, BX, H, RS, NT, WPE>(src, dst, a, s)
    switch (v) {
    case 9: LBM_BT2(64, 16, 3, 6);
    case 10: LBM_BT2(64, 16, 0, 6);
    case 11: LBM_BT2(256, 16, 4, 6);
    case 14: LBM_BT2(256, 16, 3, 6);
    case 15: LBM_BT2(256, 16, 0, 6);
    case 16: LBM_BT2B(256, 16, 3, 6, 5);
    case 21: LBM_BT2(128, 16, 3, 6);
    case 22: LBM_BT2(128, 16, 0, 6);
    default: return hipErrorInvalidValue;
    }
#undef LBM_BT2
#undef LBM_BT2B
}

template <int ST, int CO>
hipError_t dispatch9b(int v, const void *src, void *dst, const StepArgs &a_in, hipStream_t s)
{
    using T = typename Form<ST>::T;
    // Tiles run in launch order; shapes 5 and 6 are 3 and 4 with tiles in
    // XCD-banded order instead (measured slower, kept as candidates), and so
    // are the two-step shapes 17-20 (of 9, 14, 15 and 10).
    StepArgs a = a_in;
    a.xcd_swizzle = 0;
    if (v == 5 || v == 6) {
        a.xcd_swizzle = 1;
        v -= 2;
    }
    if (banded_base(v) != v) {
        a.xcd_swizzle = 1;
        v = banded_base(v);
    }
    switch (v) {
    case 0: hipLaunchKernelGGL((k_d2q9_batch<ST, CO, 256, 0>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 1: hipLaunchKernelGGL((k_d2q9_batch<ST, CO, 128, 0>), dim3(a.ntiles), dim3(128), 0, s, (const T *)src, (T *)dst, a); break;
    case 2: hipLaunchKernelGGL((k_d2q9_batch<ST, CO, 256, 3>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 3: hipLaunchKernelGGL((k_d2q9_batch<ST, CO, 256, 2>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 4: hipLaunchKernelGGL((k_d2q9_batch<ST, CO, 256, 6>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 7: hipLaunchKernelGGL((k_d2q9_batch<ST, CO, 256, 10>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 8: hipLaunchKernelGGL((k_d2q9_batch<ST, CO, 256, 14>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    default:
        if constexpr (CO == CO_MINXENT4) return dispatch9bt2<ST, CO>(v, false, src, dst, a, s);
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int ST>
hipError_t dispatch9bc(int coll, int v, const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    switch (coll) {
    case CO_MINXENT4: return dispatch9b<ST, CO_MINXENT4>(v, src, dst, a, s);
    case CO_MINXENT2: return dispatch9b<ST, CO_MINXENT2>(v, src, dst, a, s);
    case CO_SRT: return dispatch9b<ST, CO_SRT>(v, src, dst, a, s);
    case CO_TRT: return dispatch9b<ST, CO_TRT>(v, src, dst, a, s);
    case CO_MRT: return dispatch9b<ST, CO_MRT>(v, src, dst, a, s);
    default: return hipErrorInvalidValue;
    }
}

struct Shape3 {
    int bx, npt;
    const char *name;
    int steps = 1;  // steps per launch (at most)
};
constexpr Shape3 kShapes3[] = {
    {256, 1, "256 nodes=1"},
    {256, 4, "256 nodes=4"},
    {512, 2, "512 nodes=2"},
    {128, 4, "128 nodes=4"},
    {256, 4, "256 nodes=4 nt-load nt-store"},
    {256, 8, "256 groups of 8 nodes, 16-byte vectors"},
    {256, 8, "256 groups of 8 nodes, 16-byte vectors nt-load nt-store"},
    {128, 8, "128 groups of 8 nodes, 16-byte vectors nt-load nt-store"},
    {256, 4, "1024-node segments in LDS, up to 16 steps per launch", 16},
    {256, 4, "1024-node segments in LDS, up to 32 steps per launch, nt-load nt-store", 32},
    {256, 4, "1024-node segments in LDS, up to 64 steps per launch, nt-load nt-store", 64},
    {128, 8, "1024-node segments in LDS (128 threads), up to 32 steps per launch, nt-load nt-store", 32},
    {256, 4, "1024-node segments in LDS, up to 256 steps per launch, nt-load nt-store", 256},
    {1024, 1, "1024-node segments in LDS (1024 threads), up to 256 steps per launch, nt-load nt-store", 256},
};
constexpr int kNumShapes3 = sizeof(kShapes3) / sizeof(kShapes3[0]);

// K-step D1Q3 launches: one block per S-node segment (a single lattice's
// segments in order, or a batch's tile table).
template <int ST, int BX, int NPT, int KMAX, int NT, bool BATCH>
hipError_t go3tk(const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    using T = typename Form<ST>::T;
    constexpr int S = BX * NPT;
    const int blocks = BATCH ? a.ntiles : (a.one.nx + S - 1) / S;
    hipLaunchKernelGGL((k_d1q3_tk<ST, BX, NPT, KMAX, NT, BATCH>), dim3(blocks), dim3(BX), tk_lds_bytes<T>(S, KMAX), s,
                       (const T *)src, (T *)dst, a);
    return hipGetLastError();
}

// LDS beyond the default 64 KiB must be allowed before the first launch
// (outside any stream capture): the 256-step window in FP64 needs it.
template <int ST, int BX, int NPT, int KMAX, int NT, bool BATCH>
hipError_t prep3tk()
{
    using T = typename Form<ST>::T;
    constexpr size_t b = tk_lds_bytes<T>(BX * NPT, KMAX);
    if (b <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k_d1q3_tk<ST, BX, NPT, KMAX, NT, BATCH>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
}

template <int ST, bool BATCH>
hipError_t dispatch3tk(int k, const void *src, void *dst, const StepArgs &a, hipStream_t s, bool prep = false)
{
#define LBM_TK(BX, NPT, K, NT) \
    return prep ? prep3tk<ST, BX, NPT, K, NT, BATCH>() : go3tk<ST, BX, NPT, K, NT, BATCH>(src, dst, a, s)
    switch (k) {
    case 0: LBM_TK(256, 4, 16, 0);
    case 1: LBM_TK(256, 4, 32, 3);
    case 2: LBM_TK(256, 4, 64, 3);
    case 3: LBM_TK(128, 8, 32, 3);
    case 4: LBM_TK(256, 4, 256, 3);
    case 5: LBM_TK(1024, 1, 256, 3);
    default: return hipErrorInvalidValue;
    }
#undef LBM_TK
}

template <int ST, int BX, int NT = 0>
hipError_t go3v(const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    using T = typename Form<ST>::T;
    const int groups = (a.one.nx + 7) / 8;
    hipLaunchKernelGGL((k_d1q3_v8<ST, BX, NT>), dim3((groups + BX - 1) / BX), dim3(BX), 0, s, (const T *)src,
                       (T *)dst, a);
    return hipGetLastError();
}

template <int ST, int BX, int NPT, int NT = 0>
hipError_t go3(const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    using T = typename Form<ST>::T;
    const int blocks = (a.one.nx + BX * NPT - 1) / (BX * NPT);
    hipLaunchKernelGGL((k_d1q3<ST, BX, NPT, NT>), dim3(blocks), dim3(BX), 0, s, (const T *)src, (T *)dst, a);
    return hipGetLastError();
}

template <int ST>
hipError_t dispatch3(int v, const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    switch (v) {
    case 0: return go3<ST, 256, 1>(src, dst, a, s);
    case 1: return go3<ST, 256, 4>(src, dst, a, s);
    case 2: return go3<ST, 512, 2>(src, dst, a, s);
    case 3: return go3<ST, 128, 4>(src, dst, a, s);
    case 4: return go3<ST, 256, 4, 3>(src, dst, a, s);
    case 5: return go3v<ST, 256>(src, dst, a, s);
    case 6: return go3v<ST, 256, 3>(src, dst, a, s);
    case 7: return go3v<ST, 128, 3>(src, dst, a, s);
    default: return dispatch3tk<ST, false>(v - 8, src, dst, a, s);
    }
}

// Batched launch shapes: D2Q9 tiles of 256 or 128 nodes (one per thread);
// D1Q3 tiles of BLK x NPT nodes.
struct ShapeB {
    int blk, npt;
    const char *name;
    int steps = 1;  // steps per launch
    int rows = 0;   // two-step shapes: tile rows (tiles are blk x rows nodes of one instance)
};
constexpr ShapeB kShapesB9[] = {{256, 1, "batch 256 nodes/block"}, {128, 1, "batch 128 nodes/block"},
                                {256, 1, "batch 256 nodes/block nt-load nt-store"},
                                {256, 1, "batch 256 nodes/block nt-store"},
                                {256, 1, "batch 256 nodes/block nt-load(unshifted planes) nt-store"},
                                {256, 1, "batch 256 nodes/block nt-store, XCD-banded"},
                                {256, 1, "batch 256 nodes/block nt-load(unshifted planes) nt-store, XCD-banded"},
                                {256, 1, "batch 256 nodes/block nt-store prio"},
                                {256, 1, "batch 256 nodes/block nt-load(unshifted planes) nt-store prio"},
                                // two steps per launch (MinxEnt4 only)
                                {64, 1, "batch two steps per launch, 64x16 tiles, 3-row ring, nt-load(unshifted planes) nt-store", 2, 16},
                                {64, 1, "batch two steps per launch, 64x16 tiles, split rings, nt-load(unshifted planes) nt-store", 2, 16},
                                {256, 1, "batch two steps per launch, 256x16 tiles, nt-load(unshifted planes) nt-store", 2, 16},
                                {64, 1, "batch two steps per launch, 64x16 tiles one per wave (4 waves/block), 3-row ring, nt-load(unshifted planes) nt-store", 2, 16},
                                {64, 1, "batch two steps per launch, 64x16 tiles one per wave (4 waves/block), split rings, nt-load(unshifted planes) nt-store", 2, 16},
                                {256, 1, "batch two steps per launch, 256x16 tiles, 3-row ring, nt-load(unshifted planes) nt-store", 2, 16},
                                {256, 1, "batch two steps per launch, 256x16 tiles, split rings, nt-load(unshifted planes) nt-store", 2, 16},
                                {256, 1, "batch two steps per launch, 256x16 tiles, 3-row ring, nt-load(unshifted planes) nt-store waves>=5", 2, 16},
                                // 9, 14, 15 and 10 with tiles in XCD-banded order
                                {64, 1, "batch two steps per launch, 64x16 tiles, 3-row ring, nt-load(unshifted planes) nt-store, XCD-banded", 2, 16},
                                {256, 1, "batch two steps per launch, 256x16 tiles, 3-row ring, nt-load(unshifted planes) nt-store, XCD-banded", 2, 16},
                                {256, 1, "batch two steps per launch, 256x16 tiles, split rings, nt-load(unshifted planes) nt-store, XCD-banded", 2, 16},
                                {64, 1, "batch two steps per launch, 64x16 tiles, split rings, nt-load(unshifted planes) nt-store, XCD-banded", 2, 16},
                                {128, 1, "batch two steps per launch, 128x16 tiles, 3-row ring, nt-load(unshifted planes) nt-store", 2, 16},
                                {128, 1, "batch two steps per launch, 128x16 tiles, split rings, nt-load(unshifted planes) nt-store", 2, 16}};
// Single-step batch shapes (every collision rule); the rest of kShapesB9 are
// two-step shapes of MinxEnt4.
constexpr int kNumB9One = 9;
constexpr ShapeB kShapesB3[] = {{256, 1, "batch 256x1 nodes/block"}, {128, 1, "batch 128x1 nodes/block"},
                                {256, 4, "batch 256x4 nodes/block"}, {256, 8, "batch 256x8 nodes/block"},
                                {256, 4, "batch 256x4 nodes/block nt-load nt-store"},
                                {256, 8, "batch 256 groups of 8 nodes, 16-byte vectors"},
                                {256, 8, "batch 256 groups of 8 nodes, 16-byte vectors nt-load nt-store"},
                                {128, 8, "batch 128 groups of 8 nodes, 16-byte vectors nt-load nt-store"},
                                {128, 1, "batch 128x1 nodes/block, XCD-banded"},
                                {256, 8, "batch 256 groups of 8 nodes, 16-byte vectors, XCD-banded"},
                                {256, 4, "batch 1024-node segments in LDS, up to 16 steps per launch", 16},
                                {256, 4, "batch 1024-node segments in LDS, up to 32 steps per launch, nt-load nt-store", 32},
                                {256, 4, "batch 1024-node segments in LDS, up to 64 steps per launch, nt-load nt-store", 64},
                                {128, 8, "batch 1024-node segments in LDS (128 threads), up to 32 steps per launch, nt-load nt-store", 32},
                                {256, 4, "batch 1024-node segments in LDS, up to 256 steps per launch, nt-load nt-store", 256},
                                {1024, 1, "batch 1024-node segments in LDS (1024 threads), up to 256 steps per launch, nt-load nt-store", 256}};

template <int ST>
hipError_t dispatch3b(int v, const void *src, void *dst, const StepArgs &a_in, hipStream_t s)
{
    using T = typename Form<ST>::T;
    // Tiles run in launch order; shapes 8 and 9 are 1 and 5 with tiles in
    // XCD-banded order instead (measured slower, kept as candidates); 10 on
    // take up to K steps per launch.
    StepArgs a = a_in;
    a.xcd_swizzle = 0;
    if (v >= 10) return dispatch3tk<ST, true>(v - 10, src, dst, a, s);
    if (v >= 8) {
        a.xcd_swizzle = 1;
        v = v == 8 ? 1 : 5;
    }
    switch (v) {
    case 0: hipLaunchKernelGGL((k_d1q3_batch<ST, 256, 1>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 1: hipLaunchKernelGGL((k_d1q3_batch<ST, 128, 1>), dim3(a.ntiles), dim3(128), 0, s, (const T *)src, (T *)dst, a); break;
    case 2: hipLaunchKernelGGL((k_d1q3_batch<ST, 256, 4>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 3: hipLaunchKernelGGL((k_d1q3_batch<ST, 256, 8>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 4: hipLaunchKernelGGL((k_d1q3_batch<ST, 256, 4, 3>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 5: hipLaunchKernelGGL((k_d1q3_batch_v8<ST, 256>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 6: hipLaunchKernelGGL((k_d1q3_batch_v8<ST, 256, 3>), dim3(a.ntiles), dim3(256), 0, s, (const T *)src, (T *)dst, a); break;
    case 7: hipLaunchKernelGGL((k_d1q3_batch_v8<ST, 128, 3>), dim3(a.ntiles), dim3(128), 0, s, (const T *)src, (T *)dst, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int ST>
hipError_t init_st(int lattice, const Inst &in, int bc, const double *r, const double *u, const double *w,
                   const double *f, void *buf, float scale, hipStream_t s)
{
    using T = typename Form<ST>::T;
    const int n = in.nx * in.ny;
    const int blocks = (n + 255) / 256;
    if (lattice == 9)
        hipLaunchKernelGGL((k_init<ST, 9>), dim3(blocks), dim3(256), 0, s, in, bc, r, u, w, f, (T *)buf, scale);
    else
        hipLaunchKernelGGL((k_init<ST, 3>), dim3(blocks), dim3(256), 0, s, in, bc, r, u, w, f, (T *)buf, scale);
    return hipGetLastError();
}

template <int ST>
hipError_t gather_st(int lattice, const Inst &in, int bc, const void *buf, double *r, double *u, double *w,
                     double *f, float iscale, hipStream_t s)
{
    using T = typename Form<ST>::T;
    const int n = in.nx * in.ny;
    const int blocks = (n + 255) / 256;
    if (lattice == 9)
        hipLaunchKernelGGL((k_gather<ST, 9>), dim3(blocks), dim3(256), 0, s, in, bc, (const T *)buf, r, u, w, f, iscale);
    else
        hipLaunchKernelGGL((k_gather<ST, 3>), dim3(blocks), dim3(256), 0, s, in, bc, (const T *)buf, r, u, w, f, iscale);
    return hipGetLastError();
}

}  // namespace

int d2q9_variant_count(int coll) { return coll == CO_MINXENT4 ? kNumShapes : kNumShapesOther; }
int d2q9_variant_steps(int coll, int v)
{
    return (coll == CO_MINXENT4 && v >= 0 && v < kNumShapes) ? kShapes[v].steps : 1;
}

hipError_t prepare_d2q9_variant(int st, int coll, int v)
{
    if (d2q9_variant_steps(coll, v) != 2) return hipSuccess;
    const StepArgs none{};
    switch (st) {
    case ST_F64: return dispatch9t2<ST_F64, CO_MINXENT4>(v, true, nullptr, nullptr, none, nullptr);
    case ST_F32N64: return dispatch9t2<ST_F32N64, CO_MINXENT4>(v, true, nullptr, nullptr, none, nullptr);
    case ST_F32: return dispatch9t2<ST_F32, CO_MINXENT4>(v, true, nullptr, nullptr, none, nullptr);
    case ST_F16DEV: return dispatch9t2<ST_F16DEV, CO_MINXENT4>(v, true, nullptr, nullptr, none, nullptr);
    default: return hipErrorInvalidValue;
    }
}
const char *d2q9_variant_name(int v) { return (v >= 0 && v < kNumShapes) ? kShapes[v].name : "?"; }
int d1q3_variant_count() { return kNumShapes3; }
const char *d1q3_variant_name(int v) { return (v >= 0 && v < kNumShapes3) ? kShapes3[v].name : "?"; }
constexpr int kNumB9 = sizeof(kShapesB9) / sizeof(kShapesB9[0]);
constexpr int kNumB3 = sizeof(kShapesB3) / sizeof(kShapesB3[0]);
int batch_variant_count(int lattice, int coll)
{
    if (lattice == 3) return kNumB3;
    return coll == CO_MINXENT4 ? kNumB9 : kNumB9One;
}
int batch_variant_steps(int lattice, int v)
{
    if (lattice == 3) return (v >= 0 && v < kNumB3) ? kShapesB3[v].steps : 1;
    return (v >= 0 && v < kNumB9) ? kShapesB9[v].steps : 1;
}
int d1q3_variant_steps(int v) { return (v >= 0 && v < kNumShapes3) ? kShapes3[v].steps : 1; }

hipError_t prepare_d1q3_variant(int st, int batch, int v)
{
    const int k = v - (batch ? 10 : 8);  // index among the K-step shapes
    if (k < 0) return hipSuccess;
    const StepArgs none{};
    switch (st) {
    case ST_F64: return batch ? dispatch3tk<ST_F64, true>(k, nullptr, nullptr, none, nullptr, true)
                              : dispatch3tk<ST_F64, false>(k, nullptr, nullptr, none, nullptr, true);
    case ST_F32N64: return batch ? dispatch3tk<ST_F32N64, true>(k, nullptr, nullptr, none, nullptr, true)
                                 : dispatch3tk<ST_F32N64, false>(k, nullptr, nullptr, none, nullptr, true);
    case ST_F32: return batch ? dispatch3tk<ST_F32, true>(k, nullptr, nullptr, none, nullptr, true)
                              : dispatch3tk<ST_F32, false>(k, nullptr, nullptr, none, nullptr, true);
    case ST_F16DEV: return batch ? dispatch3tk<ST_F16DEV, true>(k, nullptr, nullptr, none, nullptr, true)
                                 : dispatch3tk<ST_F16DEV, false>(k, nullptr, nullptr, none, nullptr, true);
    default: return hipErrorInvalidValue;
    }
}
int batch_tile_nodes(int lattice, int v)
{
    if (lattice == 3) return (v >= 0 && v < kNumB3) ? kShapesB3[v].blk * kShapesB3[v].npt : 0;
    if (v < 0 || v >= kNumB9) return 0;
    if (kShapesB9[v].steps == 2) return -(kShapesB9[v].blk * 4096 + kShapesB9[v].rows);
    return kShapesB9[v].blk * kShapesB9[v].npt;
}
hipError_t prepare_batch_variant(int st, int coll, int v)
{
    if (coll != CO_MINXENT4 || batch_variant_steps(9, v) != 2) return hipSuccess;
    const StepArgs none{};
    switch (st) {
    case ST_F64: return dispatch9bt2<ST_F64, CO_MINXENT4>(v, true, nullptr, nullptr, none, nullptr);
    case ST_F32N64: return dispatch9bt2<ST_F32N64, CO_MINXENT4>(v, true, nullptr, nullptr, none, nullptr);
    case ST_F32: return dispatch9bt2<ST_F32, CO_MINXENT4>(v, true, nullptr, nullptr, none, nullptr);
    case ST_F16DEV: return dispatch9bt2<ST_F16DEV, CO_MINXENT4>(v, true, nullptr, nullptr, none, nullptr);
    default: return hipErrorInvalidValue;
    }
}
const char *batch_variant_name(int lattice, int v)
{
    if (lattice == 3) return (v >= 0 && v < kNumB3) ? kShapesB3[v].name : "?";
    return (v >= 0 && v < kNumB9) ? kShapesB9[v].name : "?";
}

hipError_t launch_d2q9_step(int st, int coll, int v, const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    if (v < 0 || v >= d2q9_variant_count(coll)) return hipErrorInvalidValue;
    switch (st) {
    case ST_F64: return dispatch9c<ST_F64>(coll, v, src, dst, a, s);
    case ST_F32N64: return dispatch9c<ST_F32N64>(coll, v, src, dst, a, s);
    case ST_F32: return dispatch9c<ST_F32>(coll, v, src, dst, a, s);
    case ST_F16DEV: return dispatch9c<ST_F16DEV>(coll, v, src, dst, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_d2q9_batch_step(int st, int coll, int v, const void *src, void *dst, const StepArgs &a,
                                  hipStream_t s)
{
    if (v < 0 || v >= batch_variant_count(9, coll)) return hipErrorInvalidValue;
    switch (st) {
    case ST_F64: return dispatch9bc<ST_F64>(coll, v, src, dst, a, s);
    case ST_F32N64: return dispatch9bc<ST_F32N64>(coll, v, src, dst, a, s);
    case ST_F32: return dispatch9bc<ST_F32>(coll, v, src, dst, a, s);
    case ST_F16DEV: return dispatch9bc<ST_F16DEV>(coll, v, src, dst, a, s);
    default: return hipErrorInvalidValue;
    }
}

namespace {
template <int ST, int CO>
hipError_t lds_go(const void *src, void *dst, const StepArgs &a, int nsteps, int block, size_t smem, hipStream_t s)
{
    using T = typename Form<ST>::T;
    hipError_t e = hipFuncSetAttribute((const void *)k_d2q9_lds<ST, CO>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_d2q9_lds<ST, CO>), dim3(a.ntiles), dim3(block), smem, s, (const T *)src, (T *)dst, a,
                       nsteps);
    return hipGetLastError();
}

template <int ST>
hipError_t lds_coll(int coll, const void *src, void *dst, const StepArgs &a, int nsteps, int block, size_t smem,
                    hipStream_t s)
{
    switch (coll) {
    case CO_MINXENT4: return lds_go<ST, CO_MINXENT4>(src, dst, a, nsteps, block, smem, s);
    case CO_MINXENT2: return lds_go<ST, CO_MINXENT2>(src, dst, a, nsteps, block, smem, s);
    case CO_SRT: return lds_go<ST, CO_SRT>(src, dst, a, nsteps, block, smem, s);
    case CO_TRT: return lds_go<ST, CO_TRT>(src, dst, a, nsteps, block, smem, s);
    case CO_MRT: return lds_go<ST, CO_MRT>(src, dst, a, nsteps, block, smem, s);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_d2q9_lds(int st, int coll, const void *src, void *dst, const StepArgs &a, int nsteps, int block,
                           size_t smem, hipStream_t s)
{
    if (nsteps <= 0) return hipSuccess;
    switch (st) {
    case ST_F64: return lds_coll<ST_F64>(coll, src, dst, a, nsteps, block, smem, s);
    case ST_F32N64: return lds_coll<ST_F32N64>(coll, src, dst, a, nsteps, block, smem, s);
    case ST_F32: return lds_coll<ST_F32>(coll, src, dst, a, nsteps, block, smem, s);
    case ST_F16DEV: return lds_coll<ST_F16DEV>(coll, src, dst, a, nsteps, block, smem, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_d1q3_step(int st, int v, const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    switch (st) {
    case ST_F64: return dispatch3<ST_F64>(v, src, dst, a, s);
    case ST_F32N64: return dispatch3<ST_F32N64>(v, src, dst, a, s);
    case ST_F32: return dispatch3<ST_F32>(v, src, dst, a, s);
    case ST_F16DEV: return dispatch3<ST_F16DEV>(v, src, dst, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_d1q3_batch_step(int st, int v, const void *src, void *dst, const StepArgs &a, hipStream_t s)
{
    if (v < 0 || v >= batch_variant_count(3, 0)) return hipErrorInvalidValue;
    switch (st) {
    case ST_F64: return dispatch3b<ST_F64>(v, src, dst, a, s);
    case ST_F32N64: return dispatch3b<ST_F32N64>(v, src, dst, a, s);
    case ST_F32: return dispatch3b<ST_F32>(v, src, dst, a, s);
    case ST_F16DEV: return dispatch3b<ST_F16DEV>(v, src, dst, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(int lattice, int st, const Inst &in, int bc, const double *r, const double *u,
                       const double *w, const double *f, void *buf, float scale, hipStream_t s)
{
    switch (st) {
    case ST_F64: return init_st<ST_F64>(lattice, in, bc, r, u, w, f, buf, scale, s);
    case ST_F32N64: return init_st<ST_F32N64>(lattice, in, bc, r, u, w, f, buf, scale, s);
    case ST_F32: return init_st<ST_F32>(lattice, in, bc, r, u, w, f, buf, scale, s);
    case ST_F16DEV: return init_st<ST_F16DEV>(lattice, in, bc, r, u, w, f, buf, scale, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather(int lattice, int st, const Inst &in, int bc, const void *buf, double *r, double *u,
                         double *w, double *f, float iscale, hipStream_t s)
{
    switch (st) {
    case ST_F64: return gather_st<ST_F64>(lattice, in, bc, buf, r, u, w, f, iscale, s);
    case ST_F32N64: return gather_st<ST_F32N64>(lattice, in, bc, buf, r, u, w, f, iscale, s);
    case ST_F32: return gather_st<ST_F32>(lattice, in, bc, buf, r, u, w, f, iscale, s);
    case ST_F16DEV: return gather_st<ST_F16DEV>(lattice, in, bc, buf, r, u, w, f, iscale, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 256 * kCopyVec - 1) / (256 * kCopyVec);
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (u32x4 *)dst, (const u32x4 *)src, n);
    return hipGetLastError();
}

hipError_t launch_add_step_base(int64_t *b, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_base, dim3(1), dim3(64), 0, s, b, n, 1);
    return hipGetLastError();
}

hipError_t launch_set_step_base(int64_t *b, int64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_base, dim3(1), dim3(64), 0, s, b, v, 0);
    return hipGetLastError();
}

hipError_t launch_clear_status(DevStatus *st, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_status, dim3((n + 255) / 256), dim3(256), 0, s, st, n);
    return hipGetLastError();
}

}  // namespace lbm
