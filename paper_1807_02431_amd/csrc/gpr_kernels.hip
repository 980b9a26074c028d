// gpr_kernels.hip -- gfx950 kernels of the Gen.ParRep hot path.
//
// Two stepping paths share every arithmetic routine, so they give bit-identical results:
//   plain      : per step, k_integrate (B A O A of Eq. 1's BAOAB discretisation),
//                k_bonded, k_nonbonded (pair forces, the closing B kick, pair-list rebuild
//                when due); observables and state tests as separate launches;
//   persistent : k_persist advances one replica per workgroup for a whole check period,
//                with its positions and parameters resident in LDS and its velocities and
//                forces in registers.
// Gen.ParRep bookkeeping (Sec. 2.4.1 branching and Gelman-Rubin, Sec. 2.4.2 exit vote)
// runs in k_check / k_clone once per check.
#include "gpr_kernels.h"

namespace gpr {

// ------------------------------------------------------------------ small helpers
__device__ __forceinline__ float kick(float v, float F, float h, float im) { return v + (h * F) * im; }

__device__ __forceinline__ long long wave_sum_ll(long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// the P = 4 lanes of one atom are consecutive: (s0 + s1) + (s2 + s3) in a fixed order
__device__ __forceinline__ float quad_sum(float v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    return v;
}

struct PosLDS {
    const float4 *xs;
    __device__ float3 operator()(int a) const { const float4 p = xs[a]; return make_float3(p.x, p.y, p.z); }
};
struct PosGlob {
    const GPR_GLOBAL float *x;
    int np;
    __device__ float3 operator()(int a) const { return make_float3(x[a], x[np + a], x[2 * np + a]); }
};

__device__ __forceinline__ float3 neg3(float3 f) { return make_float3(-f.x, -f.y, -f.z); }

// ------------------------------------------------------------------ bonded terms of an atom range
// Terms touching atoms [a0, a1), by kind (bond, angle, torsion, restraint, 1-4).  Terms are
// sorted by their smallest atom and span at most `span` atoms, so those touching [a0, a1) have
// their smallest atom in [a0 - span, a1): of kind k the entries [lo[k], lo[k] + cnt[k]).  They
// occupy the slots [off[k], off[k] + cnt[k]) of one flat index space in which every kind starts
// at a multiple of 64 (so a wave sees one kind).
struct BondedPlan {
    int lo[5], cnt[5], off[6];
};

__device__ __forceinline__ BondedPlan bonded_plan(const Dev &S, int a0, int a1)
{
    const Topo &T = S.tp;
    BondedPlan bp;
    // a molecular system has all five start arrays (n + 1 entries each, all zero for a kind
    // without terms) and the toy none: one branch, then the ten reads go out together instead
    // of one dependent round trip per kind
    if (S.kind == KIND_MOL) {
        const int *const start[5] = {T.b_start, T.a_start, T.t_start, T.r_start, T.p_start};
        const int span[5] = {T.b_span, T.a_span, T.t_span, 0, T.p_span};
        int lo[5], hi[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            lo[k] = gconst(start[k])[max(0, a0 - span[k])];
            hi[k] = gconst(start[k])[a1];
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            bp.lo[k] = lo[k];
            bp.cnt[k] = hi[k] - lo[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) bp.lo[k] = bp.cnt[k] = 0;
    }
    bp.off[0] = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) bp.off[k + 1] = bp.off[k] + (bp.cnt[k] + 63) / 64 * 64;
    return bp;
}

// Adds, for every term of the plan, the fixed-point forces on the atoms of [a0, a1) to
// fa[3][len] (LDS, index a - a0); the energy of a term is counted by the range holding its
// smallest atom.  Each thread takes up to U slots at a time and issues all their topology
// loads before computing any of them.  nthr must be a multiple of 64.
template <class Pos, int U = 4>
__device__ void bonded_range(const Dev &S, const BondedPlan &bp, const Pos &pos, int a0, int a1, long long *fa,
                             int len, long long *e_acc, int tid, int nthr)
{
    // the topology's pointers, read once per call (not again after each LDS atomic)
    const Topo T = S.tp;
    auto add = [&](int a, float3 f) {
        if (a >= a0 && a < a1) {
            lds_add(&fa[a - a0], fix_f(f.x));
            lds_add(&fa[len + a - a0], fix_f(f.y));
            lds_add(&fa[2 * len + a - a0], fix_f(f.z));
        }
    };
    long long e = 0;
    const int total = bp.off[5];
    for (int base = 0; base < total; base += U * nthr) {
        int kind[U];
        int4 idx[U];
        float4 prm[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int slot = base + u * nthr + tid;
            // kind and topology index of the slot (static indices into the plan: no scratch)
            int k = -1, t = 0;
            if (slot < total) {
                int local, cnt, lo;
                if (slot < bp.off[1]) { k = 0; local = slot; cnt = bp.cnt[0]; lo = bp.lo[0]; }
                else if (slot < bp.off[2]) { k = 1; local = slot - bp.off[1]; cnt = bp.cnt[1]; lo = bp.lo[1]; }
                else if (slot < bp.off[3]) { k = 2; local = slot - bp.off[2]; cnt = bp.cnt[2]; lo = bp.lo[2]; }
                else if (slot < bp.off[4]) { k = 3; local = slot - bp.off[3]; cnt = bp.cnt[3]; lo = bp.lo[3]; }
                else { k = 4; local = slot - bp.off[4]; cnt = bp.cnt[4]; lo = bp.lo[4]; }
                if (local >= cnt) k = -1;
                t = lo + local;
            }
            kind[u] = k;
            idx[u] = make_int4(0, 0, 0, 0);
            prm[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (k < 0) continue;
            if (k == 0) {
                const int2 ij = gld(gconst(T.b_ij) + t);
                const float2 p = gld(gconst(T.b_p) + t);
                idx[u] = make_int4(ij.x, ij.y, 0, 0);
                prm[u] = make_float4(p.x, p.y, 0.f, 0.f);
            } else if (k == 1) {
                idx[u] = gld(gconst(T.a_ijk) + t);
                const float2 p = gld(gconst(T.a_p) + t);
                prm[u] = make_float4(p.x, p.y, 0.f, 0.f);
            } else if (k == 2) {
                idx[u] = gld(gconst(T.t_ijkl) + t);
                prm[u] = gld(gconst(T.t_p) + t);
            } else if (k == 3) {
                idx[u] = make_int4(gconst(T.r_i)[t], 0, 0, 0);
                prm[u] = gld(gconst(T.r_p) + t);
            } else {
                const int2 ij = gld(gconst(T.p_ij) + t);
                idx[u] = make_int4(ij.x, ij.y, 0, 0);
                prm[u] = gld(gconst(T.p_p) + t);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = kind[u];
            if (k < 0) continue;
            const int4 q = idx[u];
            const float4 p = prm[u];
            float u_e;
            int mn;
            if (k == 0) {
                float3 fi;
                u_e = term_bond(pos(q.x), pos(q.y), make_float2(p.x, p.y), fi);
                add(q.x, fi);
                add(q.y, neg3(fi));
                mn = min(q.x, q.y);
            } else if (k == 1) {
                float3 fi, fk;
                u_e = term_angle(pos(q.x), pos(q.y), pos(q.z), make_float2(p.x, p.y), fi, fk);
                add(q.x, fi);
                add(q.z, fk);
                add(q.y, make_float3(-fi.x - fk.x, -fi.y - fk.y, -fi.z - fk.z));
                mn = min(q.x, min(q.y, q.z));
            } else if (k == 2) {
                float3 fi, fj, fk, fl;
                u_e = term_torsion(pos(q.x), pos(q.y), pos(q.z), pos(q.w), p, fi, fj, fk, fl);
                add(q.x, fi);
                add(q.y, fj);
                add(q.z, fk);
                add(q.w, fl);
                mn = min(min(q.x, q.y), min(q.z, q.w));
            } else if (k == 3) {
                const float3 x = pos(q.x);
                const float dx = x.x - p.x, dy = x.y - p.y, dz = x.z - p.z;
                add(q.x, make_float3(-p.w * dx, -p.w * dy, -p.w * dz));
                u_e = 0.5f * p.w * (dx * dx + dy * dy + dz * dz);
                mn = q.x;
            } else {
                float3 fi;
                u_e = term_pair14(pos(q.x), pos(q.y), p, fi);
                add(q.x, fi);
                add(q.y, neg3(fi));
                mn = min(q.x, q.y);
            }
            if (e_acc && mn >= a0) e += fix_f(u_e);
        }
    }
    if (e_acc && e != 0) lds_add(e_acc, e);
}

// the double well of the toy system, U = (x^2 - 1)^2 + 2 y^2
__device__ __forceinline__ float toy_force(float x, float y, float &fx, float &fy)
{
    const float x2m1 = x * x - 1.0f;
    fx = -4.0f * x * x2m1;
    fy = -4.0f * y;
    return x2m1 * x2m1 + 2.0f * y * y;
}

// ------------------------------------------------------------------ pair search
// Bounding spheres of blocks of BLK consecutive atoms (chain-local, so compact).  Each radius
// is padded slightly so that rounding cannot drop a pair.
__device__ void block_spheres(const Dev &S, const float4 *xs, float4 *sph, int tid, int nthr)
{
    const int nblk = (S.n + BLK - 1) / BLK;
    for (int t = tid; t < nblk; t += nthr) {
        const int a0 = t * BLK, a1 = min(S.n, a0 + BLK);
        float cx = 0.f, cy = 0.f, cz = 0.f;
        for (int a = a0; a < a1; ++a) { cx += xs[a].x; cy += xs[a].y; cz += xs[a].z; }
        const float inv = 1.0f / (float)(a1 - a0);
        cx *= inv; cy *= inv; cz *= inv;
        float r2 = 0.f;
        for (int a = a0; a < a1; ++a) {
            const float dx = xs[a].x - cx, dy = xs[a].y - cy, dz = xs[a].z - cz;
            r2 = fmaxf(r2, dx * dx + dy * dy + dz * dz);
        }
        sph[t] = make_float4(cx, cy, cz, sqrtf(r2) * 1.0001f + 1e-6f);
    }
}

// a value that every lane holds alike, as a scalar
__device__ __forceinline__ float uniform_f(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }

// min / max over the 16 atoms of a wave (the four lanes of an atom hold the same value)
__device__ __forceinline__ float wave16_min(float v)
{
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave16_max(float v)
{
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Pair lists of the 16 atoms of one wave; lane = 4 (i - i0) + q for the wave's first atom
// i0.  All 64 lanes call it together: the culling is wave-wide (each lane tests a block
// sphere against the bounding box of the wave's atoms, and the wave visits the blocks that
// any lane found near); lanes with valid == false take part but own no list.
// Sub-list (i, q): partners j = q (mod P), j != i, not excluded, |x_i - x_j| < r_list, in
// ascending order; entry k is the 16-bit word k % 4 of group k / 4; the last group is padded
// with the dummy atom n.  allpairs: no distance tests (vacuum, no cutoff; r_list^2 = inf).
// Per 64-block chunk the near blocks are listed in the wave's LDS scratch wblk (ascending);
// their candidates are tested without branches, the outcomes kept as bits (BLK / P per block,
// 32 blocks per batch), and each lane then appends the entries it keeps, four per pass.
// Itself and excluded partners within 32 atoms of it are dropped in the tests, only for
// blocks near the wave's own atoms; farther excluded partners are merged out entry by entry
// (only while some lane of the wave still has one ahead); atoms past n are staged far away,
// so the distance test drops them.  UNR blocks are read at a time (more registers, fewer
// exposed LDS latencies); the plain path's pair kernel uses 1 to keep its occupancy.
template <int UNR, bool PAD>
__device__ __noinline__ int build_wave(const Dev &S, int r, int i, int q, bool valid, const GPR_LDS gv_f4 *xs,
                                       const GPR_LDS gv_f4 *sph, GPR_LDS int *wblk, bool allpairs)
{
    const int n = S.n;
    const size_t stride = (size_t)S.np * P;
    const gv_f4 pi = xs[valid ? i : n];
    // bounding box of the wave's valid atoms
    const float big = 3.0e38f;
    // (the same in every lane: held as scalars)
    const float mnx = uniform_f(wave16_min(valid ? pi.x : big)), mxx = uniform_f(wave16_max(valid ? pi.x : -big));
    if (!(mnx <= mxx)) return 0;                                // no valid lane in this wave
    const float mny = uniform_f(wave16_min(valid ? pi.y : big)), mxy = uniform_f(wave16_max(valid ? pi.y : -big));
    const float mnz = uniform_f(wave16_min(valid ? pi.z : big)), mxz = uniform_f(wave16_max(valid ? pi.z : -big));
    const float rlb = S.rl;
    // finite even without a cutoff, so that the far-away atoms past n never pass
    const float rl2 = fminf(S.rl2, 1.0e30f);
    // atoms [iw, iw + 16) of the wave (lane 0 holds the first)
    const int iw = __builtin_amdgcn_readfirstlane(i);
    // partners to drop: excluded and 1-4 pairs within +-32 of i, and i itself (bit 32)
    const unsigned long long ex = (valid ? gconst(S.excl)[i] : 0ull) | (1ull << 32);
    // excluded and 1-4 partners farther than that: i's ascending list far_j[far_start[i] ..
    // far_start[i + 1]), merged against the entries as they are emitted (also ascending)
    int flo = 0, fhi = 0;
    const GPR_GLOBAL int *fj = gconst(S.far_j);
    if (S.has_far && valid) { flo = gconst(S.far_start)[i]; fhi = gconst(S.far_start)[i + 1]; }
    const int cap = 4 * S.Kg;
    // the replica's lists (a scalar base) and this lane's column in them: group g of sub-list
    // (i, q) is word g * np * P + i * P + q
    GPR_GLOBAL unsigned long long *const Lr = (GPR_GLOBAL unsigned long long *)gmut(S.nbl) + (size_t)r * S.Kg * stride;
    const unsigned col = (unsigned)((valid ? i : 0) * P + q), stride32 = (unsigned)stride;
    const int lane = threadIdx.x & 63;
    const int nblk = (n + BLK - 1) / BLK;
    constexpr int CPB = BLK / P;                                // candidates per block and lane
    constexpr int BATCH = 64 / CPB;                             // blocks per batch of bits
    static_assert(CPB == 2, "a half batch is 32 candidates of 16 blocks");
    static_assert(BATCH % UNR == 0, "a batch holds whole groups of UNR blocks");
    unsigned long long bits = 0ull;
    // entries so far; the cnt % 4 entries of the unfinished group sit in the low 16-bit words
    // of pend, in order; group g = cnt / 4 goes to word g * stride + col, if g < Kg
    unsigned long long pend = 0ull;
    int cnt = 0;
    auto emit = [&](int base) {
        __builtin_amdgcn_wave_barrier();
        const bool merge = __ballot(flo < fhi) != 0ull;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            unsigned b32 = h ? (unsigned)(bits >> 32) : (unsigned)bits;
            const int hb = base + 16 * h;
            if (!merge) {
                // candidate k of the half is partner wblk[hb + k / 2] * BLK + (k % 2) * P + q:
                // lane k < 32 holds that base, which the lanes read through the crossbar.  The
                // passes are wave-uniform (a lane out of entries takes none), so that every lane
                // is active at the crossbar read: an inactive source lane would read as zero.
                const int jt = lane < 32 ? wblk[hb + (lane >> 1)] * BLK + (lane & 1) * P : 0;
                while (__ballot(b32 != 0u) != 0ull) {
                    const int c = min(4, __popc(b32));
                    unsigned jv[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int k = __ffs(b32) - 1;           // -1 once no bit is left
                        b32 &= b32 - 1u;
                        const int j = __shfl(jt, k & 31, 64) + q;
                        jv[e] = k >= 0 ? (unsigned)j : 0u;
                    }
                    const unsigned long long ch = (unsigned long long)(jv[0] | (jv[1] << 16)) |
                                                  ((unsigned long long)(jv[2] | (jv[3] << 16)) << 32);
                    const int sh = 16 * (cnt & 3);
                    const unsigned long long lo = pend | (ch << sh);
                    if ((cnt & 3) + c >= 4) {
                        if (cnt < cap) gst(Lr + ((unsigned)(cnt >> 2) * stride32 + col), lo);
                        pend = sh ? ch >> (64 - sh) : 0ull;
                    } else {
                        pend = lo;
                    }
                    cnt += c;
                }
            } else {
                while (b32) {
                    const int k = __ffs(b32) - 1;
                    b32 &= b32 - 1u;
                    const unsigned j = (unsigned)(wblk[hb + k / CPB] * BLK + q + (k % CPB) * P);
                    if (flo < fhi) {
                        while (flo < fhi && (unsigned)fj[flo] < j) ++flo;
                        if (flo < fhi && (unsigned)fj[flo] == j) continue;
                    }
                    pend |= (unsigned long long)j << (16 * (cnt & 3));
                    if ((cnt & 3) == 3) {
                        if (cnt < cap) gst(Lr + ((unsigned)(cnt >> 2) * stride32 + col), pend);
                        pend = 0ull;
                    }
                    ++cnt;
                }
            }
        }
        bits = 0ull;
        __builtin_amdgcn_wave_barrier();
    };
    for (int cb = 0; cb < nblk; cb += 64) {
        const int b = cb + lane;
        bool near = b < nblk;
        if (near && !allpairs) {
            // distance from the block's centre to the wave's box, against r_list + its radius
            const gv_f4 c = sph[b];
            const float dx = fmaxf(0.f, fmaxf(mnx - c.x, c.x - mxx));
            const float dy = fmaxf(0.f, fmaxf(mny - c.y, c.y - mxy));
            const float dz = fmaxf(0.f, fmaxf(mnz - c.z, c.z - mxz));
            const float lim = (rlb + c.w) * 1.0001f + 1e-6f;
            near = dx * dx + dy * dy + dz * dz < lim * lim;
        }
        const unsigned long long m = __ballot(near);
        const int cntm = __popcll(m);
        if (cntm == 0) continue;
        __builtin_amdgcn_wave_barrier();
        if (near) wblk[__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))] = b;
        __builtin_amdgcn_wave_barrier();
        int base = 0;
        for (int k0 = 0; k0 < cntm; k0 += UNR) {
            // the next UNR blocks; past the last one (cntm) the last block again, whose test bits
            // the mask `live` drops.  Every lane reads the same entries, so the block indices and
            // what follows from them (candidate bases, the exclusion test below) stay scalar; all
            // reads are in flight before the first use.
            int raw[UNR], bb[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) raw[u] = wblk[min(k0 + u, cntm - 1)];
#pragma unroll
            for (int u = 0; u < UNR; ++u) bb[u] = __builtin_amdgcn_readfirstlane(raw[u]);
            const int nlive = min(UNR, cntm - k0);
            const unsigned live = nlive == UNR ? ~0u : (1u << (nlive * CPB)) - 1u;
            // (x, y, z) only: a 12-byte read leaves no unused destination register that the
            // compiler could reuse, and so wait for, before the read completes
            gv_f3 pj[UNR][CPB];
            const GPR_LDS gv_f3 *x3 = (const GPR_LDS gv_f3 *)xs;
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int t = 0; t < CPB; ++t)
                    pj[u][t] = x3[bb[u] * BLK + q + t * P];
            __builtin_amdgcn_sched_barrier(0);                  // keep the reads ahead of the tests
            // a slot past n in the last block holds a far-away position and fails the test; a
            // lane without an atom (its position also the far-away one) keeps no bit
            unsigned tb = 0u;
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int t = 0; t < CPB; ++t) {
                    const float dx = pi.x - pj[u][t].x, dy = pi.y - pj[u][t].y, dz = pi.z - pj[u][t].z;
                    tb |= (unsigned)(fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < rl2) << (u * CPB + t);
                }
            tb = valid ? tb & live : 0u;
            // blocks that may hold the wave's atoms or their excluded partners (wave-uniform)
            bool self = false;
#pragma unroll
            for (int u = 0; u < UNR; ++u)
                self |= u < nlive && bb[u] * BLK + BLK > iw - 32 && bb[u] * BLK < iw + 16 + 32;
            if (self) {
#pragma unroll
                for (int u = 0; u < UNR; ++u)
#pragma unroll
                    for (int t = 0; t < CPB; ++t) {
                        const int off = bb[u] * BLK + q + t * P - i + 32;
                        const unsigned drop = (unsigned)((unsigned)off < 64u) & (unsigned)((ex >> (off & 63)) & 1ull);
                        tb &= ~(drop << (u * CPB + t));
                    }
            }
            bits |= (unsigned long long)tb << (((k0 - base) % BATCH) * CPB);
            if (k0 + UNR - base == BATCH) {
                emit(base);
                base += BATCH;
            }
        }
        emit(base);
    }
    if (!valid) return 0;
    const int ng = min((cnt + 3) >> 2, S.Kg);
    if ((cnt & 3) != 0 && cnt < cap) {
        const unsigned long long pad = (unsigned long long)n * 0x0001000100010001ull;
        gst(Lr + ((unsigned)(cnt >> 2) * stride32 + col), pend | (pad << (16 * (cnt & 3))));
    }
    // PAD: the four sub-lists of an atom padded to the same number of groups with the
    // far-away atom n (exact zeros), so that one count (the largest, returned) serves the
    // atom's four lanes; the counts array keeps each sub-list's own count
    int kq = ng;
    if (PAD) {
        kq = max(ng, __shfl_xor(ng, 1, 64));
        kq = max(kq, __shfl_xor(kq, 2, 64));
        const unsigned long long pad = (unsigned long long)n * 0x0001000100010001ull;
        for (int w = ng; w < kq; ++w) gst(Lr + ((unsigned)w * stride32 + col), pad);
    }
    gmut(S.nbc)[(size_t)r * stride + (size_t)i * P + q] = (unsigned short)ng;
    if (cnt > cap) atomicOr(&S.err[ERR_LIST], 1);
    return kq;
}

// ------------------------------------------------------------------ nonbonded partial sum of one lane
// Lennard-Jones + Coulomb (vacuum when krf = crf = 0 and rc2 = inf; reaction field
// otherwise) of one pair, accumulated into (fx, fy, fz) and, with energy, U/2 into e.
__device__ __forceinline__ void pair_term(const float4 pi, const float2 ppi, const float4 pj, const float2 ppj,
                                          float rc2, float krf2, float krf, float crf, bool energy,
                                          float &fx, float &fy, float &fz, float &e)
{
    const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r2i = ri * ri;
    const float sg = ppi.x + ppj.x;
    const float s2 = (sg * sg) * r2i;
    const float s6 = (s2 * s2) * s2;
    const float e4 = ppi.y * ppj.y;
    const float qq = pi.w * pj.w;
    // -dU/dr / r = e4 r2i (12 s6^2 - 6 s6) + qq (ri r2i - 2 krf)
    const float lj = (e4 * r2i) * (s6 * fmaf(12.0f, s6, -6.0f));
    const float fs0 = fmaf(qq, fmaf(ri, r2i, -krf2), lj);
    const bool in = r2 < rc2;
    const float fs = in ? fs0 : 0.0f;
    fx = fmaf(fs, dx, fx);
    fy = fmaf(fs, dy, fy);
    fz = fmaf(fs, dz, fz);
    if (energy) {
        const float u = fmaf(e4 * s6, s6 - 1.0f, qq * (fmaf(krf, r2, ri) - crf));
        e = in ? fmaf(0.5f, u, e) : e;
    }
}

// The pair loop's parameters, as values (read once per step in a persistent launch)
struct NbConsts {
    const uint2 *nbl;
    const unsigned short *nbc;
    int np, Kg;
    float rc2, krf, crf;
};
__device__ __forceinline__ NbConsts nb_consts(const Dev &S)
{
    NbConsts k;
    k.nbl = S.nbl; k.nbc = S.nbc; k.np = S.np; k.Kg = S.Kg; k.rc2 = S.rc2; k.krf = S.krf; k.crf = S.crf;
    return k;
}

// Sum over sub-list (i, q), four partners per 8-byte list word, the next word loaded one
// group ahead; returns (F_x, F_y, F_z, sum U/2).
template <bool ENERGY>
__device__ __forceinline__ float4 nb_lane_t(const NbConsts &S, int r, int i, int q, const float4 *xs, const float2 *pp,
                                            int ngk)
{
    const size_t stride = (size_t)S.np * P;
    const GPR_GLOBAL uint2 *L = gconst(S.nbl) + (size_t)r * S.Kg * stride + (size_t)i * P + q;
    // groups in the sub-list: given (the atom's count kept in LDS), or read from the counts
    const int ng = ngk >= 0 ? ngk : (int)gconst(S.nbc)[(size_t)r * stride + (size_t)i * P + q];
    const float4 pi = xs[i];
    const float2 ppi = pp[i];
    const float rc2 = S.rc2, krf = S.krf, krf2 = 2.0f * S.krf, crf = S.crf;
    float fx = 0.f, fy = 0.f, fz = 0.f, e = 0.f;
    // the next word is read one group ahead, without a branch, through a running pointer that
    // stops at the last group (which is then read again, from the cache)
    const GPR_GLOBAL uint2 *Ln = L;
    const unsigned step = (unsigned)stride;
    uint2 nxt = make_uint2(0u, 0u);
    if (ng > 0) nxt = gld(Ln);
    for (int g = 0; g < ng; ++g) {
        const uint2 cur = nxt;
        Ln += g + 1 < ng ? step : 0u;
        nxt = gld(Ln);
        const int j0 = cur.x & 0xFFFF, j1 = cur.x >> 16, j2 = cur.y & 0xFFFF, j3 = cur.y >> 16;
        const float4 x0 = xs[j0], x1 = xs[j1], x2 = xs[j2], x3 = xs[j3];
        const float2 p0 = pp[j0], p1 = pp[j1], p2 = pp[j2], p3 = pp[j3];
        pair_term(pi, ppi, x0, p0, rc2, krf2, krf, crf, ENERGY, fx, fy, fz, e);
        pair_term(pi, ppi, x1, p1, rc2, krf2, krf, crf, ENERGY, fx, fy, fz, e);
        pair_term(pi, ppi, x2, p2, rc2, krf2, krf, crf, ENERGY, fx, fy, fz, e);
        pair_term(pi, ppi, x3, p3, rc2, krf2, krf, crf, ENERGY, fx, fy, fz, e);
    }
    return make_float4(fx, fy, fz, e);
}

__device__ __forceinline__ float4 nb_lane(const NbConsts &S, int r, int i, int q, const float4 *xs, const float2 *pp,
                                          bool energy, int ngk = -1)
{
    return energy ? nb_lane_t<true>(S, r, i, q, xs, pp, ngk) : nb_lane_t<false>(S, r, i, q, xs, pp, ngk);
}

// ------------------------------------------------------------------ one B A O A for one atom
// The integrator's constants, as values: a persistent launch holds them in registers (read
// through the descriptor they would be loaded again after every fence of a step).
struct IntConsts {
    float h, c1;
    uint32_t key0, key1;
    int toy;
};
__device__ __forceinline__ IntConsts int_consts(const Dev &S)
{
    IntConsts k;
    k.h = S.h; k.c1 = S.c1; k.key0 = S.key0; k.key1 = S.key1; k.toy = S.kind == KIND_TOY;
    return k;
}

__device__ __forceinline__ void integrate_baoa_k(const IntConsts &K, int a, int r, long long s, float3 &x, float3 &v,
                                                 float3 F, float im, float sd)
{
    const float h = K.h, c1 = K.c1;
    v.x = kick(v.x, F.x, h, im);
    v.y = kick(v.y, F.y, h, im);
    v.z = kick(v.z, F.z, h, im);
    x.x = x.x + h * v.x;
    x.y = x.y + h * v.y;
    x.z = x.z + h * v.z;
    const float3 g = gauss3(philox_ctr((uint32_t)a, s, (uint32_t)r, STREAM_NOISE, K.key0, K.key1));
    v.x = c1 * v.x + sd * g.x;
    v.y = c1 * v.y + sd * g.y;
    if (!K.toy) v.z = c1 * v.z + sd * g.z;
    x.x = x.x + h * v.x;
    x.y = x.y + h * v.y;
    x.z = x.z + h * v.z;
}

__device__ __forceinline__ void integrate_baoa(const Dev &S, int a, int r, long long s, float3 &x, float3 &v,
                                               float3 F, float im, float sd)
{
    integrate_baoa_k(int_consts(S), a, r, s, x, v, F, im, sd);
}

__device__ __forceinline__ bool finite3(float3 a) { return isfinite(a.x) && isfinite(a.y) && isfinite(a.z); }

// ------------------------------------------------------------------ states and observables (FP64)
// Workgroup-collective.  Sums over atoms are taken in 2^-32 fixed point so that they do
// not depend on the launch shape.  red: LDS int64 scratch [MAX_OBS * 8 + 8].
// velocity component load; coh: device-coherent load of values another workgroup wrote
__device__ __forceinline__ float ldv(const float *p, bool coh)
{
    return coh ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}

__device__ void group_sum_wg(const Dev &S, const float4 *xs, const float *vg, int off, int cnt, int what,
                             long long *dst, int tid, int nthr, bool coh = false)
{
    // what: 0 -> sum m x (3 slots), 1 -> sum |v|^2 (1 slot)
    for (int base = 0; base < cnt; base += nthr) {
        const int k = base + tid;
        long long s0 = 0, s1 = 0, s2 = 0;
        if (k < cnt) {
            const int a = S.groups[off + k];
            if (what == 0) {
                const double m = (double)S.mass[a];
                s0 = fix_d(m * (double)xs[a].x);
                s1 = fix_d(m * (double)xs[a].y);
                s2 = fix_d(m * (double)xs[a].z);
            } else {
                const double vx = ldv(vg + a, coh), vy = ldv(vg + S.np + a, coh), vz = ldv(vg + 2 * S.np + a, coh);
                s0 = fix_d(vx * vx + vy * vy + vz * vz);
            }
        }
        s0 = wave_sum_ll(s0);
        if (what == 0) { s1 = wave_sum_ll(s1); s2 = wave_sum_ll(s2); }
        if ((tid & 63) == 0) {
            lds_add(&dst[0], s0);
            if (what == 0) { lds_add(&dst[1], s1); lds_add(&dst[2], s2); }
        }
    }
}

__device__ __forceinline__ double3 xs_d(const float4 *xs, int a)
{
    return make_double3((double)xs[a].x, (double)xs[a].y, (double)xs[a].z);
}

__device__ int state_wg(const Dev &S, const float4 *xs, long long *red, int *sbuf, int tid, int nthr)
{
    const StateDesc &st = *S.st;
    if (st.kind == ST_SIGN_X) return xs[st.atoms[0]].x >= 0.0f ? 1 : 0;
    if (st.kind == ST_BOXES) {
        if (tid == 0) {
            const double phi = dihedral_d(xs_d(xs, st.atoms[0]), xs_d(xs, st.atoms[1]), xs_d(xs, st.atoms[2]), xs_d(xs, st.atoms[3]));
            const double psi = dihedral_d(xs_d(xs, st.atoms[4]), xs_d(xs, st.atoms[5]), xs_d(xs, st.atoms[6]), xs_d(xs, st.atoms[7]));
            int id = -1;
            for (int b = 0; b < st.nbox; ++b)
                if (st.box[b][0] < phi && phi <= st.box[b][1] && st.box[b][2] < psi && psi <= st.box[b][3]) { id = b; break; }
            *sbuf = id;
        }
        __syncthreads();
        const int id = *sbuf;
        __syncthreads();
        return id;
    }
    // centre of mass within a sphere
    if (tid < 3) red[tid] = 0;
    __syncthreads();
    group_sum_wg(S, xs, nullptr, st.g_off, st.g_n, 0, red, tid, nthr);
    __syncthreads();
    if (tid == 0) {
        const double cx = unfix_d(red[0]) / st.gm, cy = unfix_d(red[1]) / st.gm, cz = unfix_d(red[2]) / st.gm;
        const double dx = cx - st.center[0], dy = cy - st.center[1], dz = cz - st.center[2];
        *sbuf = sqrt(dx * dx + dy * dy + dz * dz) < st.radius ? 1 : 0;
    }
    __syncthreads();
    const int id = *sbuf;
    __syncthreads();
    return id;
}

// observable values into out[MAX_OBS] (LDS), valid after return
__device__ void observables_wg(const Dev &S, const float4 *xs, const float *vg, double U, long long *red,
                               double *out, int tid, int nthr, bool coh = false)
{
    if (tid < MAX_OBS * 8) red[tid] = 0;
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < S.nobs; ++j) {
        const ObsDesc &o = S.obs[j];
        long long *dst = red + 8 * j;
        if (o.kind == OB_KIN) {
            for (int base = 0; base < S.n; base += nthr) {
                const int a = base + tid;
                long long s = 0;
                if (a < S.n) {
                    const double vx = ldv(vg + a, coh), vy = ldv(vg + S.np + a, coh), vz = ldv(vg + 2 * S.np + a, coh);
                    s = fix_d(0.5 * (double)S.mass[a] * (vx * vx + vy * vy + vz * vz));
                }
                s = wave_sum_ll(s);
                if ((tid & 63) == 0) lds_add(dst, s);
            }
        } else if (o.kind == OB_COMD) {
            group_sum_wg(S, xs, vg, o.ga_off, o.ga_n, 0, dst, tid, nthr);
            group_sum_wg(S, xs, vg, o.gb_off, o.gb_n, 0, dst + 3, tid, nthr);
        } else if (o.kind == OB_RMSV) {
            group_sum_wg(S, xs, vg, o.ga_off, o.ga_n, 1, dst, tid, nthr, coh);
        }
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll 1
        for (int j = 0; j < S.nobs; ++j) {
            const ObsDesc &o = S.obs[j];
            const long long *src = red + 8 * j;
            double val = 0.0;
            switch (o.kind) {
            case OB_COORD: {
                const float4 p = xs[o.atoms[0]];
                val = o.atoms[1] == 0 ? (double)p.x : (o.atoms[1] == 1 ? (double)p.y : (double)p.z);
                break;
            }
            case OB_POT: val = U; break;
            case OB_KIN: val = unfix_d(src[0]); break;
            case OB_DIH:
                val = dihedral_d(xs_d(xs, o.atoms[0]), xs_d(xs, o.atoms[1]), xs_d(xs, o.atoms[2]), xs_d(xs, o.atoms[3]));
                break;
            case OB_COMD: {
                const double ax = unfix_d(src[0]) / o.ma, ay = unfix_d(src[1]) / o.ma, az = unfix_d(src[2]) / o.ma;
                const double bx = unfix_d(src[3]) / o.mb, by = unfix_d(src[4]) / o.mb, bz = unfix_d(src[5]) / o.mb;
                val = sqrt((ax - bx) * (ax - bx) + (ay - by) * (ay - by) + (az - bz) * (az - bz));
                break;
            }
            case OB_RMSV: val = sqrt(unfix_d(src[0]) / (double)o.ga_n); break;
            default: break;
            }
            out[j] = val;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void accumulate_obs(const Dev &S, int r, const double *out)
{
    double *acc = S.acc + (size_t)r * MAX_OBS * 2;
    for (int j = 0; j < S.nobs; ++j) {
        const double xj = out[j] - S.shift[j];
        acc[2 * j] += xj;
        const double x2 = xj * xj;
        acc[2 * j + 1] += x2;
    }
}

// stage positions (x, y, z, q sqrt f) and (sigma/2, 2 sqrt eps) of replica r into LDS
__device__ __forceinline__ void stage_replica(const Dev &S, int r, float4 *xs, float2 *pp, int tid, int nthr)
{
    const GPR_GLOBAL float *xg = gconst(S.x) + (size_t)r * 3 * S.np;
    for (int a = tid; a < S.np; a += nthr) {
        const float4 pr = gld(gconst(S.prm) + a);
        if (a < S.n) xs[a] = make_float4(xg[a], xg[S.np + a], xg[2 * S.np + a], pr.z);
        else xs[a] = make_float4(FAR, FAR, FAR, 0.f);
        if (pp) pp[a] = make_float2(pr.x, pr.y);
    }
}

// ================================================================== plain path kernels
// Step and energy flag of a plain-path kernel: as given, or (codes DCLK_*) step k of a cycle
// that starts at the device clock (s, t) = (clock[0], clock[1]), with k passed in s; such a
// step samples when (t + k + 1) is a multiple of t_GR.
__device__ __forceinline__ void step_args(const Dev &S, long long &s, int &energy)
{
    if (energy < DCLK_SAMPLE) return;
    const long long k = s;
    const bool samp = energy == DCLK_SAMPLE && (S.clock[1] + k + 1) % S.t_gr == 0;
    s = S.clock[0] + k;
    energy = (samp && S.need_energy) ? 1 : 0;
}

__global__ void k_set_clock(const Dev *__restrict__ Sp, long long s, long long t)
{
    Sp->clock[0] = s;
    Sp->clock[1] = t;
}

__global__ void k_tick(const Dev *__restrict__ Sp, long long n)
{
    Sp->clock[0] += n;
    Sp->clock[1] += n;
}
// B A O A for every atom of replicas r_off + blockIdx.y; displacement guard; energy reset.
__global__ void __launch_bounds__(256) k_integrate(const Dev *__restrict__ Sp, long long s, int r_off, int energy)
{
    const Dev &S = *Sp;
    step_args(S, s, energy);
    const int r = r_off + blockIdx.y;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    int *guard = S.guard + (s & 1) * S.R + r;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (energy) S.E[r] = 0;
        if (S.need_build[r]) { atomicOr(guard, 1); S.need_build[r] = 0; }
    }
    if (a >= S.n) return;
    const size_t b = (size_t)r * 3 * S.np;
    const int np = S.np;
    GPR_GLOBAL float *X = gmut(S.x) + b, *V = gmut(S.v) + b;
    const GPR_GLOBAL float *XB = gconst(S.xb) + b;
    const GPR_GLOBAL long long *Fp = gconst(S.F) + b;
    float3 x = make_float3(X[a], X[np + a], X[2 * np + a]);
    float3 v = make_float3(V[a], V[np + a], V[2 * np + a]);
    const float3 F = make_float3(unfix_f(Fp[a]), unfix_f(Fp[np + a]), unfix_f(Fp[2 * np + a]));
    const float im = gld(gconst(S.prm) + a).w;
    integrate_baoa(S, a, r, s, x, v, F, im, gconst(S.sd)[a]);
    X[a] = x.x; X[np + a] = x.y; X[2 * np + a] = x.z;
    V[a] = v.x; V[np + a] = v.y; V[2 * np + a] = v.z;
    if (!finite3(x) || !finite3(v)) atomicOr(&S.err[ERR_UNSTABLE], 1);
    if (S.cutoff_on) {
        const float dx = x.x - XB[a], dy = x.y - XB[np + a], dz = x.z - XB[2 * np + a];
        if (!(dx * dx + dy * dy + dz * dz <= S.half_skin2)) atomicOr(guard, 1);
    }
}

// Bonded forces of atom range [blockIdx.x * blockDim.x, +blockDim.x) of replica r:
// fixed-point LDS accumulation, then a plain store that initialises F for the step.
__global__ void __launch_bounds__(256) k_bonded(const Dev *__restrict__ Sp, long long s, int r_off, int energy)
{
    const Dev &S = *Sp;
    step_args(S, s, energy);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    long long *fa = (long long *)lds_raw;
    __shared__ long long e_acc;
    const int r = r_off + blockIdx.y;
    const int len = blockDim.x;
    const int a0 = blockIdx.x * len, a1 = min(S.n, a0 + len);
    const int tid = threadIdx.x;
    for (int k = tid; k < 3 * len; k += len) fa[k] = 0;
    if (tid == 0) e_acc = 0;
    __syncthreads();
    const size_t b = (size_t)r * 3 * S.np;
    if (S.kind == KIND_TOY) {
        if (tid == 0 && a0 == 0) {
            float fx, fy;
            const float u = toy_force(S.x[b], S.x[b + S.np], fx, fy);
            fa[0] = fix_f(fx);
            fa[len] = fix_f(fy);
            if (energy) e_acc = fix_f(u);
        }
    } else {
        bonded_range(S, bonded_plan(S, a0, a1), PosGlob{gconst(S.x) + b, S.np}, a0, a1, fa, len,
                     energy ? &e_acc : nullptr, tid, len);
    }
    __syncthreads();
    const int a = a0 + tid;
    if (a < a1) {
        S.F[b + a] = fa[tid];
        S.F[b + S.np + a] = fa[len + tid];
        S.F[b + 2 * S.np + a] = fa[2 * len + tid];
    }
    if (energy && tid == 0 && e_acc != 0) atomicAdd((unsigned long long *)&S.E[r], (unsigned long long)e_acc);
}

// Nonbonded forces of atoms [blockIdx.x * blockDim.x / P, ...) of replica r (P lanes per
// atom), added to the bonded forces; then the closing B kick (apply_b).  The pair lists of
// the block's atoms are rebuilt first when due (period, displacement guard, force_build).
__global__ void __launch_bounds__(1024) k_nonbonded(const Dev *__restrict__ Sp, long long s, int r_off, int energy, int apply_b,
                                                   int force_build)
{
    step_args(*Sp, s, energy);
    const Dev &S = *Sp;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float4 *xs = (float4 *)lds_raw;
    float2 *pp = (float2 *)(xs + S.np);
    float4 *sph = (float4 *)(pp + S.np);
    int *wscr = (int *)(sph + (S.n + BLK - 1) / BLK);      // [16][WBLK] build scratch per wave
    __shared__ long long e_acc;
    const int r = r_off + blockIdx.y;
    const int tid = threadIdx.x, nthr = blockDim.x;
    stage_replica(S, r, xs, pp, tid, nthr);
    if (tid == 0) e_acc = 0;
    // rebuild when forced, when flagged (displacement guard or a new configuration), or on the
    // steps s with s + 1 a multiple of period, the same steps for every replica: one launch
    // serves all replicas, so rebuilds that coincide cost one long launch instead of many.
    // The step of the last build is recorded by step parity (block 0 writes the next step's
    // slot while the other blocks read this step's) for the persistent path.
    bool rebuild = force_build != 0;
    if (!force_build) {
        long long lb = 0;
        if (S.cutoff_on) {
            lb = S.last_build[(s & 1) * S.R + r];
            rebuild = (s + 1) % S.period == 0 || S.guard[(s & 1) * S.R + r] != 0;
        }
        if (blockIdx.x == 0 && tid == 0) {
            S.guard[((s + 1) & 1) * S.R + r] = 0;
            S.last_build[((s + 1) & 1) * S.R + r] = rebuild ? s : lb;
            if (rebuild) S.list_pad[r] = 0;
        }
    } else if (blockIdx.x == 0 && tid == 0) {
        S.last_build[r] = s;
        S.last_build[S.R + r] = s;
        S.list_pad[r] = 0;
    }
    __syncthreads();
    const int i = blockIdx.x * (nthr / P) + tid / P;
    const int q = tid % P;
    const size_t b = (size_t)r * 3 * S.np;
    if (rebuild) {
        block_spheres(S, xs, sph, tid, nthr);
        __syncthreads();
        build_wave<1, false>(S, r, i, q, i < S.n, (const GPR_LDS gv_f4 *)xs, (const GPR_LDS gv_f4 *)sph,
                   (GPR_LDS int *)wscr + (tid >> 6) * WBLK, !S.cutoff_on);
        if (i < S.n && q == 0) {
            S.xb[b + i] = xs[i].x; S.xb[b + S.np + i] = xs[i].y; S.xb[b + 2 * S.np + i] = xs[i].z;
        }
        __syncthreads();
    }
    long long eatom = 0;
    if (i < S.n) {
        float4 f = nb_lane(nb_consts(S), r, i, q, xs, pp, energy != 0);
        f.x = quad_sum(f.x);
        f.y = quad_sum(f.y);
        f.z = quad_sum(f.z);
        if (energy) f.w = quad_sum(f.w);
        if (q == 0) {
            GPR_GLOBAL long long *Fp = gmut(S.F) + b;
            GPR_GLOBAL float *V = gmut(S.v) + b;
            const long long Fx = Fp[i] + fix_f(f.x);
            const long long Fy = Fp[S.np + i] + fix_f(f.y);
            const long long Fz = Fp[2 * S.np + i] + fix_f(f.z);
            Fp[i] = Fx; Fp[S.np + i] = Fy; Fp[2 * S.np + i] = Fz;
            const float fx = unfix_f(Fx), fy = unfix_f(Fy), fz = unfix_f(Fz);
            if (bad_force(fx) || bad_force(fy) || bad_force(fz)) atomicOr(&S.err[ERR_UNSTABLE], 1);
            if (apply_b) {
                const float im = gld(gconst(S.prm) + i).w, h = S.h;
                V[i] = kick(V[i], fx, h, im);
                V[S.np + i] = kick(V[S.np + i], fy, h, im);
                V[2 * S.np + i] = kick(V[2 * S.np + i], fz, h, im);
            }
            if (energy) eatom = fix_f(f.w);
        }
    }
    if (energy) {
        eatom = wave_sum_ll(eatom);
        if ((tid & 63) == 0 && eatom != 0) lds_add(&e_acc, eatom);
        __syncthreads();
        if (tid == 0 && e_acc != 0) atomicAdd((unsigned long long *)&S.E[r], (unsigned long long)e_acc);
    }
}

// observables of replicas r_off + blockIdx.x: accumulate (mode 0, workers), set the shift
// c_j from replica 0 (mode 1), or write the values to out[r][MAX_OBS] (mode 2)
__global__ void __launch_bounds__(256) k_obs(const Dev *__restrict__ Sp, int r_off, int mode, double *out, int k)
{
    const Dev &S = *Sp;
    if (mode == 3 && (S.clock[1] + k + 1) % S.t_gr != 0) return;    // step k of a device-clock cycle: no sample
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float4 *xs = (float4 *)lds_raw;
    __shared__ long long red[MAX_OBS * 8 + 8];
    __shared__ double vals[MAX_OBS];
    const int r = r_off + blockIdx.x;
    stage_replica(S, r, xs, nullptr, threadIdx.x, blockDim.x);
    __syncthreads();
    const float *vg = S.v + (size_t)r * 3 * S.np;
    observables_wg(S, xs, vg, unfix_d(S.E[r]), red, vals, threadIdx.x, blockDim.x);
    if (threadIdx.x == 0) {
        if (mode == 0 || mode == 3) accumulate_obs(S, r, vals);
        else if (mode == 1) for (int j = 0; j < S.nobs; ++j) S.shift[j] = vals[j];
        else for (int j = 0; j < S.nobs; ++j) out[(size_t)r * MAX_OBS + j] = vals[j];
    }
}

// state ids of replicas r_off + blockIdx.x
__global__ void __launch_bounds__(256) k_state(const Dev *__restrict__ Sp, int r_off)
{
    const Dev &S = *Sp;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float4 *xs = (float4 *)lds_raw;
    __shared__ long long red[8];
    __shared__ int sbuf;
    const int r = r_off + blockIdx.x;
    stage_replica(S, r, xs, nullptr, threadIdx.x, blockDim.x);
    __syncthreads();
    const int id = state_wg(S, xs, red, &sbuf, threadIdx.x, blockDim.x);
    if (threadIdx.x == 0) S.state[r] = id;
}

// ================================================================== force-field parameter gradient
// dU_r/dtheta for theta = (eps_i, sigma_i, q_i, torsion k_t), weighted by w[r] and summed over
// the replicas in 2^-32 fixed point (gacc).  With eps_ij = sqrt(eps_i eps_j), sigma_ij =
// (sigma_i + sigma_j)/2, s = sigma_ij / r and Coulomb kernel g(r):
//   dU/deps_i   = 1/(2 eps_i) sum_j 4 eps_ij (s^12 - s^6)
//   dU/dsigma_i = sum_j 1/2 4 eps_ij (12 s^12 - 6 s^6) / sigma_ij
//   dU/dq_i     = sqrt(f) sum_j (q_j sqrt(f)) g(r)
//   dU/dk_t     = 1 + cos(n phi - phi0)
// the constant factors 1/(2 eps_i) and sqrt(f) applied in k_grad_finish.  Pair sums run over
// the full pair lists (every partner of i in i's own sub-lists), so each atom's sums are
// complete without scattering to j; 1-4 pairs (scaled) and torsions come one term per thread.

// nonbonded pairs of replicas r_off + blockIdx.y at their current positions and pair lists
__global__ void __launch_bounds__(1024) k_grad_nb(const Dev *__restrict__ Sp, const double *w)
{
    const Dev &S = *Sp;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float4 *xs = (float4 *)lds_raw;
    float2 *pp = (float2 *)(xs + S.np);
    const int r = blockIdx.y;
    const int tid = threadIdx.x, nthr = blockDim.x;
    stage_replica(S, r, xs, pp, tid, nthr);
    __syncthreads();
    const int i = blockIdx.x * (nthr / P) + tid / P;
    const int q = tid % P;
    float se = 0.f, ss = 0.f, sq = 0.f;
    if (i < S.n) {
        const size_t stride = (size_t)S.np * P;
        const GPR_GLOBAL uint2 *L = gconst(S.nbl) + (size_t)r * S.Kg * stride + (size_t)i * P + q;
        const int ng = gconst(S.nbc)[(size_t)r * stride + (size_t)i * P + q];
        const float4 pi = xs[i];
        const float2 ppi = pp[i];
        const float rc2 = S.rc2, krf = S.krf, crf = S.crf;
        for (int g = 0; g < ng; ++g) {
            const uint2 wv = gld(L + (size_t)g * stride);
            const int jj[4] = {(int)(wv.x & 0xFFFF), (int)(wv.x >> 16), (int)(wv.y & 0xFFFF), (int)(wv.y >> 16)};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float4 pj = xs[jj[k]];
                const float2 ppj = pp[jj[k]];
                const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float sg = ppi.x + ppj.x;
                const float t = sg * ri;
                const float s2 = t * t;
                const float s6 = s2 * s2 * s2, s12 = s6 * s6;
                const float e4 = ppi.y * ppj.y;
                const bool in = r2 < rc2;
                se += in ? e4 * (s12 - s6) : 0.0f;
                ss += in ? 0.5f * e4 * (12.0f * s12 - 6.0f * s6) * __builtin_amdgcn_rcpf(sg) : 0.0f;
                sq += in ? pj.w * (ri + krf * r2 - crf) : 0.0f;
            }
        }
    }
    se = quad_sum(se);
    ss = quad_sum(ss);
    sq = quad_sum(sq);
    if (i < S.n && q == 0) {
        const double wr = w[r];
        unsigned long long *G = (unsigned long long *)S.gacc;
        atomicAdd(G + i, (unsigned long long)fix_d(wr * se));
        atomicAdd(G + S.np + i, (unsigned long long)fix_d(wr * ss));
        atomicAdd(G + 2 * S.np + i, (unsigned long long)fix_d(wr * sq));
    }
}

// 1-4 pairs (no cutoff, vacuum Coulomb, scaled) and torsions of replica blockIdx.y
__global__ void __launch_bounds__(256) k_grad_terms(const Dev *__restrict__ Sp, const double *w)
{
    const Dev &S = *Sp;
    const Topo &T = S.tp;
    const int r = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const double wr = w[r];
    const PosGlob pos{gconst(S.x) + (size_t)r * 3 * S.np, S.np};
    unsigned long long *G = (unsigned long long *)S.gacc;
    if (t < T.n14) {
        const int2 ij = gld(gconst(T.p_ij) + t);
        const float4 a = gld(gconst(S.prm) + ij.x), b = gld(gconst(S.prm) + ij.y);
        const float3 xa = pos(ij.x), xb = pos(ij.y);
        const float dx = xa.x - xb.x, dy = xa.y - xb.y, dz = xa.z - xb.z;
        const float ri = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
        const float sg = a.x + b.x, tt = sg * ri, s2 = tt * tt, s6 = s2 * s2 * s2, s12 = s6 * s6;
        const float e4 = a.y * b.y, sc = S.scale14;
        const double ulj = (double)(sc * e4 * (s12 - s6));
        const double dsg = (double)(sc * 0.5f * e4 * (12.0f * s12 - 6.0f * s6) * __builtin_amdgcn_rcpf(sg));
        atomicAdd(G + ij.x, (unsigned long long)fix_d(wr * ulj));
        atomicAdd(G + ij.y, (unsigned long long)fix_d(wr * ulj));
        atomicAdd(G + S.np + ij.x, (unsigned long long)fix_d(wr * dsg));
        atomicAdd(G + S.np + ij.y, (unsigned long long)fix_d(wr * dsg));
        atomicAdd(G + 2 * S.np + ij.x, (unsigned long long)fix_d(wr * (double)(sc * b.z * ri)));
        atomicAdd(G + 2 * S.np + ij.y, (unsigned long long)fix_d(wr * (double)(sc * a.z * ri)));
    }
    if (t < T.nt) {
        const int4 q = gld(gconst(T.t_ijkl) + t);
        const float ca = torsion_cos(pos(q.x), pos(q.y), pos(q.z), pos(q.w), gld(gconst(T.t_p) + t));
        atomicAdd(G + 3 * S.np + t, (unsigned long long)fix_d(wr * (double)(1.0f + ca)));
    }
}

__global__ void __launch_bounds__(256) k_grad_finish(const Dev *__restrict__ Sp, double *d_eps, double *d_sigma,
                                                     double *d_charge, double *d_tk)
{
    const Dev &S = *Sp;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const double sqrt_f = S.sqrt_f;
    if (a < S.n) {
        if (d_eps) d_eps[a] = unfix_d(S.gacc[a]) * S.inv2eps[a];
        if (d_sigma) d_sigma[a] = unfix_d(S.gacc[S.np + a]);
        if (d_charge) d_charge[a] = unfix_d(S.gacc[2 * S.np + a]) * sqrt_f;
    }
    if (a < S.tp.nt && d_tk) d_tk[S.tor_orig[a]] = unfix_d(S.gacc[3 * S.np + a]);
}

// dx[r] = w[r] dU_r/dx = -w[r] F_r, from the fixed-point forces
__global__ void __launch_bounds__(256) k_weighted_dx(const Dev *__restrict__ Sp, const double *w, float *dx)
{
    const Dev &S = *Sp;
    const int r = blockIdx.y;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < S.n) {
        const double wr = w[r];
        for (int d = 0; d < 3; ++d)
            dx[((size_t)r * 3 + d) * S.n + a] = (float)(-wr * unfix_d(S.F[((size_t)r * 3 + d) * S.np + a]));
    }
}

// energies and forces of every replica out of the fixed-point accumulators
__global__ void __launch_bounds__(256) k_unfix_out(const Dev *__restrict__ Sp, double *energy, float *forces)
{
    const Dev &S = *Sp;
    const int r = blockIdx.y;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a == 0 && energy) energy[r] = unfix_d(S.E[r]);
    if (a < S.n && forces) {
        for (int d = 0; d < 3; ++d)
            forces[((size_t)r * 3 + d) * S.n + a] = (float)unfix_d(S.F[((size_t)r * 3 + d) * S.np + a]);
    }
}

// ================================================================== persistent path
// Phase timers, in a build with GPR_PHASE_PROBE defined (a measurement library built beside
// the product one; the product build has none of this).  Thread 0 of every workgroup reads
// the constant-rate clock at the ends of the phases of each step and adds the differences,
// per (replica, group), to gpr_phase_acc[(r * PHASE_MAX_G + g) * NPHASE + k]; the phases end
// at workgroup barriers the body has anyway, so thread 0's clock marks the group's progress.
// The timers add a few instructions per phase and change no result.
#ifdef GPR_PHASE_PROBE
__device__ unsigned long long gpr_phase_acc[PHASE_MAX_R * PHASE_MAX_G * NPHASE];
// (the last reading is kept in LDS too, so that no register is held across the phases)
#define PHASE_MARK(k)                                                       \
    do {                                                                    \
        if (tid == 0) {                                                     \
            const unsigned long long t_ = __builtin_amdgcn_s_memrealtime(); \
            ph_acc[(k)] += t_ - ph_acc[NPHASE];                             \
            ph_acc[NPHASE] = t_;                                            \
        }                                                                   \
    } while (0)
#define PHASE_COUNT(k) do { if (tid == 0) ph_acc[(k)] += 1; } while (0)
#else
#define PHASE_MARK(k) ((void)0)
#define PHASE_COUNT(k) ((void)0)
#endif

hipError_t phase_take(unsigned long long *out, int R, hipStream_t st)
{
#ifdef GPR_PHASE_PROBE
    if (R < 1 || R > PHASE_MAX_R) return hipErrorInvalidValue;
    const size_t bytes = sizeof(unsigned long long) * (size_t)R * PHASE_MAX_G * NPHASE;
    void *acc = nullptr;
    hipError_t e = hipGetSymbolAddress(&acc, HIP_SYMBOL(gpr_phase_acc));
    if (e == hipSuccess) e = hipMemcpyAsync(out, acc, bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemsetAsync(acc, 0, bytes, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
#else
    (void)out; (void)R; (void)st;
    return hipErrorNotSupported;
#endif
}

// Barrier among the G workgroups of one replica: every thread waits for its own global
// stores to complete, then one thread adds to the replica's counter (device-scope relaxed
// atomic) and waits, with a bounded spin, for all G arrivals of this generation.  Data
// exchanged between the groups is written and read with device-scope relaxed atomics, so
// no cache writeback or invalidation is needed.  Returns false after a timeout.
__device__ __forceinline__ bool group_barrier(int *ctr, int target, int *err, int *sbuf)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int spins = 0, ok = 1;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > SPIN_MAX) {
                atomicOr(err + ERR_BARRIER, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        *sbuf = ok;
    }
    __syncthreads();
    const bool ok = *sbuf != 0;
    __syncthreads();
    return ok;
}

__device__ __forceinline__ void st_coh(float *p, float v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ float ld_coh(const float *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
// (x, y) of one atom as one 64-bit word, for the position exchange
__device__ __forceinline__ void st_coh2(unsigned long long *p, float x, float y)
{
    const unsigned long long w = (unsigned long long)__float_as_uint(x) | ((unsigned long long)__float_as_uint(y) << 32);
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float2 ld_coh2(const unsigned long long *p)
{
    const unsigned long long w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((unsigned)w), __uint_as_float((unsigned)(w >> 32)));
}

// G workgroups per replica advance nsteps BAOAB steps.  Group g of replica r owns the atoms
// [a0, a1) = [sp.bnd[g], sp.bnd[g + 1]) (ranges chosen on the host to even out the work); its LDS holds the positions (float4 with the
// scaled charge) and LJ parameters of every atom of the replica, and the velocities and
// fixed-point force accumulators of its own atoms (the accumulators carry the forces from one
// step to the next), block spheres and reduction scratch.  Per step: B A O A of own atoms ->
// (G > 1) positions exchanged through device-coherent stores, barrier -> pair-list rebuild of
// own atoms when due -> bonded terms touching own atoms (LDS atomics) -> pair forces of own
// atoms (P lanes per atom) -> closing B; every t_GR steps (t counted from t0) the observables
// of workers are accumulated by group 0.  With state_end group 0 writes the state id.
// Workgroups map to replicas so that a replica's groups are meant to share an XCD (equal
// blockIdx mod 8) when the replica count allows; results do not depend on G, the block size or
// the placement.
// Pair-loop order of a group's nl atoms.  A task of the pair loop is 16 atoms on the 64 lanes
// of a wave and runs as long as its longest list, so the atoms go longest list first (key: the
// atom's longest sub-list, in words): tasks of similar lists, taken heaviest first.  perm has
// 16 * ceil(nl / 16) slots; those past nl hold 0xFFFF.  Forces do not depend on the order: an
// atom's four lanes stay together and sum its own sub-lists in their fixed order.
__device__ void order_atoms(const unsigned short *key, unsigned short *perm, int *hist, int nl, int tid, int nthr)
{
    const int nt = (nl + 15) >> 4;
    for (int k = tid; k < 16 * nt; k += nthr) perm[k] = 0xFFFF;
    for (int k = tid; k < 64; k += nthr) hist[k] = 0;
    __syncthreads();
    for (int l = tid; l < nl; l += nthr) atomicAdd(&hist[63 - min((int)key[l], 63)], 1);
    __syncthreads();
    if (tid < 64) {                                        // exclusive prefix sum of the bins
        const int c = hist[tid];
        int x = c;
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d, 64);
            if (tid >= d) x += y;
        }
        hist[tid] = x - c;
    }
    __syncthreads();
    for (int l = tid; l < nl; l += nthr) {
        const int k = atomicAdd(&hist[63 - min((int)key[l], 63)], 1);
        perm[k] = (unsigned short)l;
    }
    __syncthreads();
}

__device__ __forceinline__ void persist_replica(const Dev &S, int G, int lmax, int a0, int a1, int r, int g,
                                                long long s0, int nsteps, int t0, int sample, int state_end)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int np = S.np, n = S.n;
    long long *fa = (long long *)lds_raw;                 // [3][lmax]
    long long *red = fa + 3 * lmax;                        // [MAX_OBS * 8 + 8]
    double *vals = (double *)(red + MAX_OBS * 8 + 8);      // [MAX_OBS]
    float4 *xs = (float4 *)(vals + MAX_OBS);               // [np]
    float2 *pp = (float2 *)(xs + np);                      // [np]
    float *vs = (float *)(pp + np);                        // [3][lmax]
    float *iml = vs + 3 * lmax;                            // [lmax] 1/m of own atoms
    float *sdl = iml + lmax;                               // [lmax] noise amplitude of own atoms
    float *xbl = sdl + lmax;                               // [3][lmax] own positions at the last list build
    float4 *sph = (float4 *)(xbl + 3 * lmax);              // [nblk]
    int *wscr = (int *)(sph + (n + BLK - 1) / BLK);        // [16][WBLK] build scratch per wave
    unsigned short *perm = (unsigned short *)(wscr + 16 * WBLK);   // [16 ceil(lmax / 16)] pair-loop order
    unsigned short *keyl = perm + 16 * ((lmax + 15) >> 4);  // [lmax] groups in each of an atom's sub-lists
    __shared__ int sbuf, bbuf, hbuf, hist[64], ptask, btask;

    const int tid = threadIdx.x, BT = blockDim.x;
#ifdef GPR_PHASE_PROBE
    __shared__ unsigned long long ph_acc[NPHASE + 1];
    if (tid < NPHASE) ph_acc[tid] = 0;
#endif
    const size_t b = (size_t)r * 3 * np;
    GPR_GLOBAL float *xg = gmut(S.x) + b, *xbg = gmut(S.xb) + b;
    float *vg = S.v + b;
    GPR_GLOBAL long long *Fg = gmut(S.F) + b;
    const GPR_GLOBAL float4 *prm = gconst(S.prm);
    const GPR_GLOBAL float *sdv = gconst(S.sd);
    int *sync = S.sync + (size_t)r * 64;
    // position exchange, one buffer per step parity: a group writes step s + 1 only after the
    // barrier of step s, which every group passes after reading step s - 1
    unsigned long long *xch_xy0 = (unsigned long long *)(S.xchg + 2 * b);        // [2][np] (x, y)
    float *xch_z0 = S.xchg + 2 * b + 4 * np;                                        // [2][np] z
    int gen = 0;

#ifdef GPR_PHASE_PROBE
    if (tid == 0) ph_acc[NPHASE] = ph_acc[PH_START] = __builtin_amdgcn_s_memrealtime();
#endif
    stage_replica(S, r, xs, pp, tid, BT);
    for (int k = tid; k < 3 * lmax; k += BT) {
        const int d = k / lmax, a = a0 + k % lmax;
        vs[k] = a < a1 ? gconst(vg)[d * np + a] : 0.f;
        fa[k] = a < a1 ? Fg[d * np + a] : 0;
        xbl[k] = a < a1 ? xbg[d * np + a] : 0.f;
    }
    for (int l = tid; l < lmax; l += BT) {
        const int a = a0 + l;
        iml[l] = a < a1 ? gld(prm + a).w : 0.f;
        sdl[l] = a < a1 ? sdv[a] : 0.f;
    }
    // the pair loop below runs each atom's four sub-lists to one count, which needs lists
    // padded as this kernel's search writes them: lists from the plain path's search, or a
    // replica marked for a rebuild (a new configuration), are rebuilt at the first step;
    // padded lists from an earlier launch are kept, their counts and order recomputed
    const bool toy = S.kind == KIND_TOY;
    bool need = !toy && (S.need_build[r] != 0 || S.list_pad[r] == 0);
    long long lastb = S.last_build[(s0 & 1) * S.R + r];     // step of the last pair-list build
    const int nl = a1 - a0, nslot = 16 * ((nl + 15) >> 4);
    if (!toy && !need) {
        const size_t stride = (size_t)np * P;
        const GPR_GLOBAL unsigned short *cnt = gconst(S.nbc) + (size_t)r * stride;
        for (int l = tid; l < nl; l += BT) {
            const int i = a0 + l;
            int k = 0;
#pragma unroll
            for (int q = 0; q < P; ++q) k = max(k, (int)cnt[(size_t)i * P + q]);
            keyl[l] = (unsigned short)k;
        }
        __syncthreads();
        order_atoms(keyl, perm, hist, nl, tid, BT);
    }
    __syncthreads();
    // descriptor fields used every step, held in registers for the launch
    const IntConsts ik = int_consts(S);
    const int t_gr = S.t_gr, need_energy = S.need_energy, cutoff_on = S.cutoff_on, period = S.period;
    const float half_skin2 = S.half_skin2;
    int *const errp = S.err;
    // with several groups every wave waits at the barrier on its own and then takes its share
    // of the other groups' positions: one round trip of device-coherent reads per step
    const bool split = G > 1 && !toy && BT >= 128;
    // the bonded terms touching the group's atoms, on its last (up to) eight waves: their
    // topology loads wait on memory, and the other waves meanwhile start the pair tasks
    const BondedPlan bplan = bonded_plan(S, a0, a1);
    const int nwv = BT >> 6, nbw = min(nwv, 8), bw0 = nwv - nbw;
    long long *eacc = red + MAX_OBS * 8;
    bool alive = true;
    bool pend = false;                                      // the previous step's closing B is due
    PHASE_MARK(PH_PROLOGUE);

    for (int step = 0; step < nsteps && alive; ++step) {
        const long long s = s0 + step;
        const int tl = t0 + step + 1;
        const bool samp = sample && r >= 1 && (tl % t_gr == 0);
        const bool energy = samp && need_energy;
        unsigned long long *xch_xy = xch_xy0 + (s & 1) * np;
        float *xch_z = xch_z0 + (s & 1) * np;
        int hit = 0, bad = 0;
        for (int a = a0 + tid; a < a1; a += BT) {
            const int l = a - a0;
            float3 x = make_float3(xs[a].x, xs[a].y, xs[a].z);
            float3 v = make_float3(vs[l], vs[lmax + l], vs[2 * lmax + l]);
            const float3 F = make_float3(unfix_f(fa[l]), unfix_f(fa[lmax + l]), unfix_f(fa[2 * lmax + l]));
            if (pend) {
                // the previous step's closing B, deferred to here (same forces, same order)
                const float im = iml[l];
                v.x = kick(v.x, F.x, ik.h, im);
                v.y = kick(v.y, F.y, ik.h, im);
                v.z = kick(v.z, F.z, ik.h, im);
                bad |= bad_force(F.x) || bad_force(F.y) || bad_force(F.z);
            }
            integrate_baoa_k(ik, a, r, s, x, v, F, iml[l], sdl[l]);
            xs[a].x = x.x; xs[a].y = x.y; xs[a].z = x.z;
            vs[l] = v.x; vs[lmax + l] = v.y; vs[2 * lmax + l] = v.z;
            if (G > 1) { st_coh2(xch_xy + a, x.x, x.y); st_coh(xch_z + a, x.z); }
            bad |= !(finite3(x) && finite3(v));
            if (cutoff_on) {
                const float dx = x.x - xbl[l], dy = x.y - xbl[lmax + l], dz = x.z - xbl[2 * lmax + l];
                hit |= !(dx * dx + dy * dy + dz * dz <= half_skin2);
            }
        }
        if (bad) atomicOr(&errp[ERR_UNSTABLE], 1);
        int any_hit;
        if (G > 1) {
            // displacement-guard flags in three rotating slots; group 0 clears the slot of the next step
            if (hit) __hip_atomic_fetch_or(sync + 16 + 16 * (int)(s % 3), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (g == 0 && tid == 0) __hip_atomic_store(sync + 16 + 16 * (int)((s + 1) % 3), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (split) {
                // arrive; each wave waits (bounded spin by its first lane), then all threads
                // fetch the other groups' positions
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();                     // own positions stored, forces read
                PHASE_MARK(PH_INTEGRATE);
                if (tid == 0) {
                    __hip_atomic_fetch_add(sync, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bbuf = 1;
                }
                for (int k = tid; k < 3 * lmax; k += BT) fa[k] = 0;
                if (tid == 0) { *eacc = 0; ptask = 0; }
                __syncthreads();
                const int target = G * ++gen;
                if ((tid & 63) == 0) {
                    int spins = 0;
                    while (__hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                        if (++spins > SPIN_MAX) {
                            atomicOr(errp + ERR_BARRIER, 1);
                            bbuf = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __builtin_amdgcn_wave_barrier();
                if (tid == 0) hbuf = __hip_atomic_load(sync + 16 + 16 * (int)(s % 3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // all loads of a batch in flight before the first LDS write
                constexpr int XU = 4;
                for (int a0x = 0; a0x < n; a0x += XU * BT) {
                    float2 xy[XU];
                    float z[XU];
#pragma unroll
                    for (int u = 0; u < XU; ++u) {
                        const int a = a0x + u * BT + tid;
                        const bool other = a < n && (a < a0 || a >= a1);
                        xy[u] = other ? ld_coh2(xch_xy + a) : make_float2(0.f, 0.f);
                        z[u] = other ? ld_coh(xch_z + a) : 0.f;
                    }
#pragma unroll
                    for (int u = 0; u < XU; ++u) {
                        const int a = a0x + u * BT + tid;
                        if (a < n && (a < a0 || a >= a1)) { xs[a].x = xy[u].x; xs[a].y = xy[u].y; xs[a].z = z[u]; }
                    }
                }
                __syncthreads();
                alive = bbuf != 0;
                if (!alive) break;
            } else {
                alive = group_barrier(sync, G * ++gen, errp, &bbuf);
                if (!alive) break;
                if (tid == 0) hbuf = __hip_atomic_load(sync + 16 + 16 * (int)(s % 3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int a = tid; a < n; a += BT) {
                    if (a >= a0 && a < a1) continue;
                    const float2 xy = ld_coh2(xch_xy + a);
                    xs[a].x = xy.x; xs[a].y = xy.y; xs[a].z = ld_coh(xch_z + a);
                }
                __syncthreads();
            }
            any_hit = hbuf;
        } else {
            any_hit = __syncthreads_or(hit);
            PHASE_MARK(PH_INTEGRATE);
        }
        PHASE_MARK(PH_EXCHANGE);
        // each replica is its own set of workgroups here, so its list is rebuilt when it is
        // period steps old (or flagged), independently of the other replicas
        if (need || (cutoff_on && (any_hit || s - lastb >= period))) {
            PHASE_COUNT(PH_NREBUILD);
            lastb = s;
            // The search in tasks of 16 consecutive atoms (one wave each), costliest first by
            // the lists of the last build (the summed longest sub-lists of the task's atoms),
            // taken by the waves from a counter as they come free.  The order changes no list:
            // each lane builds its own sub-list.  The costs sit in the waves' search scratch
            // until the search starts (16 WBLK ints hold the tasks of 16,384 atoms).
            const int ntk = (nl + 15) >> 4;
            int *tcost = wscr;
            for (int c = tid; c < ntk; c += BT) {
                int sum = 0;
                for (int l = 16 * c; l < min(16 * c + 16, nl); ++l) sum += keyl[l];
                tcost[c] = sum;
            }
            if (tid == 0) btask = 0;
            block_spheres(S, xs, sph, tid, BT);
            __syncthreads();
            for (int c = tid; c < ntk; c += BT) {
                const int mine = tcost[c];
                int rank = 0;
                for (int d = 0; d < ntk; ++d) rank += (tcost[d] > mine) | (tcost[d] == mine && d < c);
                perm[rank] = (unsigned short)c;
            }
            __syncthreads();
            for (;;) {
                int t = 0;
                if ((tid & 63) == 0) t = atomicAdd(&btask, 1);
                t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
                if (t >= ntk) break;
                const int c = __builtin_amdgcn_readfirstlane((int)perm[t]);
                const int L = a0 * P + 64 * c + (tid & 63), i = L / P, q = L % P;
                const bool valid = L < a1 * P;
                const int ngw = build_wave<4, true>(S, r, i, q, valid, (const GPR_LDS gv_f4 *)xs,
                                              (const GPR_LDS gv_f4 *)sph, (GPR_LDS int *)wscr + (tid >> 6) * WBLK,
                                              false);
                if (valid && q == 0) {
                    const int l = i - a0;
                    xbl[l] = xs[i].x; xbl[lmax + l] = xs[i].y; xbl[2 * lmax + l] = xs[i].z;
                    keyl[l] = (unsigned short)ngw;
                }
            }
            __syncthreads();                     // every task has read its entry of perm
            order_atoms(keyl, perm, hist, nl, tid, BT);
            if (need && g == 0 && tid == 0) S.list_pad[r] = 1;
            need = false;
        }
        PHASE_MARK(PH_REBUILD);
        if (!split) {
            for (int k = tid; k < 3 * lmax; k += BT) fa[k] = 0;
            if (tid == 0) { *eacc = 0; ptask = 0; }
            __syncthreads();
        }
        if (toy) {
            if (tid == 0 && a0 == 0 && a1 > 0) {
                float fx, fy;
                const float u = toy_force(xs[0].x, xs[0].y, fx, fy);
                fa[0] = fix_f(fx);
                fa[lmax] = fix_f(fy);
                if (energy) *eacc = fix_f(u);
            }
        } else {
            // bonded terms on the last waves, then the pair loop, whose tasks (16 atoms each,
            // longest lists first) the waves take from a shared counter as they come free
            if ((tid >> 6) >= bw0)
                bonded_range<PosLDS, 2>(S, bplan, PosLDS{xs}, a0, a1, fa, lmax, energy ? eacc : nullptr, tid - bw0 * 64,
                                        nbw * 64);
            const int ntask = nslot >> 4;
            const NbConsts nbk = nb_consts(S);
            for (;;) {
                int t = 0;
                if ((tid & 63) == 0) t = atomicAdd(&ptask, 1);
                t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
                if (t >= ntask) break;
                const int q = tid & 3;
                const int l = perm[16 * t + ((tid & 63) >> 2)];
                long long eatom = 0;
                if (l != 0xFFFF) {
                    const int i = a0 + l;
                    float4 f = nb_lane(nbk, r, i, q, xs, pp, energy, keyl[l]);
                    f.x = quad_sum(f.x);
                    f.y = quad_sum(f.y);
                    f.z = quad_sum(f.z);
                    if (energy) f.w = quad_sum(f.w);
                    if (q == 0) {
                        lds_add(&fa[l], fix_f(f.x));
                        lds_add(&fa[lmax + l], fix_f(f.y));
                        lds_add(&fa[2 * lmax + l], fix_f(f.z));
                        if (energy) eatom = fix_f(f.w);
                    }
                }
                if (energy) {
                    eatom = wave_sum_ll(eatom);
                    if ((tid & 63) == 0 && eatom != 0) lds_add(eacc, eatom);
                }
            }
        }
        __syncthreads();
        PHASE_MARK(PH_FORCES);
        // the closing B: here when the step's velocities are read (a sample, the end of the
        // launch), else by the next step's integrator
        pend = !(samp || step + 1 == nsteps);
        if (!pend) {
            for (int a = a0 + tid; a < a1; a += BT) {
                const int l = a - a0;
                const float im = iml[l], h = ik.h;
                const float Fx = unfix_f(fa[l]), Fy = unfix_f(fa[lmax + l]), Fz = unfix_f(fa[2 * lmax + l]);
                vs[l] = kick(vs[l], Fx, h, im);
                vs[lmax + l] = kick(vs[lmax + l], Fy, h, im);
                vs[2 * lmax + l] = kick(vs[2 * lmax + l], Fz, h, im);
                if (bad_force(Fx) || bad_force(Fy) || bad_force(Fz)) atomicOr(&errp[ERR_UNSTABLE], 1);
            }
        }
        if (samp) {
            __syncthreads();
            if (G == 1) {
                for (int k = tid; k < 3 * np; k += BT) gmut(vg)[k] = k % np < n ? vs[(k / np) * lmax + k % np] : 0.f;
                __syncthreads();
                observables_wg(S, xs, vg, unfix_d(*eacc), red, vals, tid, BT);
                if (tid == 0) accumulate_obs(S, r, vals);
            } else {
                // own velocities and energy to the group 0 of the replica
                for (int a = a0 + tid; a < a1; a += BT) {
                    const int l = a - a0;
                    st_coh(vg + a, vs[l]); st_coh(vg + np + a, vs[lmax + l]); st_coh(vg + 2 * np + a, vs[2 * lmax + l]);
                }
                if (tid == 0 && energy && *eacc != 0)
                    __hip_atomic_fetch_add(S.esum + r, *eacc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                alive = group_barrier(sync, G * ++gen, S.err, &bbuf);
                if (!alive) break;
                if (g == 0) {
                    __shared__ long long etot;
                    if (tid == 0) {
                        etot = __hip_atomic_load(S.esum + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(S.esum + r, 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    __syncthreads();
                    observables_wg(S, xs, vg, unfix_d(etot), red, vals, tid, BT, true);
                    if (tid == 0) accumulate_obs(S, r, vals);
                }
            }
        }
        __syncthreads();
        PHASE_MARK(PH_TAIL);
        PHASE_COUNT(PH_NSTEP);
    }
    // write back this group's atoms
    for (int a = a0 + tid; a < a1; a += BT) {
        const int l = a - a0;
        xg[a] = xs[a].x; xg[np + a] = xs[a].y; xg[2 * np + a] = xs[a].z;
        for (int d = 0; d < 3; ++d) {
            gmut(vg)[d * np + a] = vs[d * lmax + l];
            Fg[d * np + a] = fa[d * lmax + l];
            xbg[d * np + a] = xbl[d * lmax + l];
        }
    }
    if (g == 0 && tid == 0 && nsteps > 0) {
        S.need_build[r] = 0;
        S.last_build[((s0 + nsteps) & 1) * S.R + r] = lastb;
    }
    if (state_end && g == 0) {
        __syncthreads();
        const int id = state_wg(S, xs, red, &sbuf, tid, BT);
        if (tid == 0) S.state[r] = id;
    }
    if (G > 1 && nsteps > 0) {
        // the replica's barrier line is left clear for the next launch by the last of its groups
        // to finish (each group counts itself out in slot 8 once none of its waves reads the
        // line again), so that no launch needs it cleared beforehand
        __syncthreads();
        if (tid == 0 && __hip_atomic_fetch_add(sync + 8, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == G - 1) {
            __hip_atomic_store(sync, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int k = 16; k < 64; k += 16) __hip_atomic_store(sync + k, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(sync + 8, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
#ifdef GPR_PHASE_PROBE
    PHASE_MARK(PH_EPILOGUE);
    if (tid == 0 && r < PHASE_MAX_R && g < PHASE_MAX_G) {
        unsigned long long *acc = gpr_phase_acc + ((size_t)r * PHASE_MAX_G + g) * NPHASE;
        for (int k = 0; k < PH_START; ++k) acc[k] += ph_acc[k];
        acc[PH_START] = ph_acc[PH_START];
        acc[PH_END] = __builtin_amdgcn_s_memrealtime();
    }
#endif
}

// One system, one replica per set: replicas roff, roff + 1, ... (a system with more replicas
// than sets that fit at once takes several launches, each with the body inlined).
__global__ void __launch_bounds__(1024) k_persist(PersistItem it)
{
    int set, g;
    if (!persist_place(it, (int)blockIdx.x, set, g) || set + it.roff >= it.nrep) return;
    long long s0 = it.s0;
    int t0 = it.t0;
    if (it.cyc) {
        // cycle of a captured run: nothing after the check that ended the call
        if (it.cyc->halt_cycle < it.cycle) return;
        const long long first = (long long)it.cycle * it.nsteps;
        s0 = it.cyc->s_start + first;
        t0 = (int)((it.cyc->t_start + first) % it.dev->t_gr);
    }
    persist_replica(*it.dev, it.sp.G, it.sp.lmax, it.sp.bnd[g], it.sp.bnd[g + 1], set + it.roff, g, s0, it.nsteps,
                    t0, it.sample, it.state_end);
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni64(long long v)
{
    const int lo = uni((int)(unsigned)v), hi = uni((int)(v >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// the per-replica body as a function of its own (one call per replica and launch), so that
// the loop around it in k_persist_batch does not add to the body's register pressure.  The
// arguments of a call arrive in vector registers; they are wave-uniform, and made so again,
// so that the values and branches that depend on them stay scalar.
__device__ __noinline__ void persist_replica_call(const Dev *dev, int G, int lmax, int a0, int a1, int r, int g,
                                                  long long s0, int nsteps, int t0, int sample, int state_end)
{
    const Dev *d = (const Dev *)uni64((long long)dev);
    persist_replica(*d, uni(G), uni(lmax), uni(a0), uni(a1), uni(r), uni(g), uni64(s0), uni(nsteps), uni(t0),
                    uni(sample), uni(state_end));
}

// Several systems, each item's sets taking its replicas r = set, set + nsets, ... in turn.
__global__ void __launch_bounds__(1024) k_persist_batch(PersistBatch pb)
{
    int k = 0;
    while (k + 1 < pb.nitems && (int)blockIdx.x >= pb.it[k + 1].boff) ++k;
    const PersistItem &it = pb.it[k];
    int set, g;
    if (!persist_place(it, (int)blockIdx.x - it.boff, set, g)) return;
    for (int r = set; r < it.nrep; r += it.nsets) {
        persist_replica_call(it.dev, it.sp.G, it.sp.lmax, it.sp.bnd[g], it.sp.bnd[g + 1], r, g, it.s0, it.nsteps,
                             it.t0, it.sample, it.state_end);
        __syncthreads();
    }
}


// ================================================================== Gen.ParRep bookkeeping
// Sums over workers follow one canonical pairwise tree: the m terms padded with zeros to the
// next power of two p, each node the sum of its lower half and its upper half.  A wave
// evaluates it with lane l holding the c = max(1, p / 64) consecutive terms [l c, l c + c):
// their subtree inside the lane, then xor shuffles at partner distances 1, 2, 4, ... over the
// lanes that hold terms, which form exactly the upper levels of the tree (the two lanes of a
// pair add the same two values in either order, with identical bits).
constexpr int TREE_C = 16;                 // terms per lane summed in registers

// subtree of the c (a power of two) terms f(base .. base + c), those >= m being zero
template <class Fn>
__device__ __forceinline__ double lane_tree16(Fn f, int m, int base, int c)
{
    double e[TREE_C];
#pragma unroll
    for (int i = 0; i < TREE_C; ++i) e[i] = (i < c && base + i < m) ? f(base + i) : 0.0;
#pragma unroll
    for (int w = 1; w < TREE_C; w <<= 1)
#pragma unroll
        for (int i = 0; i + w < TREE_C; i += 2 * w)
            if (w < c) e[i] += e[i + w];
    return e[0];
}

template <class Fn>
__device__ double lane_tree(Fn f, int m, int base, int c)
{
    if (c <= TREE_C) return lane_tree16(f, m, base, c);
    // more terms than registers: subtrees of TREE_C terms merged in order by a binary counter
    // (a new subtree is added to the pending one of its own height, lower half first)
    double stk[12];
    int lvl[12], sp = 0;
    for (int b = 0; b < c; b += TREE_C) {
        double v = lane_tree16(f, m, base + b, TREE_C);
        int L = 0;
        while (sp > 0 && lvl[sp - 1] == L) { v = stk[--sp] + v; ++L; }
        stk[sp] = v; lvl[sp] = L; ++sp;
    }
    return stk[0];
}

// the whole wave: the tree over f(0 .. m), in every lane that holds terms
template <class Fn>
__device__ double wave_pairwise(Fn f, int m)
{
    int p = 1;
    while (p < m) p <<= 1;
    const int lanes = p > 64 ? 64 : p, c = p > 64 ? p / 64 : 1;
    const int lane = threadIdx.x & 63;
    double v = lane < lanes ? lane_tree(f, m, lane * c, c) : 0.0;
    for (int o = 1; o < lanes; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Gelman-Rubin R-hat (Eq. 3) of one observable over nw workers from the shifted sums S1, S2
// of n samples; the whole wave calls it, the value is valid in lane 0
template <class F1, class F2>
__device__ double rhat_wave(int nw, long long n, F1 s1, F2 s2)
{
    const double dn = (double)n, dw = (double)nw;
    const double m1 = wave_pairwise([&](int k) { return s1(k) / dn; }, nw) / dw;
    const double m2 = wave_pairwise([&](int k) { return s2(k) / dn; }, nw) / dw;
    const double den = wave_pairwise([&](int k) {
        const double ob = s1(k) / dn;
        const double a = s2(k) / dn;
        const double o2 = ob * ob;
        return a - o2;
    }, nw) / dw;
    const double m1sq = m1 * m1;
    const double num = m2 - m1sq;
    return den > 0.0 ? num / den : __longlong_as_double(0x7FF0000000000000LL);
}

// Survivors of a check (Sec. 2.4.1): the workers r >= 1 not exited, ascending, into surv[];
// returns their number.  Block-collective (blockDim a multiple of 64); wsum: LDS int[16].
template <class Ex>
__device__ int survivors_block(int R, Ex exited, int *surv, int *wsum)
{
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
    int run = 0;
    for (int base = 1; base < R; base += nthr) {
        const int r = base + tid;
        const bool f = r < R && !exited(r);
        const unsigned long long m = __ballot(f);
        const int pre = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (lane == 0) wsum[wv] = __popcll(m);
        __syncthreads();
        int off = run, tot = 0;
        for (int k = 0; k < nwv; ++k) {
            off += k < wv ? wsum[k] : 0;
            tot += wsum[k];
        }
        if (f) surv[off + pre] = r;
        run += tot;
        __syncthreads();
    }
    return run;
}

// Fleming-Viot donor of worker r at the check of global step s (Sec. 2.4.1): -1 for a
// survivor, S[(u |S|) >> 32] for an exited worker (u the first Philox word of (0, s, r,
// stream 2), S the ascending survivors, ns = |S|), -2 for every worker when no worker
// survived; replica 0 (the reference walker) is never branched: -1, or -2 with no survivor.
template <class Ex>
__device__ __forceinline__ int fv_donor(uint32_t k0, uint32_t k1, long long s, int r, Ex exited, const int *surv, int ns)
{
    if (ns == 0) return -2;
    if (r == 0 || !exited(r)) return -1;
    const uint4 w = philox_ctr(0u, s, (uint32_t)r, STREAM_BRANCH, k0, k1);
    const unsigned long long pick = ((unsigned long long)w.x * (unsigned long long)ns) >> 32;
    return surv[pick];
}

// Exit vote of Eq. 5 on first-exit check indices (0: no exit): M = the smallest positive
// fec, k = 1 + the smallest r with fec[r] = M, tau = (R (M - 1) + k) t_check; (0, 0, 0) when
// no replica exited.  Block-collective; the result is valid in thread 0.  red: LDS long long[32].
template <class Fec>
__device__ void vote_block(int R, Fec fec, long long t_check, long long *red, long long *M, int *k, long long *tau)
{
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
    // key = (fec, r) ordered lexicographically; no exit is the largest key
    long long bf = 0x7FFFFFFFFFFFFFFFLL;
    int br = 0x7FFFFFFF;
    for (int r = tid; r < R; r += nthr) {
        const long long f = fec(r);
        if (f > 0 && (f < bf || (f == bf && r < br))) { bf = f; br = r; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const long long of = __shfl_xor(bf, o, 64);
        const int orr = __shfl_xor(br, o, 64);
        if (of < bf || (of == bf && orr < br)) { bf = of; br = orr; }
    }
    if (lane == 0) { red[2 * wv] = bf; red[2 * wv + 1] = br; }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < nwv; ++w) {
            const long long of = red[2 * w];
            const int orr = (int)red[2 * w + 1];
            if (of < bf || (of == bf && orr < br)) { bf = of; br = orr; }
        }
        if (bf == 0x7FFFFFFFFFFFFFFFLL) { *M = 0; *k = 0; *tau = 0; }
        else { *M = bf; *k = br + 1; *tau = ((long long)R * (bf - 1) + (br + 1)) * t_check; }
    }
    __syncthreads();
}

// Per-check bookkeeping and Fleming-Viot clone-on-kill in one launch; blocks of 256
// threads, grid (nx, ny).  Block (0, 0) writes the status: CHK_STATE reports replica 0's
// state; CHK_DEPHASE takes the reference-exit test, the branching plan (donor[], surv[])
// and R-hat over the workers with the sums they hold after this check's branching;
// CHK_PARALLEL records the replicas outside Omega at check `check_index` and takes the exit
// vote of Eq. 5 (M, k, tau; to_state of replica k - 1); CHK_ADVANCE records first exit
// checks in fec[] and computes, but does not act on, the plan and R-hat.  With CHK_DEPHASE
// the blocks of row y = r (ny = R) copy (x, v, F) of replica r's donor into replica r when
// r was killed (a slice of nx blocks each), mark r for a pair-list rebuild and copy the
// donor's observable sums (cleared when every worker is re-copied from the reference).
__global__ void __launch_bounds__(256) k_check(const Dev *__restrict__ Sp, int mode, long long s, int omega, int nrep,
                                               long long nsamp, long long check_index, long long t_check, Status *st,
                                               int *donor, int *surv, long long *fec, CycRec *cyc, int cycle)
{
    const Dev &S = *Sp;
    const int tid = threadIdx.x;
    const int r = blockIdx.y;
    __shared__ int wsum[16];
    __shared__ long long red[32];
    __shared__ int sh_ne;
    __shared__ double rh_l[MAX_OBS];
    const int *state = S.state;
    auto ex = [&](int q) { return state[q] != omega; };
    const bool head = blockIdx.x == 0 && r == 0;
    long long t_now = 0;                                   // cycle mode: steps of the call at this check
    if (cyc) {
        // cycle `cycle` of a captured run: its step, check index and status slot; nothing after
        // the check that ended the call
        if (cyc->halt_cycle < cycle) return;
        omega = cyc->omega;
        const long long after = (long long)(cycle + 1) * cyc->nsteps;
        s = cyc->s_start + after;
        check_index = cyc->M_start + cycle + 1;
        t_now = cyc->t_start + after;
        st += cycle;
        if (head) nsamp = cyc->nsamp + (t_now / S.t_gr - (t_now - cyc->nsteps) / S.t_gr);
    }
    if (mode == CHK_DEPHASE) {
        if (state[0] != omega) {
            // the reference walker left Omega: nothing is branched
            if (head && tid == 0) {
                st->mode = mode; st->ref_exited = 1; st->n_exited = 0; st->n_surv = 0; st->k = 0;
                st->M = 0; st->tau = 0; st->to_state = state[0];
                for (int e = 0; e < 4; ++e) st->err[e] = S.err[e];
                for (int j = 0; j < MAX_OBS; ++j) st->rhat[j] = __longlong_as_double(0x7FF0000000000000LL);
                if (cyc) { cyc->nsamp = nsamp; cyc->halt_cycle = cycle; }
            }
            return;
        }
        if (!head && (r == 0 || !ex(r))) return;          // survivors are never copied
    } else if (!head) {
        return;
    }
    // survivors (every block that needs a donor): into the global list from block (0, 0),
    // into LDS elsewhere
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int *sl = head ? surv : (int *)lds_raw;
    const int ns = survivors_block(nrep, ex, sl, wsum);
    if (!head) {
        // an exited worker: copy its donor (the reference walker when no worker survived)
        __syncthreads();
        const int d = ns == 0 ? 0 : fv_donor(S.key0, S.key1, s, r, ex, sl, ns);
        const size_t bs = (size_t)d * 3 * S.np, bd = (size_t)r * 3 * S.np;
        for (int k = blockIdx.x * blockDim.x + tid; k < 3 * S.np; k += gridDim.x * blockDim.x) {
            S.x[bd + k] = S.x[bs + k];
            S.v[bd + k] = S.v[bs + k];
            S.F[bd + k] = S.F[bs + k];
        }
        if (blockIdx.x == 0 && tid == 0) S.need_build[r] = 1;
        if (blockIdx.x == 0 && tid < 2 * MAX_OBS)
            S.acc[(size_t)r * 2 * MAX_OBS + tid] = d == 0 ? 0.0 : S.acc[(size_t)d * 2 * MAX_OBS + tid];
        return;
    }
    // block (0, 0): the plan, the status and R-hat
    if (tid == 0) { sh_ne = 0; }
    __syncthreads();
    int ne = 0;
    for (int q = tid; q < nrep; q += blockDim.x) {
        const int dq = fv_donor(S.key0, S.key1, s, q, ex, sl, ns);
        if (mode == CHK_DEPHASE || mode == CHK_ADVANCE) donor[q] = dq;
        ne += q > 0 && ex(q);
        if (mode == CHK_ADVANCE && fec[q] == 0 && ex(q)) fec[q] = check_index;
    }
    for (int o = 32; o > 0; o >>= 1) ne += __shfl_xor(ne, o, 64);
    if ((tid & 63) == 0 && ne) atomicAdd(&sh_ne, ne);
    long long vM = 0, vtau = 0;
    int vk = 0;
    if (mode == CHK_PARALLEL)
        vote_block(nrep, [&](int q) { return ex(q) ? check_index : 0ll; }, t_check, red, &vM, &vk, &vtau);
    __syncthreads();
    if (tid == 0) {
        st->mode = mode;
        st->ref_exited = 0;
        st->n_exited = (mode == CHK_DEPHASE || mode == CHK_ADVANCE) ? sh_ne : 0;
        st->n_surv = (mode == CHK_DEPHASE || mode == CHK_ADVANCE) ? ns : 0;
        st->k = vk;
        st->M = vM;
        st->tau = vtau;
        st->to_state = state[vk > 0 ? vk - 1 : 0];
        for (int e = 0; e < 4; ++e) st->err[e] = S.err[e];
    }
    if (mode == CHK_DEPHASE || mode == CHK_ADVANCE) {
        // one wave per observable; after this check's branching a killed worker holds its
        // donor's sums, and with no survivor every worker restarts (R-hat undefined)
        const int wv = tid >> 6, nwv = blockDim.x >> 6;
        for (int j = wv; j < MAX_OBS; j += nwv) {
            double rh = __longlong_as_double(0x7FF0000000000000LL);
            const bool skip = (mode == CHK_DEPHASE && ns == 0) || nsamp < 1 || j >= S.nobs;
            if (!skip) {
                auto src = [&](int k) {
                    const int q = k + 1;
                    return (mode == CHK_DEPHASE && donor[q] >= 0) ? donor[q] : q;
                };
                auto s1 = [&](int k) { return S.acc[((size_t)src(k) * MAX_OBS + j) * 2]; };
                auto s2 = [&](int k) { return S.acc[((size_t)src(k) * MAX_OBS + j) * 2 + 1]; };
                rh = rhat_wave(nrep - 1, nsamp, s1, s2);
            }
            if ((tid & 63) == 0) { st->rhat[j] = rh; rh_l[j] = rh; }
        }
    }
    if (cyc) {
        // the decision the host takes from the status, taken here so that the later cycles of
        // the run know whether to run: converged (Eq. 4 test, with the samples restarted when
        // every worker was re-copied) or a first exit in the parallel step
        __syncthreads();
        if (tid == 0) {
            bool halt = false;
            if (mode == CHK_DEPHASE) {
                const long long nafter = (ns == 0 && nrep > 1) ? 0 : nsamp;
                bool conv = t_now >= S.t_min && nafter >= 2;
                for (int j = 0; j < S.nobs && conv; ++j) conv = rh_l[j] < 1.0 + S.tol;
                cyc->nsamp = nafter;
                halt = conv;
            } else if (mode == CHK_PARALLEL) {
                halt = vk > 0;
            }
            if (halt) cyc->halt_cycle = cycle;
        }
    }
}

// Copies (x, v, F) of replica donor[r] into replica r for every r with donor[r] >= 0 and
// marks r for a pair-list rebuild; observable sums are copied too (acc_mode 1), or cleared
// when the donor is the reference walker (a fresh broadcast).
__global__ void __launch_bounds__(256) k_clone(const Dev *__restrict__ Sp, const int *donor, int acc_mode)
{
    const Dev &S = *Sp;
    const int r = blockIdx.y;
    const int d = donor[r];
    if (d < 0 || d == r) return;
    const size_t bs = (size_t)d * 3 * S.np, bd = (size_t)r * 3 * S.np;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < 3 * S.np; k += gridDim.x * blockDim.x) {
        S.x[bd + k] = S.x[bs + k];
        S.v[bd + k] = S.v[bs + k];
        S.F[bd + k] = S.F[bs + k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) S.need_build[r] = 1;
    if (acc_mode && blockIdx.x == 0 && threadIdx.x < 2 * MAX_OBS) {
        S.acc[(size_t)r * 2 * MAX_OBS + threadIdx.x] = d == 0 ? 0.0 : S.acc[(size_t)d * 2 * MAX_OBS + threadIdx.x];
    }
}

// Maxwell-Boltzmann velocities of replica 0 (stream 1, step 0)
__global__ void __launch_bounds__(256) k_init_vel(const Dev *__restrict__ Sp, float kT)
{
    const Dev &S = *Sp;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.n) return;
    const float3 g = gauss3(philox_ctr((uint32_t)a, 0, 0u, STREAM_INIT, S.key0, S.key1));
    const float sdev = sqrtf(kT * S.prm[a].w);
    S.v[a] = sdev * g.x;
    S.v[S.np + a] = sdev * g.y;
    S.v[2 * S.np + a] = S.kind == KIND_TOY ? 0.0f : sdev * g.z;
}

// ------------------------------------------------------------------ building blocks
__global__ void __launch_bounds__(256) k_noise_test(uint32_t k0, uint32_t k1, int replica, long long step, int stream,
                                                    int n, uint32_t *words, float *gauss)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const uint4 w = philox_ctr((uint32_t)a, step, (uint32_t)replica, (uint32_t)stream, k0, k1);
    const float3 g = gauss3(w);
    words[4 * a] = w.x; words[4 * a + 1] = w.y; words[4 * a + 2] = w.z; words[4 * a + 3] = w.w;
    gauss[3 * a] = g.x; gauss[3 * a + 1] = g.y; gauss[3 * a + 2] = g.z;
}

// the branching plan of one check, by the routines k_check runs (one block of 256 threads)
__global__ void __launch_bounds__(256) k_fvplan_test(uint32_t k0, uint32_t k1, long long s, int R, const uint8_t *exited,
                                                     int *donor, int *surv)
{
    __shared__ int wsum[16];
    auto ex = [&](int r) { return exited[r] != 0; };
    const int ns = survivors_block(R, ex, surv, wsum);
    for (int r = threadIdx.x; r < R; r += blockDim.x) donor[r] = fv_donor(k0, k1, s, r, ex, surv, ns);
}

// R-hat of observable blockIdx.x, by the routine k_check runs (one wave per observable)
__global__ void __launch_bounds__(64) k_rhat_test(int nw, int nobs, long long n, const double *S1, const double *S2,
                                                  double *out)
{
    const int j = blockIdx.x;
    auto s1 = [&](int k) { return S1[(size_t)k * nobs + j]; };
    auto s2 = [&](int k) { return S2[(size_t)k * nobs + j]; };
    const double rh = rhat_wave(nw, n, s1, s2);
    if (threadIdx.x == 0) out[j] = rh;
}

// the exit vote of Eq. 5, by the routine k_check runs (one block of 256 threads)
__global__ void __launch_bounds__(256) k_vote_test(int R, const long long *fec, long long t_check, long long *out)
{
    __shared__ long long red[32];
    long long M, tau;
    int k;
    vote_block(R, [&](int r) { return fec[r]; }, t_check, red, &M, &k, &tau);
    if (threadIdx.x == 0) { out[0] = M; out[1] = k; out[2] = tau; }
}

} // namespace gpr
