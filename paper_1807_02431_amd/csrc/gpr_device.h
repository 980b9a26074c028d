// gpr_device.h -- device-side data layout and arithmetic of the MI355X Gen.ParRep hot path.
//
// Layout in HBM (per system; R replicas, n atoms padded to np = multiple of 64):
//   x, v      float  [R][3][np]   SoA per replica (coalesced per coordinate)
//   F         int64  [R][3][np]   forces in 64-bit fixed point, 2^-32 kJ/mol/nm per unit
//   xb        float  [R][3][np]   positions at the last pair-list build (displacement guard)
//   nbl       uint2  [R][Kg][np*P] pair lists in groups of four 16-bit partner indices,
//                                 slot-major: group g of sub-list (i, q) at g*np*P + i*P + q,
//                                 so the P lanes of consecutive atoms read consecutive 8-byte
//                                 words; the last group is padded with the dummy atom n
//   nbc       uint16 [R][np*P]    groups per sub-list
// Atom n (np >= n + 1) is a dummy placed far away with zero parameters: a pair with it
// contributes an exact zero.
//   acc       double [R][MAX_OBS][2]  observable sums S1, S2 (Eq. 2-3)
// Per-atom parameters (shared by all replicas): prm = (sigma/2, 2 sqrt(eps), q sqrt(f), 1/m).
//
// Determinism: every force contribution that is scattered (bonded terms) is rounded to the
// 2^-32 fixed-point grid and added as an integer; the nonbonded force of atom i is an FP32
// sum over P sub-lists, sub-list q holding the partners j = q (mod P) in ascending order,
// and pairs beyond the cutoff add an exact zero, so the sum does not depend on the list
// contents beyond the in-cutoff pairs, nor on launch shape or list rebuild times.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpr {

constexpr int P = 4;            // lanes per atom in the pair loop (sub-lists by j mod P)
constexpr int MAX_OBS = 8;
constexpr int CHMAX = 4;        // atoms per thread in the integrator mapping
constexpr int BLK = 8;          // consecutive atoms per bounding sphere in the pair search (a multiple of P)
constexpr int WBLK = 64;        // LDS ints per wave: the near blocks of one 64-block chunk in the pair search
constexpr double FIX = 4294967296.0;          // 2^32
constexpr double FIX_INV = 2.3283064365386963e-10;  // 2^-32
constexpr float FMAX_FIX = 2.5e5f;             // |F| beyond this (kJ/mol/nm) counts as unstable
constexpr float FSAT = 524287.0f;              // 2^19 - 1: fixed-point conversions saturate here
constexpr float FAR = 1.0e15f;                 // coordinate of the dummy atom
constexpr int SPIN_MAX = 1 << 22;              // bound on a barrier wait (then ERR_BARRIER)
// energy codes of the plain-path kernels: 0 / 1 given by the host; DCLK_* take the step s and
// the sampling decision from the device clock (so that a captured cycle of steps replays)
constexpr int DCLK_SAMPLE = 2;                 // workers' observables sampled every t_GR steps
constexpr int DCLK_NOSAMPLE = 3;

enum { KIND_TOY = 1, KIND_MOL = 2 };
enum { ST_SIGN_X = 1, ST_BOXES = 2, ST_COM = 3 };
enum { OB_COORD = 1, OB_POT = 2, OB_KIN = 3, OB_DIH = 4, OB_COMD = 5, OB_RMSV = 6 };
enum { STREAM_NOISE = 0, STREAM_INIT = 1, STREAM_BRANCH = 2 };
enum { ERR_UNSTABLE = 0, ERR_LIST = 1, ERR_BARRIER = 2 };

struct ObsDesc {
    int kind;
    int atoms[4];
    int ga_off, ga_n, gb_off, gb_n;
    double ma, mb;   // total masses of the groups
};

struct StateDesc {
    int kind;
    int atoms[8];
    int nbox;
    double box[8][4];
    int g_off, g_n;
    double gm;       // total mass of the group
    double center[3];
    double radius;
};

// bonded terms, each type sorted by its smallest atom index; *_start[a] is the first term
// whose smallest atom is >= a (length n+1); *_span the largest index spread of a term
struct Topo {
    int nb; const int2 *b_ij; const float2 *b_p; const int *b_start; int b_span;            // (r0, k)
    int na; const int4 *a_ijk; const float2 *a_p; const int *a_start; int a_span;           // (theta0, k)
    int nt; const int4 *t_ijkl; const float4 *t_p; const int *t_start; int t_span;          // (k, cos phi0, sin phi0, n)
    int nr; const int *r_i; const float4 *r_p; const int *r_start;                          // (ref xyz, k)
    int n14; const int2 *p_ij; const float4 *p_p; const int *p_start; int p_span;           // (s, 4e*sc, qq*sc)
};

struct Dev {
    int kind, n, np, R;
    const float4 *prm;
    const float *sd;                       // sqrt((1 - c1^2) kT / m)
    const float *mass;
    const unsigned long long *excl;        // bit (j - i + 32) set: pair excluded or 1-4
    int has_far;                           // some excluded or 1-4 pair lies 32 or more indices apart:
    const int *far_start, *far_j;          // [n + 1] offsets and ascending partners of those pairs
    float *x, *v, *xb;
    long long *F;
    long long *E;                          // [R] potential energy, fixed point
    uint2 *nbl;
    unsigned short *nbc;
    int Kg;                                // capacity of one sub-list, in groups of four
    int *guard;                            // [2][R] displacement guard flags by step parity
    int *need_build;                       // [R]
    int *list_pad;                         // [R] 1: the replica's lists are the persistent search's (sub-lists
                                           // of an atom padded to one count), 0: the plain search's
    long long *last_build;                 // [2][R] step of the last pair-list build, by step parity
    long long *clock;                      // [2]: global step s and steps t of the current call (device-clocked plain steps)
    int *err;                              // [4] error flags
    int *sync;                             // [R][64] per-replica barrier counter, flags, leave count (groups > 1)
    float *xchg;                           // [R][2][3][np] position exchange between a replica's groups (by step parity)
    long long *esum;                       // [R] energy partial sums of a replica's groups
    double *acc;                           // [R][MAX_OBS][2]
    double *shift;                         // [MAX_OBS]
    int *state;                            // [R]
    const int *groups;
    int nobs;
    int need_energy;                       // an observable is the potential energy
    const ObsDesc *obs;                    // [MAX_OBS], device memory
    const StateDesc *st;                   // device memory
    Topo tp;
    // force-field parameter gradient (molecular systems)
    long long *gacc;                       // [3][np] + [nt]: fixed-point sums for eps, sigma, charge, torsion k
    const double *inv2eps;                 // [n] 1 / (2 eps_i)
    const int *tor_orig;                   // [nt] caller's index of the k-th torsion in sorted order
    float scale14;
    double sqrt_f;                         // square root of the Coulomb constant
    float h, c1, rc2, rl, rl2, krf, crf, half_skin2;
    int cutoff_on, period;
    uint32_t key0, key1;
    int t_gr;
    double tol;                            // convergence: R-hat < 1 + tol for every observable
    long long t_min;                       // convergence: at least t_min steps of dephasing
};

// Pointers read from the device-resident descriptor are generic; casting them to the global
// address space makes the compiler emit global (not flat) memory instructions, whose
// completion is tracked apart from LDS traffic.
#define GPR_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const GPR_GLOBAL T *gconst(const T *p) { return (const GPR_GLOBAL T *)p; }
template <class T>
__device__ __forceinline__ GPR_GLOBAL T *gmut(T *p) { return (GPR_GLOBAL T *)p; }

// LDS address space, for arrays that a non-inlined function reads (so that it emits LDS, not
// flat, instructions)
#define GPR_LDS __attribute__((address_space(3)))

// vector loads/stores through native vector types (HIP's vector classes cannot be copied
// from an address-space-qualified reference)
typedef int gv_i2 __attribute__((ext_vector_type(2)));
typedef int gv_i4 __attribute__((ext_vector_type(4)));
typedef unsigned gv_u2 __attribute__((ext_vector_type(2)));
typedef float gv_f2 __attribute__((ext_vector_type(2)));
typedef float gv_f4 __attribute__((ext_vector_type(4)));
typedef float gv_f3 __attribute__((ext_vector_type(3)));   // 16-byte size and alignment, 12-byte loads
__device__ __forceinline__ int2 gld(const GPR_GLOBAL int2 *p) { const gv_i2 v = *(const GPR_GLOBAL gv_i2 *)p; return make_int2(v.x, v.y); }
__device__ __forceinline__ int4 gld(const GPR_GLOBAL int4 *p) { const gv_i4 v = *(const GPR_GLOBAL gv_i4 *)p; return make_int4(v.x, v.y, v.z, v.w); }
__device__ __forceinline__ uint2 gld(const GPR_GLOBAL uint2 *p) { const gv_u2 v = *(const GPR_GLOBAL gv_u2 *)p; return make_uint2(v.x, v.y); }
__device__ __forceinline__ float2 gld(const GPR_GLOBAL float2 *p) { const gv_f2 v = *(const GPR_GLOBAL gv_f2 *)p; return make_float2(v.x, v.y); }
__device__ __forceinline__ float4 gld(const GPR_GLOBAL float4 *p) { const gv_f4 v = *(const GPR_GLOBAL gv_f4 *)p; return make_float4(v.x, v.y, v.z, v.w); }
__device__ __forceinline__ void gst(GPR_GLOBAL uint2 *p, uint2 v) { gv_u2 w; w.x = v.x; w.y = v.y; *(GPR_GLOBAL gv_u2 *)p = w; }
__device__ __forceinline__ void gst(GPR_GLOBAL unsigned long long *p, unsigned long long v) { *p = v; }

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): ten rounds; each multiplies words 0 and 2 by fixed
// 32-bit constants, crosses the high halves with words 1 and 3 and the round key, and
// bumps the key by the Weyl increments between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        // one 32 x 32 -> 64-bit product per word (a single v_mad_u64_u32)
        const unsigned long long p0 = (unsigned long long)c.x * 0xD2511F53u;
        const unsigned long long p1 = (unsigned long long)c.z * 0xCD9E8D57u;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint4 philox_ctr(uint32_t atom, long long step, uint32_t replica, uint32_t stream,
                                            uint32_t k0, uint32_t k1)
{
    const unsigned long long us = (unsigned long long)step;
    return philox10(make_uint4(atom, (uint32_t)us, replica, (stream << 24) | ((uint32_t)(us >> 32) & 0xFFFFFFu)),
                    k0, k1);
}

// odd multiple of 2^-24 in (0, 1): exact in FP32
__device__ __forceinline__ float unit_open(uint32_t w)
{
    return (float)(2u * (w >> 9) + 1u) * 5.9604644775390625e-08f;
}

// Box-Muller: (z0, z1) from (u0, u1), z2 from (u2, u3), on the hardware transcendentals:
// v_log_f32 gives log2 (so -2 ln u = -2 ln 2 log2 u), v_sin_f32 / v_cos_f32 take their argument
// in revolutions (sin 2 pi u directly).  Over every uniform the generator produces their
// largest errors are 1.3e-7 (sin, cos, absolute) and 1.2e-7 (log2, relative).
__device__ __forceinline__ float3 gauss3(uint4 w)
{
    constexpr float M2LN2 = -1.3862943611198906f;          // -2 ln 2
    const float ra = __builtin_amdgcn_sqrtf(M2LN2 * __builtin_amdgcn_logf(unit_open(w.x)));
    const float rb = __builtin_amdgcn_sqrtf(M2LN2 * __builtin_amdgcn_logf(unit_open(w.z)));
    const float u1 = unit_open(w.y), u3 = unit_open(w.w);
    return make_float3(ra * __builtin_amdgcn_cosf(u1), ra * __builtin_amdgcn_sinf(u1), rb * __builtin_amdgcn_cosf(u3));
}

// ------------------------------------------------------------------ fixed point
// f 2^32 rounded to the nearest integer (ties to even) as a 64-bit integer.  In FP64 the sum
// f 2^32 + 1.5 2^52 lies in [2^52, 2^53), where the spacing is 1, so one rounding leaves the
// integer in the low bits of the mantissa: exact while |f| < 2^19.  Larger values (and NaN)
// saturate at +-FSAT, which the FMAX_FIX test on the summed force reports as unstable.
__device__ __forceinline__ long long fix_f(float f)
{
    const float c = fminf(fmaxf(f, -FSAT), FSAT);
    const double y = __builtin_fma((double)c, FIX, 6755399441055744.0);
    return __double_as_longlong(y) - 0x4338000000000000LL;
}
__device__ __forceinline__ long long fix_d(double d) { return __double2ll_rn(d * FIX); }
__device__ __forceinline__ float unfix_f(long long a) { return (float)((double)a * FIX_INV); }
__device__ __forceinline__ double unfix_d(long long a) { return (double)a * FIX_INV; }

__device__ __forceinline__ void lds_add(long long *p, long long v)
{
    atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

__device__ __forceinline__ bool bad_force(float f) { return !(fabsf(f) < FMAX_FIX); }

// ------------------------------------------------------------------ bonded terms (FP32)
// Each returns the energy and writes the force on every atom of the term.

// bond 1/2 k (r - r0)^2
// arctangent on [0, 1] as a P(a^2), P of degree 8 fitted by iteratively reweighted least
// squares to atan(a)/a (maximum error 6e-9 in exact arithmetic, 1e-7 evaluated in FP32)
__device__ __forceinline__ float atan01(float a)
{
    const float s = a * a;
    float p = 0.002454932313412428f;
    p = fmaf(p, s, -0.014395107515156269f);
    p = fmaf(p, s, 0.039772968739271164f);
    p = fmaf(p, s, -0.07234375923871994f);
    p = fmaf(p, s, 0.10498868674039841f);
    p = fmaf(p, s, -0.141612708568573f);
    p = fmaf(p, s, 0.19985927641391754f);
    p = fmaf(p, s, -0.3333260118961334f);
    p = fmaf(p, s, 0.9999998807907104f);
    return a * p;
}
// the angle atan2(y, x) in [0, pi] for y >= 0 (octant reduction to [0, 1])
__device__ __forceinline__ float atan2_upper(float y, float x)
{
    const float ax = fabsf(x);
    const float mx = fmaxf(y, ax), mn = fminf(y, ax);
    float t = mx > 0.f ? atan01(mn * __builtin_amdgcn_rcpf(mx)) : 0.f;
    if (y > ax) t = 1.5707963267948966f - t;
    if (x < 0.f) t = 3.141592653589793f - t;
    return t;
}

__device__ __forceinline__ float term_bond(float3 pi, float3 pj, float2 p, float3 &fi)
{
    const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float dr = r2 * ri - p.x;
    const float g = p.y * dr * ri;   // force on i along (pj - pi)
    fi = make_float3(g * dx, g * dy, g * dz);
    return 0.5f * p.y * dr * dr;
}
__device__ __forceinline__ float term_angle(float3 pi, float3 pj, float3 pk, float2 p, float3 &fi, float3 &fk)
{
    const float ux = pi.x - pj.x, uy = pi.y - pj.y, uz = pi.z - pj.z;
    const float wx = pk.x - pj.x, wy = pk.y - pj.y, wz = pk.z - pj.z;
    const float cx = uy * wz - uz * wy, cy = uz * wx - ux * wz, cz = ux * wy - uy * wx;
    const float sn = __builtin_amdgcn_sqrtf(cx * cx + cy * cy + cz * cz);
    const float cs = ux * wx + uy * wy + uz * wz;
    const float th = atan2_upper(sn, cs);
    const float dth = th - p.x;
    const float lu2 = ux * ux + uy * uy + uz * uz, lw2 = wx * wx + wy * wy + wz * wz;
    // d theta / d p_i = (cos(theta) u/|u|^2 - w/(|u||w|)) / sin(theta); sin(theta) |u||w| = sn
    const float g = -p.y * dth;
    const float a = g * __builtin_amdgcn_rcpf(sn);          // g / (|u||w| sin theta)
    const float cu = cs * __builtin_amdgcn_rcpf(lu2), cw = cs * __builtin_amdgcn_rcpf(lw2);
    fi = make_float3(a * (cu * ux - wx), a * (cu * uy - wy), a * (cu * uz - wz));
    fk = make_float3(a * (cw * wx - ux), a * (cw * wy - uy), a * (cw * wz - uz));
    return 0.5f * p.y * dth * dth;
}
// cos(n phi - phi0) for p = (k, cos phi0, sin phi0, n), by the same algebra as term_torsion
__device__ __forceinline__ float torsion_cos(float3 pi, float3 pj, float3 pk, float3 pl, float4 p)
{
    const float b1x = pj.x - pi.x, b1y = pj.y - pi.y, b1z = pj.z - pi.z;
    const float b2x = pk.x - pj.x, b2y = pk.y - pj.y, b2z = pk.z - pj.z;
    const float b3x = pl.x - pk.x, b3y = pl.y - pk.y, b3z = pl.z - pk.z;
    const float n1x = b1y * b2z - b1z * b2y, n1y = b1z * b2x - b1x * b2z, n1z = b1x * b2y - b1y * b2x;
    const float n2x = b2y * b3z - b2z * b3y, n2y = b2z * b3x - b2x * b3z, n2z = b2x * b3y - b2y * b3x;
    const float lb2sq = b2x * b2x + b2y * b2y + b2z * b2z;
    const float lb2 = lb2sq * __builtin_amdgcn_rsqf(lb2sq);
    const float xx = n1x * n2x + n1y * n2y + n1z * n2z;
    const float yy = lb2 * (b1x * n2x + b1y * n2y + b1z * n2z);
    const float ih = __builtin_amdgcn_rsqf(xx * xx + yy * yy);
    const float c = xx * ih, sn = yy * ih;
    float C = 1.0f, Sn = 0.0f;
    const int nm = (int)p.w;
    for (int m = 0; m < nm; ++m) {
        const float C2 = C * c - Sn * sn;
        Sn = C * sn + Sn * c;
        C = C2;
    }
    return C * p.y + Sn * p.z;
}

// k (1 + cos(n phi - phi0)) with p = (k, cos phi0, sin phi0, n): cos phi and sin phi come from the
// two projections that define the dihedral, cos n phi and sin n phi by repeated complex
// multiplication, so no inverse or direct trigonometric function is evaluated.
__device__ __forceinline__ float term_torsion(float3 pi, float3 pj, float3 pk, float3 pl, float4 p,
                                              float3 &fi, float3 &fj, float3 &fk, float3 &fl)
{
    const float b1x = pj.x - pi.x, b1y = pj.y - pi.y, b1z = pj.z - pi.z;
    const float b2x = pk.x - pj.x, b2y = pk.y - pj.y, b2z = pk.z - pj.z;
    const float b3x = pl.x - pk.x, b3y = pl.y - pk.y, b3z = pl.z - pk.z;
    const float n1x = b1y * b2z - b1z * b2y, n1y = b1z * b2x - b1x * b2z, n1z = b1x * b2y - b1y * b2x;
    const float n2x = b2y * b3z - b2z * b3y, n2y = b2z * b3x - b2x * b3z, n2z = b2x * b3y - b2y * b3x;
    const float lb2sq = b2x * b2x + b2y * b2y + b2z * b2z;
    const float ilb2 = __builtin_amdgcn_rsqf(lb2sq);
    const float lb2 = lb2sq * ilb2;
    const float xx = n1x * n2x + n1y * n2y + n1z * n2z;
    const float yy = lb2 * (b1x * n2x + b1y * n2y + b1z * n2z);
    const float ih = __builtin_amdgcn_rsqf(xx * xx + yy * yy);
    const float c = xx * ih, sn = yy * ih;                 // cos phi, sin phi
    float C = 1.0f, Sn = 0.0f;                            // cos n phi, sin n phi
    const int nm = (int)p.w;
    for (int m = 0; m < nm; ++m) {
        const float C2 = C * c - Sn * sn;
        Sn = C * sn + Sn * c;
        C = C2;
    }
    const float ca = C * p.y + Sn * p.z;                  // cos(n phi - phi0)
    const float sa = Sn * p.y - C * p.z;                  // sin(n phi - phi0)
    const float dUdphi = -p.x * p.w * sa;
    const float n1sq = n1x * n1x + n1y * n1y + n1z * n1z;
    const float n2sq = n2x * n2x + n2y * n2y + n2z * n2z;
    const float ai = dUdphi * lb2 * __builtin_amdgcn_rcpf(n1sq);    // F_i = +dU/dphi |b2|/|n1|^2 n1
    const float al = -dUdphi * lb2 * __builtin_amdgcn_rcpf(n2sq);   // F_l = -dU/dphi |b2|/|n2|^2 n2
    fi = make_float3(ai * n1x, ai * n1y, ai * n1z);
    fl = make_float3(al * n2x, al * n2y, al * n2z);
    const float ilb2sq = ilb2 * ilb2;
    const float p12 = (b1x * b2x + b1y * b2y + b1z * b2z) * ilb2sq;
    const float p32 = (b3x * b2x + b3y * b2y + b3z * b2z) * ilb2sq;
    // F_j = -(1 + p12) F_i + p32 F_l ; F_k = p12 F_i - (1 + p32) F_l
    const float aj = -(1.0f + p12), ak = -(1.0f + p32);
    fj = make_float3(aj * fi.x + p32 * fl.x, aj * fi.y + p32 * fl.y, aj * fi.z + p32 * fl.z);
    fk = make_float3(p12 * fi.x + ak * fl.x, p12 * fi.y + ak * fl.y, p12 * fi.z + ak * fl.z);
    return p.x * (1.0f + ca);
}
__device__ __forceinline__ float term_pair14(float3 pi, float3 pj, float4 p, float3 &fi)
{
    const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r2i = ri * ri;
    const float s2 = p.x * p.x * r2i;
    const float s6 = s2 * s2 * s2;
    const float u = p.y * (s6 * s6 - s6) + p.z * ri;
    const float fs = p.y * r2i * (12.0f * s6 * s6 - 6.0f * s6) + p.z * ri * r2i;
    fi = make_float3(fs * dx, fs * dy, fs * dz);
    return u;
}

// ------------------------------------------------------------------ FP64 geometry for states and observables
__device__ __forceinline__ double dihedral_d(double3 a, double3 b, double3 c, double3 d)
{
    const double b1x = b.x - a.x, b1y = b.y - a.y, b1z = b.z - a.z;
    const double b2x = c.x - b.x, b2y = c.y - b.y, b2z = c.z - b.z;
    const double b3x = d.x - c.x, b3y = d.y - c.y, b3z = d.z - c.z;
    const double n1x = b1y * b2z - b1z * b2y, n1y = b1z * b2x - b1x * b2z, n1z = b1x * b2y - b1y * b2x;
    const double n2x = b2y * b3z - b2z * b3y, n2y = b2z * b3x - b2x * b3z, n2z = b2x * b3y - b2y * b3x;
    const double lb2 = sqrt(b2x * b2x + b2y * b2y + b2z * b2z);
    const double xx = n1x * n2x + n1y * n2y + n1z * n2z;
    const double yy = lb2 * (b1x * n2x + b1y * n2y + b1z * n2z);
    return atan2(yy, xx);
}

} // namespace gpr
