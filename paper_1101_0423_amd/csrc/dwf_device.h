// dwf_device.h -- device-side building blocks of the gfx950 domain-wall
// stencil: field accessors for the structure-of-arrays spinor layout, gauge
// link formats with LDS staging, the spin-projected Wilson hop (Eq. (14)),
// the dense per-4D-site fifth-dimension matrix (M5 of Eq. (8) and friends)
// and the fused kernel template that strings them together with a
// prologue/epilogue and a deterministic block reduction.
//
// Device layouts (one parity of the 4D checkerboard per "half field"):
//   half 4D index  h4 = (x + Lx (y + Ly (z + Lz t))) / 2     (Lx even)
//   half 5D index  i5 = s + Ns * h4                          (s fastest)
//   FP64 spinor : double2 [h4][12][Ns]   block j = complex component j
//   FP32 spinor : float4  [h4][6][Ns]    block j = complex components 2j, 2j+1
//   FP16 spinor : 8 x binary16 [h4][3][Ns] + float norm[i5]
//                 (value = half * norm, norm = max |component| of the site)
//   complex component k = 3 * spin + colour; spins 0,1 are the + chirality
//   (gamma_5 = diag(1,1,-1,-1) in the chiral basis).
//   Gauge links, per output parity: [h4][8][n] with entries 0..3 the forward
//   links U_mu(x) and 4..7 the backward links U_mu(x - mu)^dag, each a
//   row-major 3x3 complex matrix (n = 18) or its first two rows (n = 12).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace dwf {

// ---------------------------------------------------------------------------
// spinor fields
// ---------------------------------------------------------------------------

// Every accessor addresses 5D half site i5 = s + Ns * h4 of right-hand side
// rhs.  Layout per 4D site h4: [component block j][s][16 bytes], i.e. the
// element of (i5, s, block j) is NB * i5 - (NB - 1) * s + j * Ns: the Ns
// slices of one block are adjacent (one wave reads whole 256-byte runs) and
// all of a 4D site's data is one contiguous chunk.

// Every field type has Ptrs, the pointers of one field, and with(q), a field of
// the same layout (Ns, right-hand-side strides) at q: a kernel that touches
// several fields of one layout passes one full field and the others' Ptrs,
// which keeps its arguments within the scalar registers.

struct FD {  // FP64 storage and arithmetic
    using real = double;
    double2* p;
    long ns;       // Ns (elements between component blocks of a site)
    long rstride;  // elements between right-hand sides
    struct Ptrs {
        double2* p;
    };
    __host__ __device__ Ptrs ptrs() const { return Ptrs{p}; }
    __host__ __device__ FD with(Ptrs q) const {
        FD f = *this;
        f.p = q.p;
        return f;
    }
    __device__ __forceinline__ const double2* at(int rhs, long i, int s) const {
        return p + rhs * rstride + 12 * i - 11 * (long)s;
    }
    template <class R>
    __device__ __forceinline__ void sload(int rhs, long i, int s, R* v) const {
        load(rhs, i, s, v);
    }
    template <class R>
    __device__ __forceinline__ void sstore(int rhs, long i, int s, const R* v) const {
        store(rhs, i, s, v);
    }
    template <class R>
    __device__ __forceinline__ void gather(int rhs, long i, int s, R* v) const {
        load(rhs, i, s, v);
    }
    // two-stage gather: fetch issues the loads, unpack consumes them, so that
    // a hop can keep the next neighbour's loads in flight meanwhile
    struct Raw { double v[24]; };
    __device__ __forceinline__ void fetch(int rhs, long i, int s, Raw& r) const { load(rhs, i, s, r.v); }
    template <class R>
    __device__ __forceinline__ void unpack(const Raw& r, R* v) const {
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = (R)r.v[k];
    }
    __device__ __forceinline__ void load(int rhs, long i, int s, double* v) const {
        const double2* q = at(rhs, i, s);
#pragma unroll
        for (int j = 0; j < 12; ++j) {
            double2 a = q[j * ns];
            v[2 * j] = a.x;
            v[2 * j + 1] = a.y;
        }
    }
    __device__ __forceinline__ void store(int rhs, long i, int s, const double* v) const {
        double2* q = const_cast<double2*>(at(rhs, i, s));
#pragma unroll
        for (int j = 0; j < 12; ++j) q[j * ns] = make_double2(v[2 * j], v[2 * j + 1]);
    }
    __device__ __forceinline__ void load(int rhs, long i, int s, float* v) const {
        double t[24];
        load(rhs, i, s, t);
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = (float)t[k];
    }
    __device__ __forceinline__ void store(int rhs, long i, int s, const float* v) const {
        double t[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) t[k] = v[k];
        store(rhs, i, s, t);
    }
};

struct FS {  // FP32 storage
    using real = float;
    float4* p;
    long ns;
    long rstride;
    struct Ptrs {
        float4* p;
    };
    __host__ __device__ Ptrs ptrs() const { return Ptrs{p}; }
    __host__ __device__ FS with(Ptrs q) const {
        FS f = *this;
        f.p = q.p;
        return f;
    }
    __device__ __forceinline__ const float4* at(int rhs, long i, int s) const {
        return p + rhs * rstride + 6 * i - 5 * (long)s;
    }
    // cached loads and stores (hop neighbours, data the next kernel gathers)
    __device__ __forceinline__ void load(int rhs, long i, int s, float* v) const {
        const float4* q = at(rhs, i, s);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            float4 a = q[j * ns];
            v[4 * j] = a.x;
            v[4 * j + 1] = a.y;
            v[4 * j + 2] = a.z;
            v[4 * j + 3] = a.w;
        }
    }
    __device__ __forceinline__ void gather(int rhs, long i, int s, float* v) const { load(rhs, i, s, v); }
    struct Raw { float v[24]; };
    __device__ __forceinline__ void fetch(int rhs, long i, int s, Raw& r) const { load(rhs, i, s, r.v); }
    __device__ __forceinline__ void unpack(const Raw& r, float* v) const {
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = r.v[k];
    }
    __device__ __forceinline__ void store(int rhs, long i, int s, const float* v) const {
        float4* q = const_cast<float4*>(at(rhs, i, s));
#pragma unroll
        for (int j = 0; j < 6; ++j) q[j * ns] = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
    }
    // streaming (non-temporal) loads and stores: vectors a kernel reads or
    // writes once, kept from displacing the neighbour data the hop re-reads
    __device__ __forceinline__ void sload(int rhs, long i, int s, float* v) const {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4* q = (const f4*)at(rhs, i, s);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            f4 a = __builtin_nontemporal_load(q + j * ns);
            v[4 * j] = a.x;
            v[4 * j + 1] = a.y;
            v[4 * j + 2] = a.z;
            v[4 * j + 3] = a.w;
        }
    }
    __device__ __forceinline__ void sstore(int rhs, long i, int s, const float* v) const {
        typedef float f4 __attribute__((ext_vector_type(4)));
        f4* q = (f4*)const_cast<float4*>(at(rhs, i, s));
#pragma unroll
        for (int j = 0; j < 6; ++j)
            __builtin_nontemporal_store(f4{v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]}, q + j * ns);
    }
    __device__ __forceinline__ void load(int rhs, long i, int s, double* v) const {
        float t[24];
        load(rhs, i, s, t);
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = t[k];
    }
    __device__ __forceinline__ void store(int rhs, long i, int s, const double* v) const {
        float t[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) t[k] = (float)v[k];
        store(rhs, i, s, t);
    }
};

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

struct FH {  // binary16 storage with one FP32 scale per 5D site; FP32 arithmetic
    using real = float;
    uint4* p;
    float* nrm;     // [i5]
    long ns;
    long rstride;   // data elements between right-hand sides
    long nrstride;  // norm elements between right-hand sides
    struct Ptrs {
        uint4* p;
        float* nrm;
    };
    __host__ __device__ Ptrs ptrs() const { return Ptrs{p, nrm}; }
    __host__ __device__ FH with(Ptrs q) const {
        FH f = *this;
        f.p = q.p;
        f.nrm = q.nrm;
        return f;
    }
    __device__ __forceinline__ const uint4* at(int rhs, long i, int s) const {
        return p + rhs * rstride + 3 * i - 2 * (long)s;
    }
    template <class R>
    __device__ __forceinline__ void gather(int rhs, long i, int s, R* v) const {
        load(rhs, i, s, v);
    }
    // two-stage gather: the raw 16-byte vectors and the scale, converted in unpack
    typedef unsigned int u4v __attribute__((ext_vector_type(4)));
    struct Raw {
        u4v a[3];
        float n;
    };
    __device__ __forceinline__ void fetch(int rhs, long i, int s, Raw& r) const {
        const u4v* q = (const u4v*)at(rhs, i, s);
        r.n = nrm[rhs * nrstride + i];
#pragma unroll
        for (int j = 0; j < 3; ++j) r.a[j] = q[j * ns];
    }
    __device__ __forceinline__ void unpack(const Raw& r, float* v) const {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            half8_t h = __builtin_bit_cast(half8_t, r.a[j]);
#pragma unroll
            for (int k = 0; k < 8; ++k) v[8 * j + k] = (float)h[k] * r.n;
        }
    }
    // NT: non-temporal (streaming) access, as for FS
    template <bool NT = false>
    __device__ __forceinline__ void load(int rhs, long i, int s, float* v) const {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        const u4* q = (const u4*)at(rhs, i, s);
        const float* np = nrm + rhs * nrstride + i;
        const float n = NT ? __builtin_nontemporal_load(np) : *np;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const u4 a = NT ? __builtin_nontemporal_load(q + j * ns) : q[j * ns];
            half8_t h = __builtin_bit_cast(half8_t, a);
#pragma unroll
            for (int k = 0; k < 8; ++k) v[8 * j + k] = (float)h[k] * n;
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ void store(int rhs, long i, int s, const float* v) const {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf(v[k]));
        float inv = m > 0.f ? 1.f / m : 0.f;
        u4* q = (u4*)const_cast<uint4*>(at(rhs, i, s));
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            half8_t h;
#pragma unroll
            for (int k = 0; k < 8; ++k) h[k] = (_Float16)(v[8 * j + k] * inv);
            if (NT)
                __builtin_nontemporal_store(__builtin_bit_cast(u4, h), q + j * ns);
            else
                q[j * ns] = __builtin_bit_cast(u4, h);
        }
        if (NT)
            __builtin_nontemporal_store(m, nrm + rhs * nrstride + i);
        else
            nrm[rhs * nrstride + i] = m;
    }
    __device__ __forceinline__ void sload(int rhs, long i, int s, float* v) const { load<true>(rhs, i, s, v); }
    __device__ __forceinline__ void sstore(int rhs, long i, int s, const float* v) const {
        store<true>(rhs, i, s, v);
    }
    __device__ __forceinline__ void sload(int rhs, long i, int s, double* v) const { load(rhs, i, s, v); }
    __device__ __forceinline__ void sstore(int rhs, long i, int s, const double* v) const { store(rhs, i, s, v); }
    __device__ __forceinline__ void load(int rhs, long i, int s, double* v) const {
        float t[24];
        load(rhs, i, s, t);
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = t[k];
    }
    __device__ __forceinline__ void store(int rhs, long i, int s, const double* v) const {
        float t[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) t[k] = (float)v[k];
        store(rhs, i, s, t);
    }
};

// ---------------------------------------------------------------------------
// gauge links: LDS staging of the 8 links of every site of a workgroup
// ---------------------------------------------------------------------------

template <class Real>
struct LdsLink {
    static constexpr int STR = sizeof(Real) == 4 ? 20 : 18;  // 16-byte aligned rows
    // per-site stride: 8 links plus 16 bytes, so that the sites read together
    // by one wave start on different LDS banks
    static constexpr int SITE = 8 * STR + (sizeof(Real) == 4 ? 4 : 2);
    static __device__ __forceinline__ int at(int l) { return (l >> 3) * SITE + (l & 7) * STR; }
};

template <class Real>
__device__ __forceinline__ void su3_third_row(Real* u) {
    // row2 = conj(row0 x row1)
#define RE(a, b) u[2 * (3 * (a) + (b))]
#define IM(a, b) u[2 * (3 * (a) + (b)) + 1]
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
        Real cr = RE(0, b1) * RE(1, b2) - IM(0, b1) * IM(1, b2) - (RE(0, b2) * RE(1, b1) - IM(0, b2) * IM(1, b1));
        Real ci = RE(0, b1) * IM(1, b2) + IM(0, b1) * RE(1, b2) - (RE(0, b2) * IM(1, b1) + IM(0, b2) * RE(1, b1));
        RE(2, b) = cr;
        IM(2, b) = -ci;
    }
#undef RE
#undef IM
}

// stage(lds, site0, nsites, tid, T, sc): the 8 links of nsites sites, link l
// (= 8 * site + entry) multiplied by sc(l), as row-major 3x3 in LDS.
// 18-real links: a site's 8 links are 8 x 18 contiguous reals (a multiple of
// 16 bytes), read as 16-byte vectors, DWF_STAGE_BATCH per thread in flight
// before any is written to LDS.
constexpr int DWF_STAGE_BATCH = 4;

template <class Real, class V, int PER, class Sc>
__device__ __forceinline__ void stage18(const V* __restrict__ src, Real* lds, int nsites, int tid, int T,
                                        const Sc& sc) {
    const int nv = nsites * 8 * 18 / PER;  // vectors of PER reals
    for (int base = tid; base < nv; base += DWF_STAGE_BATCH * T) {
        V q[DWF_STAGE_BATCH];
#pragma unroll
        for (int k = 0; k < DWF_STAGE_BATCH; ++k)
            if (base + k * T < nv) q[k] = src[base + k * T];
#pragma unroll
        for (int k = 0; k < DWF_STAGE_BATCH; ++k) {
            const int i = base + k * T;
            if (i >= nv) break;
            const Real* qv = (const Real*)&q[k];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int e = i * PER + j, l = e / 18, c = e - 18 * l;
                lds[LdsLink<Real>::at(l) + c] = sc(l) * qv[j];
            }
        }
    }
}

struct LinkD18 {
    using real = double;
    const double* p;  // [h4][8][18]
    template <class Sc>
    __device__ __forceinline__ void stage(double* lds, long site0, int nsites, int tid, int T, const Sc& sc) const {
        stage18<double, double2, 2>((const double2*)(p + site0 * 8 * 18), lds, nsites, tid, T, sc);
    }
};

struct LinkS18 {
    using real = float;
    const float* p;  // [h4][8][18]
    template <class Sc>
    __device__ __forceinline__ void stage(float* lds, long site0, int nsites, int tid, int T, const Sc& sc) const {
        stage18<float, float4, 4>((const float4*)(p + site0 * 8 * 18), lds, nsites, tid, T, sc);
    }
};

struct LinkS12 {
    using real = float;
    const float* p;  // [h4][8][12]
    template <class Sc>
    __device__ __forceinline__ void stage(float* lds, long site0, int nsites, int tid, int T, const Sc& sc) const {
        const float4* src = (const float4*)(p + site0 * 8 * 12);
        int nl = nsites * 8;
        for (int l = tid; l < nl; l += T) {
            float u[18];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                float4 q = src[3 * l + j];
                u[4 * j] = q.x; u[4 * j + 1] = q.y; u[4 * j + 2] = q.z; u[4 * j + 3] = q.w;
            }
            su3_third_row(u);
            const float f = sc(l);
#pragma unroll
            for (int k = 0; k < 18; ++k) lds[LdsLink<float>::at(l) + k] = f * u[k];
        }
    }
};

struct LinkH12 {
    using real = float;
    const _Float16* p;  // [h4][8][12]
    template <class Sc>
    __device__ __forceinline__ void stage(float* lds, long site0, int nsites, int tid, int T, const Sc& sc) const {
        const uint2* src = (const uint2*)(p + site0 * 8 * 12);
        int nl = nsites * 8;
        typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
        for (int l = tid; l < nl; l += T) {
            float u[18];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                half4_t h = __builtin_bit_cast(half4_t, src[3 * l + j]);
#pragma unroll
                for (int k = 0; k < 4; ++k) u[4 * j + k] = (float)h[k];
            }
            su3_third_row(u);
            const float f = sc(l);
#pragma unroll
            for (int k = 0; k < 18; ++k) lds[LdsLink<float>::at(l) + k] = f * u[k];
        }
    }
};

struct LinkNone {
    using real = double;
};

// ---------------------------------------------------------------------------
// geometry and workgroup mapping
// ---------------------------------------------------------------------------

struct Geom {
    int Lx, Ly, Lz, Lt;
    int Lxh;       // Lx / 2
    int Ns;
    int G;         // 4D sites per workgroup
    int V4h;       // 4D sites per parity
    int out_parity;
    int antiper;   // 1: links crossing the t boundary carry a factor -1
    int nblocks;
    int xcd;       // 1: map consecutive lattice blocks onto one XCD
    int nsb;       // > 0: workgroups go t-fastest: blocks per t-slice (V3h / G) ...
    int tchunk;    // ... in chunks of tchunk t-slices (one chunk per XCD)
    int nsb0;      // blocks per z-plane of a t-slice (whole planes only)
    int tilew;     // > 0: z-plane blocks walked in tiles of tilew (block_of)
};

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  Map dispatch id -> lattice block so that every XCD
// walks one contiguous slab of the lattice (neighbour re-reads then hit the
// same L2).  A bijection on [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nb, int on) {
    if (!on) return b;
    const int NX = 8;
    int q = nb / NX, r = nb - q * NX;
    int x = b % NX, idx = b / NX;
    return x < r ? x * (q + 1) + idx : r * (q + 1) + (x - r) * q + idx;
}

// Lattice block of a workgroup's position L in the (XCD-remapped) order.  With
// g.nsb > 0 the order runs t-fastest through every chunk of tchunk t-slices:
// L = (chunk, spatial block, t in chunk), so the +-t neighbours of a block
// were read one workgroup earlier and the +-z ones nsb0 * tchunk workgroups
// earlier, both still in the XCD's L2.  Where that distance is large (big
// z-planes) the blocks of a z-plane are cut into tiles of tilew and the order
// is L = (chunk, tile, z, t in chunk, block in tile): +-y neighbours sit in
// the same or the previous workgroup, +-t tilew and +-z tilew * tchunk back.
// A bijection on [0, nblocks).
__device__ __forceinline__ int block_of(int L, const Geom& g) {
    if (g.nsb <= 0) return L;
    const int per = g.nsb * g.tchunk;
    const int chunk = L / per, rem = L - chunk * per;
    if (g.tilew > 0) {
        const int i = rem % g.tilew, r2 = rem / g.tilew;
        const int tt = r2 % g.tchunk, r3 = r2 / g.tchunk;
        const int z = r3 % g.Lz, j = r3 / g.Lz;
        return (chunk * g.tchunk + tt) * g.nsb + z * g.nsb0 + j * g.tilew + i;
    }
    const int sb = rem / g.tchunk, tt = rem - sb * g.tchunk;
    return (chunk * g.tchunk + tt) * g.nsb + sb;
}

// ---------------------------------------------------------------------------
// Wilson hop along one direction, spin projected (Eq. (14)):
//   acc += (1 + SIG gamma_MU) U psi,  SIG = -1 forward, +1 backward.
// In the chiral basis (1 + SIG gamma_MU) psi is fixed by two spin components
// h0, h1; U multiplies only those and the lower two are rebuilt from U h.
// ---------------------------------------------------------------------------

// Spin projection: the two components h0, h1 that fix (1 + SIG gamma_MU) psi.
template <int MU, int SIG, class Real>
__device__ __forceinline__ void hop_proj(const Real* __restrict__ psi, Real* __restrict__ h0,
                                         Real* __restrict__ h1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const Real p0r = psi[2 * a], p0i = psi[2 * a + 1];
        const Real p1r = psi[2 * (3 + a)], p1i = psi[2 * (3 + a) + 1];
        const Real p2r = psi[2 * (6 + a)], p2i = psi[2 * (6 + a) + 1];
        const Real p3r = psi[2 * (9 + a)], p3i = psi[2 * (9 + a) + 1];
        if (MU == 0) {  // h0 = p0 - SIG i p3, h1 = p1 - SIG i p2
            h0[2 * a] = p0r + SIG * p3i; h0[2 * a + 1] = p0i - SIG * p3r;
            h1[2 * a] = p1r + SIG * p2i; h1[2 * a + 1] = p1i - SIG * p2r;
        } else if (MU == 1) {  // h0 = p0 - SIG p3, h1 = p1 + SIG p2
            h0[2 * a] = p0r - SIG * p3r; h0[2 * a + 1] = p0i - SIG * p3i;
            h1[2 * a] = p1r + SIG * p2r; h1[2 * a + 1] = p1i + SIG * p2i;
        } else if (MU == 2) {  // h0 = p0 - SIG i p2, h1 = p1 + SIG i p3
            h0[2 * a] = p0r + SIG * p2i; h0[2 * a + 1] = p0i - SIG * p2r;
            h1[2 * a] = p1r - SIG * p3i; h1[2 * a + 1] = p1i + SIG * p3r;
        } else {  // h0 = p0 + SIG p2, h1 = p1 + SIG p3
            h0[2 * a] = p0r + SIG * p2r; h0[2 * a + 1] = p0i + SIG * p2i;
            h1[2 * a] = p1r + SIG * p3r; h1[2 * a + 1] = p1i + SIG * p3i;
        }
    }
}

// acc += (1 + SIG gamma_MU) U psi from the projected h0, h1: colour multiply
// of the two components, then the lower two rebuilt from them.  CHAIN: each
// real part is one chain of fused multiply-adds seeded by its first product
// (no "+ 0", which IEEE signed zeros keep the compiler from removing), and
// FIRST sets acc instead of adding to it; otherwise the products are summed
// per complex term into accumulators that start at zero.
template <int MU, int SIG, bool FIRST, bool CHAIN, class Real>
__device__ __forceinline__ void hop_mul(const Real* __restrict__ h0, const Real* __restrict__ h1,
                                        const Real* __restrict__ U, Real* __restrict__ acc) {
    Real u0[6], u1[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const Real* Ua = U + 6 * a;
        Real r0, i0, r1, i1;
        if constexpr (CHAIN) {
            r0 = Ua[0] * h0[0]; i0 = Ua[0] * h0[1]; r1 = Ua[0] * h1[0]; i1 = Ua[0] * h1[1];
            r0 = fma(-Ua[1], h0[1], r0);
            i0 = fma(Ua[1], h0[0], i0);
            r1 = fma(-Ua[1], h1[1], r1);
            i1 = fma(Ua[1], h1[0], i1);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                const Real ur = Ua[2 * b], ui = Ua[2 * b + 1];
                r0 = fma(ur, h0[2 * b], r0);
                r0 = fma(-ui, h0[2 * b + 1], r0);
                i0 = fma(ur, h0[2 * b + 1], i0);
                i0 = fma(ui, h0[2 * b], i0);
                r1 = fma(ur, h1[2 * b], r1);
                r1 = fma(-ui, h1[2 * b + 1], r1);
                i1 = fma(ur, h1[2 * b + 1], i1);
                i1 = fma(ui, h1[2 * b], i1);
            }
        } else {
            r0 = 0; i0 = 0; r1 = 0; i1 = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const Real ur = Ua[2 * b], ui = Ua[2 * b + 1];
                r0 += ur * h0[2 * b] - ui * h0[2 * b + 1];
                i0 += ur * h0[2 * b + 1] + ui * h0[2 * b];
                r1 += ur * h1[2 * b] - ui * h1[2 * b + 1];
                i1 += ur * h1[2 * b + 1] + ui * h1[2 * b];
            }
        }
        u0[2 * a] = r0; u0[2 * a + 1] = i0;
        u1[2 * a] = r1; u1[2 * a + 1] = i1;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const Real r0 = u0[2 * a], i0 = u0[2 * a + 1], r1 = u1[2 * a], i1 = u1[2 * a + 1];
        Real c2r, c2i, c3r, c3i;
        if (MU == 0) {  // c2 = SIG i u1, c3 = SIG i u0
            c2r = -SIG * i1; c2i = SIG * r1; c3r = -SIG * i0; c3i = SIG * r0;
        } else if (MU == 1) {  // c2 = SIG u1, c3 = -SIG u0
            c2r = SIG * r1; c2i = SIG * i1; c3r = -SIG * r0; c3i = -SIG * i0;
        } else if (MU == 2) {  // c2 = SIG i u0, c3 = -SIG i u1
            c2r = -SIG * i0; c2i = SIG * r0; c3r = SIG * i1; c3i = -SIG * r1;
        } else {  // c2 = SIG u0, c3 = SIG u1
            c2r = SIG * r0; c2i = SIG * i0; c3r = SIG * r1; c3i = SIG * i1;
        }
        if (FIRST) {  // the first direction sets the accumulator
            acc[2 * a] = r0; acc[2 * a + 1] = i0;
            acc[2 * (3 + a)] = r1; acc[2 * (3 + a) + 1] = i1;
            acc[2 * (6 + a)] = c2r; acc[2 * (6 + a) + 1] = c2i;
            acc[2 * (9 + a)] = c3r; acc[2 * (9 + a) + 1] = c3i;
        } else {
            acc[2 * a] += r0; acc[2 * a + 1] += i0;
            acc[2 * (3 + a)] += r1; acc[2 * (3 + a) + 1] += i1;
            acc[2 * (6 + a)] += c2r; acc[2 * (6 + a) + 1] += c2i;
            acc[2 * (9 + a)] += c3r; acc[2 * (9 + a) + 1] += c3i;
        }
    }
}

// Neighbour half indices of 4D half site h4 (of parity par):
// nb[0..3] = x + mu, nb[4..7] = x - mu; tpos = 1 at t = Lt-1, 2 at t = 0.
__device__ __forceinline__ void neighbours(const Geom& g, int h4, int par, int* nb, int& tfw, int& tbw) {
    int xh = h4 % g.Lxh;
    int r = h4 / g.Lxh;
    int y = r % g.Ly;
    r /= g.Ly;
    int z = r % g.Lz;
    int t = r / g.Lz;
    int x = 2 * xh + ((y + z + t + par) & 1);
    int xp = x + 1 == g.Lx ? 0 : x + 1, xm = x == 0 ? g.Lx - 1 : x - 1;
    int yp = y + 1 == g.Ly ? 0 : y + 1, ym = y == 0 ? g.Ly - 1 : y - 1;
    int zp = z + 1 == g.Lz ? 0 : z + 1, zm = z == 0 ? g.Lz - 1 : z - 1;
    int tp = t + 1 == g.Lt ? 0 : t + 1, tm = t == 0 ? g.Lt - 1 : t - 1;
    int row = y + g.Ly * (z + g.Lz * t);
    nb[0] = (xp >> 1) + g.Lxh * row;
    nb[4] = (xm >> 1) + g.Lxh * row;
    nb[1] = xh + g.Lxh * (yp + g.Ly * (z + g.Lz * t));
    nb[5] = xh + g.Lxh * (ym + g.Ly * (z + g.Lz * t));
    nb[2] = xh + g.Lxh * (y + g.Ly * (zp + g.Lz * t));
    nb[6] = xh + g.Lxh * (y + g.Ly * (zm + g.Lz * t));
    nb[3] = xh + g.Lxh * (y + g.Ly * (z + g.Lz * tp));
    nb[7] = xh + g.Lxh * (y + g.Ly * (z + g.Lz * tm));
    tfw = (t == g.Lt - 1);
    tbw = (t == 0);
}

// The 8 directions of Eq. (14) for one (site, s) lane.  The staged links
// already carry the factor -1/2 (and the sign of links that cross an
// antiperiodic time boundary).  PIPE: software pipelined; once a direction's
// input is projected, its registers take the next neighbour's loads, which
// are in flight while the colour multiply of this direction runs (the
// scheduling barriers keep the compiler from moving them across), and the
// multiply uses fused chains (hop_mul CHAIN).  Otherwise each direction loads,
// waits and multiplies in turn.
template <class Real, bool PIPE, class F>
__device__ __forceinline__ void hop_site(const F& in, int rhs, int s, int Ns, const int* nb,
                                         const Real* __restrict__ lk, Real* acc) {
    constexpr int LS = LdsLink<Real>::STR;
    if (!PIPE)
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = 0;
    typename F::Raw raw;
    if (PIPE) in.fetch(rhs, (long)nb[0] * Ns + s, s, raw);
#define DWF_STEP(MU, SIG, L, NEXT)                                               \
    {                                                                            \
        if (!PIPE) in.fetch(rhs, (long)nb[L] * Ns + s, s, raw);                  \
        Real h0[6], h1[6];                                                       \
        {                                                                        \
            Real pa[24];                                                         \
            in.unpack(raw, pa);                                                  \
            hop_proj<MU, SIG>(pa, h0, h1);                                       \
        }                                                                        \
        if (PIPE) {                                                              \
            __builtin_amdgcn_sched_barrier(0);                                   \
            if ((NEXT) >= 0) in.fetch(rhs, (long)nb[(NEXT) & 7] * Ns + s, s, raw); \
            __builtin_amdgcn_sched_barrier(0);                                   \
        }                                                                        \
        Real U[18];                                                              \
        _Pragma("unroll") for (int k = 0; k < 18; ++k) U[k] = lk[(L) * LS + k];  \
        hop_mul<MU, SIG, (L) == 0 && PIPE, PIPE>(h0, h1, U, acc);                 \
    }
    DWF_STEP(0, -1, 0, 4)
    DWF_STEP(0, +1, 4, 1)
    DWF_STEP(1, -1, 1, 5)
    DWF_STEP(1, +1, 5, 2)
    DWF_STEP(2, -1, 2, 6)
    DWF_STEP(2, +1, 6, 3)
    DWF_STEP(3, -1, 3, 7)
    DWF_STEP(3, +1, 7, -1)
#undef DWF_STEP
}

// ---------------------------------------------------------------------------
// block reduction (deterministic: fixed shuffle tree, fixed wave order)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
    int tid = threadIdx.x, w = tid >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    if ((tid & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0;
    if (tid == 0)
        for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// fifth-dimension matrix on one column (one 4D site, one real spinor
// component, all Ns slices), values h[] at base[t * 24] in LDS.
//   MIX_DENSE: out_s = sum_t T[s][t] h_t (any Ns x Ns table)
//   MIX_SA / MIX_AS: M5 / M5^T (and M5^T gamma_5) through their O(Ns)
//   recurrences, coefficient arrays F, G, B, P, Q, O of the chirality block
//   (built on the host, see fifth_dim.h), s reversed where the shift runs
//   backwards.  All coefficients are wave-uniform (scalar loads).
// ---------------------------------------------------------------------------

enum MixMode { MIX_NONE = 0, MIX_DENSE = 1, MIX_SA = 2, MIX_AS = 3 };

template <class Real, int NSMAX>
__device__ __forceinline__ void mix_dense(Real* base, const Real* __restrict__ M, int Ns) {
    Real h[NSMAX];
#pragma unroll
    for (int t = 0; t < NSMAX; ++t)
        if (t < Ns) h[t] = base[t * 24];
#pragma unroll
    for (int ss = 0; ss < NSMAX; ++ss) {
        if (ss < Ns) {
            Real acc = 0;
#pragma unroll
            for (int t = 0; t < NSMAX; ++t)
                if (t < Ns) acc += M[ss * Ns + t] * h[t];
            base[ss * 24] = acc;
        }
    }
}

template <class Real, int NSMAX, int MODE>
__device__ __forceinline__ void mix_structured(Real* base, const Real* __restrict__ C, int N, bool rev) {
    // column in recurrence order
    Real h[NSMAX];
#pragma unroll
    for (int k = 0; k < NSMAX; ++k)
        if (k < N) h[k] = base[(rev ? N - 1 - k : k) * 24];
    const Real* F = C;
    const Real* G = C + N;
    const Real* B = C + 2 * N;
    const Real* P = C + 3 * N;
    const Real* Q = C + 4 * N;
    const Real* O = C + 5 * N;
    Real o[NSMAX];
    if constexpr (MODE == MIX_SA) {
        // w = X^-1 sqrt(w) h : alpha sweep, corner equation for w_0
        Real al[NSMAX];
        al[0] = 0;
        Real last = 0;
#pragma unroll
        for (int k = 1; k < NSMAX; ++k)
            if (k < N) {
                al[k] = F[k] * h[k] - G[k] * al[k - 1];
                last = al[k];
            }
        const Real w0 = F[0] * h[0] + G[0] * last;
        Real w[NSMAX];
        w[0] = w0;
        Real wl = w0;
#pragma unroll
        for (int k = 1; k < NSMAX; ++k)
            if (k < N) {
                w[k] = al[k] + B[k] * w0;
                wl = w[k];
            }
        // out = sqrt(w)^-1 Y w
        o[0] = P[0] * w0 + Q[0] * wl;
#pragma unroll
        for (int k = 1; k < NSMAX; ++k)
            if (k < N) o[k] = P[k] * w[k] + Q[k] * w[k - 1];
    } else {
        // g = Y^T sqrt(w)^-1 h
        Real hl = 0;
#pragma unroll
        for (int k = 0; k < NSMAX; ++k)
            if (k == N - 1) hl = h[k];
        Real gg[NSMAX];
        gg[0] = P[0] * h[0] + Q[0] * hl;
#pragma unroll
        for (int k = 1; k < NSMAX; ++k)
            if (k < N) gg[k] = P[k] * h[k] + Q[k] * h[k - 1];
        // w = X^-T g, out = sqrt(w) w
        Real al[NSMAX];
        al[0] = 0;
        Real last = 0;
#pragma unroll
        for (int k = 1; k < NSMAX; ++k)
            if (k < N) {
                al[k] = F[k] * gg[k] - G[k] * al[k - 1];
                last = al[k];
            }
        const Real w0 = F[0] * gg[0] + G[0] * last;
#pragma unroll
        for (int k = 0; k < NSMAX; ++k)
            if (k < N) o[k] = O[k] * al[k] + B[k] * w0;
    }
#pragma unroll
    for (int k = 0; k < NSMAX; ++k)
        if (k < N) base[(rev ? N - 1 - k : k) * 24] = o[k];
}

// ---------------------------------------------------------------------------
// M5 and M5^T in registers for Ns = 8, 16 and 32.  The N slices of a 4D site
// sit in N consecutive lanes of the wavefront (lane = s; a 16-lane DPP row
// holds two sites at N = 8, a site spans two rows at N = 32), so the
// recurrences above run across lanes with DPP row moves instead of an LDS
// transpose:
//   - the sweep al_k = F_k x_k - G_k al_{k-1} is a linear recurrence, done as
//     a Hillis-Steele scan (shifts by 1, 2, 4 [, 8] within the row,
//     multiplied by the products of the -G_j they skip, which are zero where
//     a shift would reach past the site's first slice or the row); at N = 32
//     the second row then takes the first row's last value times its own
//     prefix product of the -G_j;
//   - the corner equation needs al_{N-1} and the first input in every lane
//     (row broadcasts; at N = 8, where a row holds two sites, a lane read
//     through the LDS crossbar);
//   - Y and Y^T are one cyclic neighbour each (row rotation; lane read at
//     N = 8).
// The recurrence runs with s reversed for one chirality (REV): the shifts
// then go the other way along the row.
// ---------------------------------------------------------------------------

namespace dpp {
// DPP controls (row = 16 lanes): lane i reads lane i - n (shr), i + n (shl),
// (i - n) mod 16 (ror), or lane n of its row (bcast); out-of-row reads give 0.
constexpr int shr(int n) { return 0x110 + n; }
constexpr int shl(int n) { return 0x100 + n; }
constexpr int ror(int n) { return 0x120 + n; }
constexpr int bcast(int n) { return 0x150 + n; }

template <int CTRL>
__device__ __forceinline__ float mov(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double mov(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
}  // namespace dpp

// value at recurrence index k - D (0 if k < D; at N = 8 the other site's
// value where k < D, which the scan multiplies by zero)
template <bool REV, int D, class Real>
__device__ __forceinline__ Real rshift(Real x) {
    return dpp::mov<REV ? dpp::shl(D) : dpp::shr(D)>(x);
}
// x of lane src (byte address src * 4) through the LDS crossbar, no memory
__device__ __forceinline__ float lane_read(float x, int addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
}
__device__ __forceinline__ double lane_read(double x, int addr) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)b);
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lanes a slice reads at N = 8 and 32 (byte addresses for lane_read): the
// slice of recurrence index k - 1 mod N, those of indices 0 and N - 1 of its
// site and, at N = 32, that of index 15 (the end of the first DPP row in
// recurrence order).  (At N = 8 two sites share a DPP row, at N = 32 a site
// spans two, so row moves cannot serve these; one value per lane also keeps
// the compiler from carrying several copies across the component loop.)
struct LaneAddr {
    int prev, first, last, carry;
};
template <bool REV, int N>
__device__ __forceinline__ LaneAddr lane_addrs(int s) {
    const int base = (int)__lane_id() & ~(N - 1);
    const int sprev = REV ? (s + 1) & (N - 1) : (s + N - 1) & (N - 1);
    return LaneAddr{(base + sprev) * 4, (base + (REV ? N - 1 : 0)) * 4, (base + (REV ? 0 : N - 1)) * 4,
                    (base + (REV ? N - 16 : 15)) * 4};
}

// value at recurrence index (k - 1) mod N
template <bool REV, int N, class Real>
__device__ __forceinline__ Real rprev(Real x, const LaneAddr& la) {
    if constexpr (N == 16)
        return dpp::mov<REV ? dpp::ror(15) : dpp::ror(1)>(x);
    else
        return lane_read(x, la.prev);
}
// value at recurrence index K (0 or N - 1) of the lane's site
template <bool REV, int N, int K, class Real>
__device__ __forceinline__ Real ridx(Real x, const LaneAddr& la) {
    if constexpr (N == 16)
        return dpp::mov<dpp::bcast(REV ? 15 - K : K)>(x);
    else
        return lane_read(x, K == 0 ? la.first : la.last);
}
// value at recurrence index k - D within the DPP row, 1 where that leaves the row
template <bool REV, int D>
__device__ __forceinline__ float rshift_or1(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(1.0f), __float_as_int(x),
                                                      REV ? dpp::shl(D) : dpp::shr(D), 0xF, 0xF, false));
}
template <bool REV, int D>
__device__ __forceinline__ double rshift_or1(double x) {
    const long long b = __double_as_longlong(x), one = __double_as_longlong(1.0);
    constexpr int ctrl = REV ? dpp::shl(D) : dpp::shr(D);
    const int lo = __builtin_amdgcn_update_dpp((int)one, (int)b, ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(one >> 32), (int)(b >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One chirality block (12 components) of M5 (MODE = MIX_SA) or M5^T / M5^T g5
// (MIX_AS) on the lane's slice s, coefficients C = [F G B P Q O][N] of that
// block in recurrence order.  Every lane of the row must execute it.
template <class Real, int MODE, bool REV, int N>
__device__ __forceinline__ void mix_regn(Real* v, const Real* __restrict__ C, int s) {
    static_assert(N == 8 || N == 16 || N == 32, "register fifth-dimension matrices need 8, 16 or 32 slices");
    const int k = REV ? N - 1 - s : s;
    LaneAddr la{};
    if constexpr (N != 16) la = lane_addrs<REV, N>(s);
    const Real F = C[k], G = C[N + k], B = C[2 * N + k], P = C[3 * N + k], Q = C[4 * N + k], O = C[5 * N + k];
    const Real F0 = C[0], G0 = C[N];
    const Real Fk = k ? F : (Real)0;  // the sweep starts at k = 1
    // scan multipliers: A_d(k) = prod_{j = k-d+1..k} (-G_j), zero where k < d
    // (and, at N = 32, where the product would reach into the other DPP row)
    const Real A1 = k ? -G : (Real)0;
    const Real A2 = A1 * rshift<REV, 1>(A1);
    const Real A4 = A2 * rshift<REV, 2>(A2);
    Real A8 = 0;
    if constexpr (N >= 16) A8 = A4 * rshift<REV, 4>(A4);
    // N = 32: the scan runs in each DPP row alone; the second row (indices
    // 16..31) then adds prod_{j=16..k} (-G_j) times al_15, the product being
    // the row's prefix product of A1 (a multiplicative scan that reads 1
    // beyond the row start)
    Real Pc = 0;
    if constexpr (N == 32) {
        Real pr = A1;
        pr *= rshift_or1<REV, 1>(pr);
        pr *= rshift_or1<REV, 2>(pr);
        pr *= rshift_or1<REV, 4>(pr);
        pr *= rshift_or1<REV, 8>(pr);
        Pc = k >= 16 ? pr : (Real)0;
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const Real h = v[c];
        Real x;  // input of the X solve
        if constexpr (MODE == MIX_SA)
            x = h;
        else
            x = P * h + Q * rprev<REV, N>(h, la);  // Y^T sqrt(w)^-1 h
        Real al = Fk * x;
        al += A1 * rshift<REV, 1>(al);
        al += A2 * rshift<REV, 2>(al);
        al += A4 * rshift<REV, 4>(al);
        if constexpr (N >= 16) al += A8 * rshift<REV, 8>(al);
        if constexpr (N == 32) al += Pc * lane_read(al, la.carry);
        const Real w0 = F0 * ridx<REV, N, 0>(x, la) + G0 * ridx<REV, N, N - 1>(al, la);
        if constexpr (MODE == MIX_SA) {
            const Real w = al + B * w0;
            v[c] = P * w + Q * rprev<REV, N>(w, la);  // sqrt(w)^-1 Y w
        } else {
            v[c] = O * al + B * w0;  // sign sqrt(w) X^-T (...)
        }
        // one component at a time: interleaving them only raises register
        // pressure (and lowers occupancy) in these memory-bound kernels
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ---------------------------------------------------------------------------
// the fused kernel
//   phase 1: v = hop(in) on every (site, s) lane     [HOP]
//            v = prologue(site, s)                   [!HOP]
//   phase 2: the fifth-dimension matrix per 4D site  [MIXM != MIX_NONE]
//            (LDS transpose: lanes switch from (site, s) to (site, column))
//   phase 3: epilogue(site, s, v) -> norm contribution, block-reduced
//   phase 4: M5^T gamma_5 on the vector the epilogue left in v, stored by
//            epi.post                                [epilogue with kPost]
// One workgroup covers G consecutive 4D half sites x all Ns slices, lane
// (sl, s) = (tid / Ns, tid % Ns), so the SoA loads of consecutive lanes are
// consecutive 16-byte vectors and the G x 8 links are staged once in LDS
// and shared by the Ns slices (and by every right-hand side).
// ---------------------------------------------------------------------------

// A prologue or epilogue with set_ns(n) sets the component-block stride of
// its fields (kernels with the fifth-dimension matrices in registers make it a
// compile-time constant).
template <class T>
__device__ __forceinline__ auto set_ns_const(T& t, long n, int) -> decltype(t.set_ns(16L)) {
    t.set_ns(n);
}
template <class T>
__device__ __forceinline__ void set_ns_const(T&, long, long) {}

// An epilogue with a second output: kPost = true, a member ptab (the offset
// of the M5^T gamma_5 coefficients from the kernel's table, indexed per
// right-hand side in the same way) and post(rhs, i, s, v), which stores
// M5^T gamma_5 of what operator() left in v.
template <class E, class = void>
struct EpiPost {
    static constexpr bool value = false;
};
template <class E>
struct EpiPost<E, std::void_t<decltype(E::kPost)>> {
    static constexpr bool value = E::kPost;
};
// An epilogue with kPre = true also does one-workgroup work per right-hand
// side before the stencil: pre(rhs) for the launch's j-th right-hand side in
// workgroup j (mod the grid size).
template <class E, class = void>
struct EpiPre {
    static constexpr bool value = false;
};
template <class E>
struct EpiPre<E, std::void_t<decltype(E::kPre)>> {
    static constexpr bool value = E::kPre;
};

// The fifth-dimension matrix through LDS: each lane writes its (site, s)
// vector, the workgroup mixes the columns (chirality, site, real component),
// and each lane reads its vector back.  Every thread of the workgroup calls it.
template <class Real, int NSMAX, int MODE>
__device__ __forceinline__ void mix_lds(Real* v, Real* hb, const Real* __restrict__ tb, int Ns, int nsites, int sl,
                                        int s, bool act, int hs, int tid, int T) {
    if (act) {
        Real* dst = hb + sl * hs + s * 24;
#pragma unroll
        for (int k = 0; k < 24; ++k) dst[k] = v[k];
    }
    __syncthreads();
    // columns (chirality ch, site, real component c of that chirality);
    // every wave handles columns of one chirality so that the table
    // entries are wave-uniform (scalar loads).
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int nwaves = (T + 63) >> 6;
    const int ncol = nsites * 12;
    const int nch = (ncol + 63) >> 6;
    for (int c = wave; c < 2 * nch; c += nwaves) {
        const int ch = c / nch;
        const int col = (c - ch * nch) * 64 + lane;
        if (col < ncol) {
            const int cs = col / 12, cc = col - cs * 12;
            Real* base = hb + cs * hs + ch * 12 + cc;
            if constexpr (MODE == MIX_DENSE)
                mix_dense<Real, NSMAX>(base, tb + ch * Ns * Ns, Ns);
            else  // M5: reversed for L_-; M5^T: reversed for L_+^T = L_-
                mix_structured<Real, NSMAX, MODE>(base, tb + ch * 6 * Ns, Ns, (ch == 1) != (MODE == MIX_AS));
        }
    }
    __syncthreads();
    if (act) {
        const Real* src = hb + sl * hs + s * 24;
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = src[k];
    }
}

// M5 (MIX_SA) or M5^T (MIX_AS) in registers at Ns = N (8 or 16); every lane
// of the workgroup calls it (rows of inactive sites are whole rows, or at
// N = 8 half rows whose lanes hold zeros)
template <class Real, int MODE, int N>
__device__ __forceinline__ void mix_reg(Real* v, const Real* __restrict__ tb, int s) {
    // the coefficient loads stay after what precedes, whose register peak
    // they would otherwise raise
    __builtin_amdgcn_sched_barrier(0);
    constexpr bool rev0 = MODE == MIX_AS, rev1 = MODE != MIX_AS;  // M5: L_- reversed; M5^T: L_+^T
    mix_regn<Real, MODE, rev0, N>(v, tb, s);
    mix_regn<Real, MODE, rev1, N>(v + 12, tb + 6 * N, s);
}

struct KOpt {
    const int* live;       // per right-hand side; NULL = always run
    double* partials;      // [nrhs][nblocks] block sums when the epilogue reduces
    int nrhs;
    long table_rstride;    // elements between right-hand sides' tables (0 = shared)
    int rpb;               // right-hand sides per workgroup (0 = all): the grid holds
                           // nblocks x ngroups workgroups, group-major
    const int* glist;      // NULL: right-hand sides 0..nrhs-1; else glist[0] = n and
                           // glist[1..n] the right-hand sides the grid covers
    int ngroups;           // groups in the grid (0 = ceil(nrhs / rpb))
};

template <class Real>
__host__ __device__ inline int hbuf_site_stride(int Ns) {
    return Ns * 24 + (sizeof(Real) == 4 ? 12 : 6);
}

// LDS: [links G x 8 x LS reals][neighbours G x 8 ints][column buffer][reduction]
template <class Real>
__host__ __device__ inline size_t smem_links(int G, bool hop) {
    return hop ? (size_t)G * LdsLink<Real>::SITE * sizeof(Real) + (size_t)G * 8 * sizeof(int) : 0;
}

template <class Real>
__host__ __device__ inline size_t kernel_smem(int G, int Ns, bool hop, bool mix) {
    size_t b = smem_links<Real>(G, hop);
    if (mix) b += (size_t)G * hbuf_site_stride<Real>(Ns) * sizeof(Real);
    b = (b + 15) & ~(size_t)15;
    b += 16 * sizeof(double);
    return b;
}

// Which hop form a kernel uses (hop_site's PIPE).  The pipelined form with
// fused multiply-add chains takes fewer instructions and registers; it is
// faster everywhere on gfx950 except in the FP32 kernel D, whose streamed CG
// vectors already fill the register budget, which keeps the sequential form.
template <class A, class B, class C> struct EpiCgD;
template <class E> struct IsCgD { static constexpr bool value = false; };
template <class A, class B, class C> struct IsCgD<EpiCgD<A, B, C>> { static constexpr bool value = true; };
template <class F, class E> struct HopPipe {
    static constexpr bool value = !(std::is_same<F, FS>::value && IsCgD<E>::value);
};

template <class Real, class F, class LF, int NSMAX, bool HOP, int MIXM, bool REGMIX, class Pro, class Epi>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(std::is_same<F, FS>::value ? 4 : 1)))
k_dwf(Geom g, F in0, LF links, const Real* __restrict__ table, Pro pro0, Epi epi0, KOpt o) {
    // REGMIX: Ns == NSMAX (16 or 8), M5 / M5^T applied in registers (no LDS transpose)
    constexpr bool MIX = MIXM != MIX_NONE && !REGMIX;
    // With the fifth-dimension matrices in registers Ns = NSMAX: the slices of
    // a component block lie NSMAX vectors apart in every field, and with that
    // stride a constant, the vector loads and stores of a site share one
    // address (immediate offsets) and the index arithmetic folds.
    F in = in0;
    Pro pro = pro0;
    Epi epi = epi0;
    if constexpr (REGMIX) {
        in.ns = NSMAX;
        set_ns_const(pro, NSMAX, 0);
        set_ns_const(epi, NSMAX, 0);
    }
    // phase 4 runs in the same way as phase 2 (registers or LDS)
    constexpr bool POST = EpiPost<Epi>::value;
    static_assert(!POST || MIXM == MIX_SA || MIXM == MIX_AS, "phase 4 needs a kernel with a structured phase 2");
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int LS = LdsLink<Real>::STR;
    const int Ns = REGMIX ? NSMAX : g.Ns;
    const int tid = threadIdx.x, T = blockDim.x;

    // workgroup -> (group of right-hand sides, lattice block)
    const int L = xcd_remap(blockIdx.x, gridDim.x, g.xcd);
    const int grp = L / g.nblocks;
    const int lb = block_of(L - grp * g.nblocks, g);
    const int rpb = o.rpb > 0 ? o.rpb : o.nrhs;
    const int nsel = o.glist ? o.glist[0] : o.nrhs;
    const int j0 = grp * rpb, j1 = min(nsel, j0 + rpb);
    auto rhs_of = [&](int j) { return o.glist ? o.glist[1 + j] : j; };

    if constexpr (EpiPre<Epi>::value)
        for (int j = blockIdx.x; j < nsel; j += gridDim.x) epi.pre(rhs_of(j));

    if (o.live) {  // uniform early exit when no right-hand side of the group is live
        int any = 0;
        for (int j = j0; j < j1; ++j) any |= o.live[rhs_of(j)];
        if (!any) return;
    }

    Real* lk = (Real*)smem;
    int* nbl = (int*)(lk + g.G * LdsLink<Real>::SITE);
    Real* hb = (Real*)(smem + smem_links<Real>(g.G, HOP));
    size_t off = smem_links<Real>(g.G, HOP) + (MIX ? (size_t)g.G * hbuf_site_stride<Real>(Ns) * sizeof(Real) : 0);
    off = (off + 15) & ~(size_t)15;
    double* red = (double*)(smem + off);

    const long site0 = (long)lb * g.G;
    const int nsites = (int)min((long)g.G, (long)g.V4h - site0);
    const int sl = tid / Ns, s = tid - sl * Ns;
    const bool act = sl < nsites;
    const long h4 = site0 + sl;
    const long i5 = (long)s + (long)Ns * h4;
    const int hs = hbuf_site_stride<Real>(Ns);

    int nb[8];
    if constexpr (HOP) {
        // links scaled by -1/2 (Eq. (14)); links crossing the t boundary also
        // carry the antiperiodic sign
        const int vol3h = g.Lxh * g.Ly * g.Lz;
        auto sc = [&](int l) -> Real {
            const int k = l & 7;
            if (g.antiper && (k & 3) == 3) {
                const int t = (int)((site0 + (l >> 3)) / vol3h);
                if ((k == 3 && t == g.Lt - 1) || (k == 7 && t == 0)) return (Real)0.5;
            }
            return (Real)-0.5;
        };
        links.stage(lk, site0, nsites, tid, T, sc);
        // neighbour indices, once per site
        if (tid < nsites) {
            int q[8], tf, tb;
            neighbours(g, (int)(site0 + tid), g.out_parity, q, tf, tb);
#pragma unroll
            for (int k = 0; k < 8; ++k) nbl[tid * 8 + k] = q[k];
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int k = 0; k < 8; ++k) nb[k] = nbl[sl * 8 + k];
        }
    }

    for (int j = j0; j < j1; ++j) {
        const int rhs = rhs_of(j);
        if (o.live && !o.live[rhs]) continue;
        Real v[24];
        if (act) {
            if constexpr (HOP)
                hop_site<Real, HopPipe<F, Epi>::value>(in, rhs, s, Ns, nb, lk + sl * LdsLink<Real>::SITE, v);
            else
                pro(rhs, i5, s, v);
        } else {
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = 0;
        }
        if constexpr (MIX)
            mix_lds<Real, NSMAX, MIXM>(v, hb, table + rhs * o.table_rstride, Ns, nsites, sl, s, act, hs, tid, T);
        if constexpr (REGMIX) mix_reg<Real, MIXM, NSMAX>(v, table + rhs * o.table_rstride, s);
        double part = 0;
        if (act) part = epi(rhs, i5, s, v);
        if constexpr (POST) {
            const Real* tb = table + epi.ptab + rhs * o.table_rstride;
            if constexpr (REGMIX) {
                mix_reg<Real, MIX_AS, NSMAX>(v, tb, s);
            } else {
                __syncthreads();  // every lane has read back its phase-2 vector
                mix_lds<Real, NSMAX, MIX_AS>(v, hb, tb, Ns, nsites, sl, s, act, hs, tid, T);
            }
            if (act) epi.post(rhs, i5, s, v);
        }
        if constexpr (Epi::kReduce) {
            double tot = block_sum(part, red);
            if (tid == 0) o.partials[(long)rhs * g.nblocks + lb] = tot;
        }
        if constexpr (MIX) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// per-right-hand-side CG state (device arrays of length nrhs)
// ---------------------------------------------------------------------------

struct CgState {
    double* rr;         // |r|^2 of the current iterate
    double* uu;         // |u|^2 = (p, C C^dag p)
    double* alpha;
    double* beta;
    double* rr_target;  // the inner solve stops once rr <= rr_target
    double* aux;        // generic reduction results
    double* ecr;        // coefficient of r in the next direction update (kernel E)
    int* live;          // 1 while the inner solve runs
    int* iters;         // inner iterations done (all cycles)
    int* status;        // 0 running, 1 converged, 2 breakdown, 3 iteration cap, 4 diverged
    int* maxiter;
    int* live_host;     // mapped pinned host copy of live (NULL = none), written when a
                        // right-hand side stops, so the host sees it without a copy
};


// ---------------------------------------------------------------------------
// prologues (phase 1 without a hop)
// ---------------------------------------------------------------------------

template <class F>
struct ProLoad {
    F f;
    __device__ __forceinline__ void set_ns(long n) { f.ns = n; }
    template <class Real>
    __device__ __forceinline__ void operator()(int rhs, long i, int s, Real* v) const { f.load(rhs, i, s, v); }
};

// CG kernel E, for the right-hand sides that solve C C^dag w = b: the
// direction update of Algorithm 1, p = c_r r + beta p (c_r and beta as for
// kernel B), stored, and handed on for t1 = M5^T gamma_5 p.
template <class FR, class FP>
struct ProCgE {
    FR r;
    FP p;
    const double* beta;
    const double* ecr;
    __device__ __forceinline__ void set_ns(long n) { r.ns = p.ns = n; }
    template <class Real>
    __device__ __forceinline__ void operator()(int rhs, long i, int s, Real* v) const {
        r.sload(rhs, i, s, v);
        const Real a = (Real)ecr[rhs];
        const Real b = (Real)beta[rhs];
        Real q[24];
        p.sload(rhs, i, s, q);
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = a * v[k] + b * q[k];
        p.sstore(rhs, i, s, v);
    }
};

// ---------------------------------------------------------------------------
// epilogues (phase 3); return the lane's contribution to the block sum
// ---------------------------------------------------------------------------

template <class Real>
__device__ __forceinline__ double norm2_24(const Real* v) {
    Real s = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) s += v[k] * v[k];
    return (double)s;
}

template <class F, bool RED = false>
struct EpiStore {
    static constexpr bool kReduce = RED;
    F out;
    __device__ __forceinline__ void set_ns(long n) { out.ns = n; }
    template <class Real>
    __device__ __forceinline__ double operator()(int rhs, long i, int s, Real* v) const {
        out.store(rhs, i, s, v);  // the next kernel gathers it: cached
        return RED ? norm2_24(v) : 0.0;
    }
};

// Kernel C's epilogue: stores like EpiStore, and its first workgroups finish
// the reduction of kernel B for one right-hand side each before the stencil:
// (p, C C^dag p) = |u|^2 from B's block sums and alpha = |r|^2 / that, or a
// breakdown when it is not positive.  Kernel C does not read alpha, and the
// kernel boundary makes it visible to kernel D.  The first wave sums the
// block sums in a fixed order (lane l takes l, l + 64, ...; then a fixed
// butterfly), so alpha does not depend on the launch's shape or its other
// right-hand sides.
template <class F>
struct EpiStoreAlpha {
    static constexpr bool kReduce = false;
    static constexpr bool kPre = true;
    F out;
    const double* partials;  // [nrhs][nparts] block sums of kernel B
    int nparts;
    const CgState* st;       // the CG state (a copy in device memory)
    __device__ __forceinline__ void set_ns(long n) { out.ns = n; }
    template <class Real>
    __device__ __forceinline__ double operator()(int rhs, long i, int s, Real* v) const {
        out.store(rhs, i, s, v);  // the next kernel gathers it: cached
        return 0.0;
    }
    __device__ __forceinline__ void pre(int r) const;
};

template <class F>
__device__ __forceinline__ void EpiStoreAlpha<F>::pre(int r) const {
    if (threadIdx.x >= 64) return;
    if (!st->live[r]) return;
    const double* pr = partials + (long)r * nparts;
    double a = 0;
    for (int i = threadIdx.x; i < nparts; i += 64) a += pr[i];
    const double tot = wave_sum(a);
    if (threadIdx.x != 0) return;
    st->uu[r] = tot;
    if (!(tot > 0.0) || !isfinite(tot)) {  // breakdown
        st->status[r] = 2;
        st->live[r] = 0;
        if (st->live_host) st->live_host[r] = 0;
    } else {
        st->alpha[r] = st->rr[r] / tot;
    }
}

// stores nothing; returns |v|^2
struct EpiNorm {
    static constexpr bool kReduce = true;
    template <class Real>
    __device__ __forceinline__ double operator()(int, long, int, Real* v) const { return norm2_24(v); }
};

// out = ca * a + cv * (g5 ? gamma_5 v : v)
template <class FA, class FO, bool RED, bool G5>
struct EpiLin {
    static constexpr bool kReduce = RED;
    FA a;
    FO out;
    double ca, cv;
    template <class Real>
    __device__ __forceinline__ double operator()(int rhs, long i, int s, Real* v) const {
        Real w[24];
        a.load(rhs, i, s, w);
        const Real A = (Real)ca, B = (Real)cv;
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            Real vk = (G5 && k >= 12) ? -v[k] : v[k];
            w[k] = A * w[k] + B * vk;
        }
        out.store(rhs, i, s, w);
        return RED ? norm2_24(w) : 0.0;
    }
};

// CG kernel B: the new search direction in the form u = C^dag p.  Algorithm 1
// updates p = r + beta p; C^dag is linear, so u = C^dag p follows the same
// recurrence, u = c_r C^dag r + beta u, with C^dag r = r - gamma_5 v
// (v = D^OE t2, t2 = M5^T D^EO M5^T gamma_5 r) and p itself never formed.
// c_r (ecr) is 1 after every iteration; a restart sets (c_r, beta) = (1, 0)
// on a zeroed u (fresh Krylov space) or (0, 1) (reliable update: u kept).
// The right-hand sides with accp[rhs] set (C C^dag w = b, whose solution
// takes w += alpha p) form p in kernel E and t2 from it, and take
// u = C^dag p = p - gamma_5 v directly: there the solution and the residual
// must see the same direction, which a recurrence for u would let drift apart
// by the rounding of the stored vectors.  Returns |u|^2 = (p, C C^dag p).
template <class FR, class FU>
struct EpiCgB {
    static constexpr bool kReduce = true;
    FR r;
    FU u;
    typename FU::Ptrs p;  // laid out as u
    const double* beta;
    const double* ecr;
    const int* accp;
    __device__ __forceinline__ void set_ns(long n) { r.ns = u.ns = n; }
    template <class Real>
    __device__ __forceinline__ double operator()(int rhs, long i, int s, Real* v) const {
        Real w[24];
        if (accp && accp[rhs]) {
            u.with(p).sload(rhs, i, s, w);
#pragma unroll
            for (int k = 0; k < 24; ++k) w[k] = k < 12 ? w[k] - v[k] : w[k] + v[k];
        } else {
            const Real a = (Real)ecr[rhs], b = (Real)beta[rhs];
            Real rr[24];
            r.sload(rhs, i, s, rr);
            u.sload(rhs, i, s, w);
#pragma unroll
            for (int k = 0; k < 24; ++k) w[k] = a * (k < 12 ? rr[k] - v[k] : rr[k] + v[k]) + b * w[k];
        }
        u.store(rhs, i, s, w);  // gathered by the next kernel: cached
        return norm2_24(w);
    }
};

// CG kernel D: q = u - v (v = M5 D^OE t3), r -= alpha q; returns |r|^2.  The
// solution takes y += alpha u (D x = b: y = C^dag w is tracked, so r is the
// residual of C y = b''), or w += alpha p for the right-hand sides with
// accp[rhs] set (C C^dag w = b: Algorithm 1 on A = C C^dag as printed).
// Phase 4 then forms t1 = M5^T gamma_5 r of the new residual, the first
// step of the next iteration's C^dag r (kernel E replaces it with
// M5^T gamma_5 p for the right-hand sides with accp[rhs] set).
template <class FU, class FR, class FY>
struct EpiCgD {
    static constexpr bool kReduce = true;
    static constexpr bool kPost = true;
    FU u;
    FR r;
    FY y;
    const double* alpha;
    typename FU::Ptrs p;   // laid out as u
    const int* accp;
    typename FR::Ptrs t1;  // laid out as r
    int ptab;              // the M5^T gamma_5 coefficients: kernel table + ptab
    __device__ __forceinline__ void set_ns(long n) { u.ns = r.ns = y.ns = n; }
    template <class Real>
    __device__ __forceinline__ double operator()(int rhs, long i, int s, Real* v) const {
        const Real a = (Real)alpha[rhs];
        Real uu[24], w[24];
        u.sload(rhs, i, s, uu);
        r.sload(rhs, i, s, w);
        // v := the new residual (left in v for phase 4)
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = w[k] - a * (uu[k] - v[k]);
        r.sstore(rhs, i, s, v);
        if (accp && accp[rhs]) u.with(p).sload(rhs, i, s, uu);
        y.sload(rhs, i, s, w);
#pragma unroll
        for (int k = 0; k < 24; ++k) w[k] += a * uu[k];
        y.sstore(rhs, i, s, w);
        return norm2_24(v);
    }
    template <class Real>
    __device__ __forceinline__ void post(int rhs, long i, int s, const Real* v) const {
        r.with(t1).store(rhs, i, s, v);  // the next kernel gathers it: cached
    }
};

// Outer step: rhat = b'' - (yhat - v) with v = M5 D^OE M5 D^EO yhat, i.e.
// rhat = b'' - C yhat in FP64; stores the low-precision r = rhat and zeroes
// the low-precision solution y; returns |rhat|^2.
template <class FB, class FYH, class FR, class FY>
struct EpiOuter {
    static constexpr bool kReduce = true;
    FB b2;
    FYH yh;
    FR r;
    FY y;
    __device__ __forceinline__ double operator()(int rhs, long i, int s, double* v) const {
        double bb[24], yy[24];
        b2.load(rhs, i, s, bb);
        yh.load(rhs, i, s, yy);
        double nrm = 0;
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            bb[k] = bb[k] - yy[k] + v[k];
            nrm += bb[k] * bb[k];
        }
        r.store(rhs, i, s, bb);
        double z[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) z[k] = 0;
        y.store(rhs, i, s, z);
        return nrm;
    }
};

// True residual of the 5D operator on one parity:
// res = b - (Xx + v) with v = D_w^{pq} (Y x)_q; returns |res|^2, stores nothing.
template <class FB, class FX>
struct EpiTrueRes {
    static constexpr bool kReduce = true;
    FB b;
    FX xx;
    __device__ __forceinline__ double operator()(int rhs, long i, int s, double* v) const {
        double bb[24], w[24];
        b.load(rhs, i, s, bb);
        xx.load(rhs, i, s, w);
        double nrm = 0;
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            double d = bb[k] - w[k] - v[k];
            nrm += d * d;
        }
        return nrm;
    }
};

}  // namespace dwf
