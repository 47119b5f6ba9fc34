// layout.hip -- boundary conversion (Sec. 3.1: host index of Eq. (12) <->
// the device structure-of-arrays), gauge link packing and compression,
// precision conversion, solution accumulation, and the one-block kernel that
// finishes the grid reductions of the CG scalars (Sec. 3.4).
#include <algorithm>
#include <math.h>

#include "dwf_ctx.h"

namespace dwf {

namespace {

constexpr int TPB = 256;

struct Dims {
    int Lx, Ly, Lz, Lt, Ns;
    long V4, V5;
};

Dims dims_of(const dwf_ctx* c) {
    return Dims{c->dims[0], c->dims[1], c->dims[2], c->dims[3], c->Ns, c->V4, c->V4 * c->Ns};
}

__device__ __forceinline__ int parity_of(long n4, const Dims& d) {
    int x = (int)(n4 % d.Lx);
    long r = n4 / d.Lx;
    int y = (int)(r % d.Ly);
    r /= d.Ly;
    int z = (int)(r % d.Lz);
    int t = (int)(r / d.Lz);
    return (x + y + z + t) & 1;
}

// host layout (FP64, [n4][s][24]) -> two half fields; one thread per 5D site
template <class F>
__global__ void k_host_to_half(const double* __restrict__ host, Dims d, F ev, F od) {
    long n5 = blockIdx.x * (long)blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (n5 >= d.V5) return;
    long n4 = n5 / d.Ns;
    int s = (int)(n5 - n4 * d.Ns);
    const double2* src = (const double2*)(host + ((long)rhs * d.V5 + n5) * 24);
    double v[24];
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        double2 q = src[j];
        v[2 * j] = q.x;
        v[2 * j + 1] = q.y;
    }
    long i5 = s + (long)d.Ns * (n4 >> 1);
    if (parity_of(n4, d))
        od.store(rhs, i5, s, v);
    else
        ev.store(rhs, i5, s, v);
}

template <class F>
__global__ void k_half_to_host(double* __restrict__ host, Dims d, F ev, F od) {
    long n5 = blockIdx.x * (long)blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (n5 >= d.V5) return;
    long n4 = n5 / d.Ns;
    int s = (int)(n5 - n4 * d.Ns);
    long i5 = s + (long)d.Ns * (n4 >> 1);
    double v[24];
    if (parity_of(n4, d))
        od.load(rhs, i5, s, v);
    else
        ev.load(rhs, i5, s, v);
    double2* dst = (double2*)(host + ((long)rhs * d.V5 + n5) * 24);
#pragma unroll
    for (int j = 0; j < 12; ++j) dst[j] = make_double2(v[2 * j], v[2 * j + 1]);
}

template <class FA, class FB>
__global__ void k_convert(FA a, FB b, long n) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (i >= n) return;
    double v[24];
    const int s = (int)(i % a.ns);
    a.load(rhs, i, s, v);
    b.store(rhs, i, s, v);
}

template <class F>
__global__ void k_zero(F f, long n, const int* mask) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (i >= n) return;
    if (mask && !mask[rhs]) return;
    double v[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0;
    f.store(rhs, i, (int)(i % f.ns), v);
}

template <class F>
__global__ void k_copy(F dst, F src, long n, const int* mask) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (i >= n) return;
    if (mask && !mask[rhs]) return;
    double v[24];
    const int s = (int)(i % src.ns);
    src.load(rhs, i, s, v);
    dst.store(rhs, i, s, v);
}

// yhat += y (FP64 accumulation of the low-precision correction), Alg. 2
template <class F>
__global__ void k_acc(FD yh, F y, long n, const int* mask) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (i >= n) return;
    if (mask && !mask[rhs]) return;
    double a[24], b[24];
    const int s = (int)(i % yh.ns);
    yh.load(rhs, i, s, a);
    y.load(rhs, i, s, b);
#pragma unroll
    for (int k = 0; k < 24; ++k) a[k] += b[k];
    yh.store(rhs, i, s, a);
}

// Gauge links of output parity par, one thread per (site, entry):
// entries 0..3 = U_mu(x), 4..7 = U_mu(x - mu)^dag, in all four formats.
__global__ void k_pack_links(const double* __restrict__ gauge, Dims d, int par, long V4h, double* d18, float* s18,
                             float* s12, _Float16* h12) {
    long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (id >= V4h * 8) return;
    long h4 = id >> 3;
    int k = (int)(id & 7);
    int Lxh = d.Lx / 2;
    int xh = (int)(h4 % Lxh);
    long r = h4 / Lxh;
    int y = (int)(r % d.Ly);
    r /= d.Ly;
    int z = (int)(r % d.Lz);
    int t = (int)(r / d.Lz);
    int x = 2 * xh + ((y + z + t + par) & 1);
    int c[4] = {x, y, z, t};
    int L[4] = {d.Lx, d.Ly, d.Lz, d.Lt};
    int mu = k & 3;
    bool back = k >= 4;
    if (back) c[mu] = (c[mu] - 1 + L[mu]) % L[mu];
    long n4 = c[0] + (long)d.Lx * (c[1] + (long)d.Ly * (c[2] + (long)d.Lz * c[3]));
    const double* U = gauge + (n4 * 4 + mu) * 18;
    double u[18];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            if (!back) {
                u[2 * (3 * a + b)] = U[2 * (3 * a + b)];
                u[2 * (3 * a + b) + 1] = U[2 * (3 * a + b) + 1];
            } else {  // dagger: conjugate transpose
                u[2 * (3 * a + b)] = U[2 * (3 * b + a)];
                u[2 * (3 * a + b) + 1] = -U[2 * (3 * b + a) + 1];
            }
        }
    long o = h4 * 8 + k;
    for (int j = 0; j < 18; ++j) {
        d18[o * 18 + j] = u[j];
        s18[o * 18 + j] = (float)u[j];
    }
    for (int j = 0; j < 12; ++j) {
        s12[o * 12 + j] = (float)u[j];
        h12[o * 12 + j] = (_Float16)u[j];
    }
}

constexpr int kFinT = 512;

// One workgroup per right-hand side: its block sums in a fixed order (thread
// i takes i, i + T, i + 2T, ... into four accumulators, then the block tree),
// so a right-hand side's result does not depend on how many others share the
// launch, and the sums of different right-hand sides run in parallel.
__global__ void __launch_bounds__(kFinT) k_finish(const double* __restrict__ partials, int nblocks, CgState st,
                                                  int mode, const int* __restrict__ mask) {
    __shared__ double red[kFinT / 64];
    const int r = blockIdx.x;
    if (mode == FIN_BETA && !st.live[r]) return;
    if ((mode == FIN_AUX || mode == FIN_OUTER) && mask && !mask[r]) return;
    const double* __restrict__ pr = partials + (long)r * nblocks;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int i = threadIdx.x;
    for (; i + 3 * kFinT < nblocks; i += 4 * kFinT) {
        s0 += pr[i];
        s1 += pr[i + kFinT];
        s2 += pr[i + 2 * kFinT];
        s3 += pr[i + 3 * kFinT];
    }
    for (; i < nblocks; i += kFinT) s0 += pr[i];
    const double tot = block_sum((s0 + s1) + (s2 + s3), red);
    if (threadIdx.x != 0) return;
    if (mode == FIN_AUX) {
        st.aux[r] = tot;
    } else if (mode == FIN_OUTER) {
        st.aux[r] = tot;
        st.rr[r] = tot;
    } else if (mode == FIN_BETA) {
        if (!isfinite(tot)) {
            st.status[r] = 2;
            st.live[r] = 0;
            if (st.live_host) st.live_host[r] = 0;
        } else {
            st.beta[r] = tot / st.rr[r];
            st.ecr[r] = 1.0;
            st.rr[r] = tot;
            st.iters[r] += 1;
            if (tot <= st.rr_target[r]) {
                st.live[r] = 0;
                st.status[r] = 1;
            } else if (tot > 1e8 * st.aux[r]) {  // |r| grew 1e4-fold since the restart
                st.live[r] = 0;
                st.status[r] = 4;
            } else if (st.iters[r] >= st.maxiter[r]) {
                st.live[r] = 0;
                st.status[r] = 3;
            }
            if (st.live_host && !st.live[r]) st.live_host[r] = 0;
        }
    }
}

// A plain copy of n 16-byte vectors, the calibration reference of the memory
// counters: NT = 1 reads and writes with non-temporal (streaming) accesses as
// the CG kernels do for vectors they touch once, NT = 0 with ordinary cached
// accesses as for the gathered hop inputs.  Four vectors in flight per lane.
template <bool NT>
__global__ void __launch_bounds__(256) k_stream_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     long n) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += 4 * stride) {
        f4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const long j = i + k * stride;
            if (j < n) v[k] = NT ? __builtin_nontemporal_load((const f4*)src + j) : ((const f4*)src)[j];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const long j = i + k * stride;
            if (j < n) {
                if (NT)
                    __builtin_nontemporal_store(v[k], (f4*)dst + j);
                else
                    ((f4*)dst)[j] = v[k];
            }
        }
    }
}

}  // namespace

hipError_t stream_copy(const void* src, void* dst, size_t bytes, bool nontemporal, hipStream_t s) {
    const long n = (long)(bytes / 16);
    // one pass of four vectors per lane up to 65536 workgroups (the grid at
    // which plain copies measured fastest; 4096 workgroups reached 10% less)
    const unsigned blocks = (unsigned)std::max(1L, std::min(65536L, (n + 1023) / 1024));
    if (nontemporal)
        hipLaunchKernelGGL(k_stream_copy<true>, dim3(blocks), dim3(256), 0, s, (const float4*)src, (float4*)dst, n);
    else
        hipLaunchKernelGGL(k_stream_copy<false>, dim3(blocks), dim3(256), 0, s, (const float4*)src, (float4*)dst, n);
    return hipGetLastError();
}

hipError_t launch_finish(const double* partials, int nblocks, int nrhs, CgState st, int mode, hipStream_t s,
                         const int* mask) {
    return launch_kernel(k_finish, dim3((unsigned)nrhs), dim3(kFinT), 0, s, partials, nblocks, st, mode, mask);
}

hipError_t host_to_half(const dwf_ctx* c, const double* host, int nrhs, HalfField& even, HalfField& odd,
                        hipStream_t s, int rhs0) {
    Dims d = dims_of(c);
    dim3 grid((unsigned)((d.V5 + TPB - 1) / TPB), nrhs);
    const int r0 = rhs0;
    switch (even.prec) {
        case DWF_PREC_FP64: hipLaunchKernelGGL(k_host_to_half<FD>, grid, dim3(TPB), 0, s, host, d, even.fd(r0), odd.fd(r0)); break;
        case DWF_PREC_FP32: hipLaunchKernelGGL(k_host_to_half<FS>, grid, dim3(TPB), 0, s, host, d, even.fs(r0), odd.fs(r0)); break;
        default: hipLaunchKernelGGL(k_host_to_half<FH>, grid, dim3(TPB), 0, s, host, d, even.fh(r0), odd.fh(r0)); break;
    }
    return hipGetLastError();
}

hipError_t half_to_host(const dwf_ctx* c, const HalfField& even, const HalfField& odd, int nrhs, double* host,
                        hipStream_t s, int rhs0) {
    Dims d = dims_of(c);
    dim3 grid((unsigned)((d.V5 + TPB - 1) / TPB), nrhs);
    const int r0 = rhs0;
    switch (even.prec) {
        case DWF_PREC_FP64: hipLaunchKernelGGL(k_half_to_host<FD>, grid, dim3(TPB), 0, s, host, d, even.fd(r0), odd.fd(r0)); break;
        case DWF_PREC_FP32: hipLaunchKernelGGL(k_half_to_host<FS>, grid, dim3(TPB), 0, s, host, d, even.fs(r0), odd.fs(r0)); break;
        default: hipLaunchKernelGGL(k_half_to_host<FH>, grid, dim3(TPB), 0, s, host, d, even.fh(r0), odd.fh(r0)); break;
    }
    return hipGetLastError();
}

template <class FA>
static hipError_t convert_to(const FA& a, HalfField& dst, long n, int nrhs, hipStream_t s) {
    dim3 grid((unsigned)((n + TPB - 1) / TPB), nrhs);
    switch (dst.prec) {
        case DWF_PREC_FP64: hipLaunchKernelGGL((k_convert<FA, FD>), grid, dim3(TPB), 0, s, a, dst.fd(), n); break;
        case DWF_PREC_FP32: hipLaunchKernelGGL((k_convert<FA, FS>), grid, dim3(TPB), 0, s, a, dst.fs(), n); break;
        default: hipLaunchKernelGGL((k_convert<FA, FH>), grid, dim3(TPB), 0, s, a, dst.fh(), n); break;
    }
    return hipGetLastError();
}

hipError_t half_convert(const dwf_ctx* c, const HalfField& src, HalfField& dst, int nrhs, hipStream_t s) {
    long n = c->V5h;
    switch (src.prec) {
        case DWF_PREC_FP64: return convert_to(src.fd(), dst, n, nrhs, s);
        case DWF_PREC_FP32: return convert_to(src.fs(), dst, n, nrhs, s);
        default: return convert_to(src.fh(), dst, n, nrhs, s);
    }
}

hipError_t half_zero(const dwf_ctx* c, HalfField& f, int nrhs, hipStream_t s, const int* mask) {
    long n = c->V5h;
    dim3 grid((unsigned)((n + TPB - 1) / TPB), nrhs);
    switch (f.prec) {
        case DWF_PREC_FP64: hipLaunchKernelGGL(k_zero<FD>, grid, dim3(TPB), 0, s, f.fd(), n, mask); break;
        case DWF_PREC_FP32: hipLaunchKernelGGL(k_zero<FS>, grid, dim3(TPB), 0, s, f.fs(), n, mask); break;
        default: hipLaunchKernelGGL(k_zero<FH>, grid, dim3(TPB), 0, s, f.fh(), n, mask); break;
    }
    return hipGetLastError();
}

hipError_t half_copy(const dwf_ctx* c, HalfField& dst, const HalfField& src, int nrhs, const int* mask,
                     hipStream_t s) {
    long n = c->V5h;
    dim3 grid((unsigned)((n + TPB - 1) / TPB), nrhs);
    switch (src.prec) {
        case DWF_PREC_FP64: hipLaunchKernelGGL(k_copy<FD>, grid, dim3(TPB), 0, s, dst.fd(), src.fd(), n, mask); break;
        case DWF_PREC_FP32: hipLaunchKernelGGL(k_copy<FS>, grid, dim3(TPB), 0, s, dst.fs(), src.fs(), n, mask); break;
        default: hipLaunchKernelGGL(k_copy<FH>, grid, dim3(TPB), 0, s, dst.fh(), src.fh(), n, mask); break;
    }
    return hipGetLastError();
}

hipError_t half_acc(const dwf_ctx* c, HalfField& yhat, const HalfField& y, int nrhs, const int* mask,
                    hipStream_t s) {
    long n = c->V5h;
    dim3 grid((unsigned)((n + TPB - 1) / TPB), nrhs);
    switch (y.prec) {
        case DWF_PREC_FP64: hipLaunchKernelGGL(k_acc<FD>, grid, dim3(TPB), 0, s, yhat.fd(), y.fd(), n, mask); break;
        case DWF_PREC_FP32: hipLaunchKernelGGL(k_acc<FS>, grid, dim3(TPB), 0, s, yhat.fd(), y.fs(), n, mask); break;
        default: hipLaunchKernelGGL(k_acc<FH>, grid, dim3(TPB), 0, s, yhat.fd(), y.fh(), n, mask); break;
    }
    return hipGetLastError();
}

hipError_t pack_links(const dwf_ctx* c, const double* gauge_dev, hipStream_t s) {
    Dims d = dims_of(c);
    for (int par = 0; par < 2; ++par) {
        long n = c->V4h * 8;
        hipLaunchKernelGGL(k_pack_links, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, s, gauge_dev, d, par,
                           c->V4h, c->links[par][LINK_D18].as<double>(), c->links[par][LINK_S18].as<float>(),
                           c->links[par][LINK_S12].as<float>(), c->links[par][LINK_H12].as<_Float16>());
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dwf
