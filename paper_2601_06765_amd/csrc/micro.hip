// Modular arithmetic inner loop, the paper's third microbenchmark (benchmark
// protocol, "Microbenchmarks": randomized residues, Barrett against
// Montgomery update kernels, updates/s and register use).  Every chain runs
// x <- b + x*a (mod p), one update of the form of equation "mod-fma" per step,
// with the running value as a factor so that nothing is loop-invariant.  A
// thread carries MODLOOP_CPT independent chains to cover the multiply latency.
// The forms are the exact helpers the elimination kernels use, plus the
// Montgomery product of section "Montgomery multiplication and domain reuse".
#include "internal.hpp"

#define MODLOOP_CPT 4
#define MODLOOP_WG 256

template <int FORM>
__device__ __forceinline__ u32 modloop_step(const Fp& f, const Mont& m, u32 x, u32 a, u32 b) {
    if (FORM == 0) {  // p < 2^16: 24-bit product, float quotient, then a modular add
        const u32 s = fp_mul16(f, x, a) + b;
        return min(s, s - f.p);
    }
    if (FORM == 1) return fp_fma_t<true>(f, b, x, a);   // p < 2^16: one-word Barrett of b + x*a < 2^32
    if (FORM == 2) return fp_fma_t<false>(f, b, x, a);  // two-word Barrett of b + x*a
    const u32 s = mont_mul(m, x, a) + b;                // Montgomery domain throughout
    return min(s, s - m.p);
}

template <int FORM>
__global__ __launch_bounds__(MODLOOP_WG) void k_modloop(Fp f, Mont m, u32 nchains, u32 iters, const u32* __restrict__ x0,
                                                         const u32* __restrict__ a0, const u32* __restrict__ b0,
                                                         u32* __restrict__ out) {
    const u32 T = gridDim.x * MODLOOP_WG;  // chain c = t + k*T for k < MODLOOP_CPT
    const u32 t = blockIdx.x * MODLOOP_WG + threadIdx.x;
    u32 x[MODLOOP_CPT], a[MODLOOP_CPT], b[MODLOOP_CPT];
#pragma unroll
    for (u32 k = 0; k < MODLOOP_CPT; ++k) {
        const u32 c = min(t + k * T, nchains - 1);  // spare lanes repeat the last chain and store nothing
        x[k] = x0[c];
        a[k] = a0[c];
        b[k] = b0[c];
        if (FORM == 3) {  // into the Montgomery domain: v -> v*R mod p
            x[k] = mont_mul(m, x[k], m.r2);
            a[k] = mont_mul(m, a[k], m.r2);
            b[k] = mont_mul(m, b[k], m.r2);
        }
    }
    for (u32 i = 0; i < iters; ++i) {
#pragma unroll
        for (u32 k = 0; k < MODLOOP_CPT; ++k) x[k] = modloop_step<FORM>(f, m, x[k], a[k], b[k]);
    }
#pragma unroll
    for (u32 k = 0; k < MODLOOP_CPT; ++k) {
        const u32 c = t + k * T;
        if (c < nchains) out[c] = FORM == 3 ? mont_mul(m, x[k], 1u) : x[k];  // back to standard residues
    }
}

template <int FORM>
static void modloop_launch(Ctx& c, const Fp& f, const Mont& m, u32 grid, u32 nchains, u32 iters, const u32* x0,
                           const u32* a0, const u32* b0, u32* out) {
    hipLaunchKernelGGL(k_modloop<FORM>, dim3(grid), dim3(MODLOOP_WG), 0, c.stream, f, m, nchains, iters, x0, a0, b0,
                       out);
    F4_LAUNCH_CHECK();
}

template <int FORM>
static void modloop_attrs(u32* regs, u32* priv) {
    hipFuncAttributes at;
    F4_HIP_TRY(hipFuncGetAttributes(&at, reinterpret_cast<const void*>(&k_modloop<FORM>)));
    *regs = (u32)at.numRegs;
    *priv = (u32)at.localSizeBytes;
}

void modloop_run(Ctx& c, u32 p, u32 form, u32 nchains, u32 iters, const u32* x0, const u32* a0, const u32* b0, u32* out,
                 ModloopResult& res) {
    const Fp f = make_fp(p);
    const Mont m = make_mont(p);
    const u64 n = nchains;
    DBuf<u32> d(&c.pool, 4 * n);  // x0 | a | b | out
    upload(c, d.ptr, x0, n * 4);
    upload(c, d.ptr + n, a0, n * 4);
    upload(c, d.ptr + 2 * n, b0, n * 4);
    const u32 grid = (u32)ceil_div(ceil_div(n, MODLOOP_CPT), MODLOOP_WG);
    auto launch = [&](u32 it) {
        switch (form) {
            case 0: modloop_launch<0>(c, f, m, grid, nchains, it, d.ptr, d.ptr + n, d.ptr + 2 * n, d.ptr + 3 * n); break;
            case 1: modloop_launch<1>(c, f, m, grid, nchains, it, d.ptr, d.ptr + n, d.ptr + 2 * n, d.ptr + 3 * n); break;
            case 2: modloop_launch<2>(c, f, m, grid, nchains, it, d.ptr, d.ptr + n, d.ptr + 2 * n, d.ptr + 3 * n); break;
            default: modloop_launch<3>(c, f, m, grid, nchains, it, d.ptr, d.ptr + n, d.ptr + 2 * n, d.ptr + 3 * n);
        }
    };
    switch (form) {
        case 0: modloop_attrs<0>(&res.regs, &res.private_bytes); break;
        case 1: modloop_attrs<1>(&res.regs, &res.private_bytes); break;
        case 2: modloop_attrs<2>(&res.regs, &res.private_bytes); break;
        default: modloop_attrs<3>(&res.regs, &res.private_bytes);
    }
    launch(iters < 64 ? iters : 64);  // warm-up (same output buffer; the timed launch rewrites it)
    hipEvent_t e[2] = {nullptr, nullptr};
    try {
        F4_HIP_TRY(hipEventCreate(&e[0]));
        F4_HIP_TRY(hipEventCreate(&e[1]));
        F4_HIP_TRY(hipEventRecord(e[0], c.stream));
        launch(iters);
        F4_HIP_TRY(hipEventRecord(e[1], c.stream));
        F4_HIP_TRY(hipEventSynchronize(e[1]));
        float ms = 0.f;
        F4_HIP_TRY(hipEventElapsedTime(&ms, e[0], e[1]));
        res.kernel_ms = ms;
    } catch (...) {
        for (hipEvent_t v : e)
            if (v) (void)hipEventDestroy(v);
        throw;
    }
    for (hipEvent_t v : e) (void)hipEventDestroy(v);
    res.updates_per_s = res.kernel_ms > 0 ? (double)n * iters / (res.kernel_ms * 1e-3) : 0.0;
    readback(c, out, d.ptr + 3 * n, n * 4);
}
