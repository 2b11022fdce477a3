// kernels_resident.hip -- resident fold-in server kernel.
//
// The fold-in of a new user (its conditional mean against each stored
// posterior sample, averaged over the S samples; the row conditional of
// Section 2 / Algorithm 1 with z = 0) without a launch per request: a
// persistent kernel with one workgroup of S wavefronts per request slot.
// The slots live in coherent pinned host memory.  The host writes a request
// into a free slot and then bumps the slot's req_seq; the workgroup
//  * polls req_seq (one lane, relaxed loads; one acquire once it changes),
//  * copies the request into device staging of its own,
//  * computes in wavefront s the conditional mean for sample s with the same
//    building blocks (and so the same arithmetic) as bpmf_foldin, and its
//    dot products with the query columns into LDS (Lambda_s mu_s, constant,
//    is formed once at set-up),
//  * averages the S partials in sample order (wavefront 0), writes the
//    predictions into the slot and sets done_seq (one release).
// The samples of a request meet in LDS: a request costs one system-scope
// acquire and one release, where spreading its samples over workgroups would
// need device-wide fences per sample, and on a chip of several L2 caches each
// of those writes back or invalidates a whole L2.
//
// Every wave ends: on the host's stop flag, or after idle_polls polls during
// which the server assigned no request to any slot (about a microsecond each
// with the sleep between them); the host relaunches the kernel when a request
// is pending and the kernel has ended.
#include "resident.hpp"
#include "rowsolve.hpp"

namespace bpmf {

namespace {

template <int KP>
constexpr int resident_wave_floats()
{
    return RowShape<KP>::UNION + 64 + 3 * KP + 16;
}

extern __shared__ __attribute__((aligned(16))) float resident_lds[];

// Wavefront w of a request: conditional mean m_s against sample s = w, then
// m_s . v_q for the request's queries into the wavefront's u[q].  Not
// inlined: inside the persistent loop the compiler would otherwise hoist the
// per-lane addressing of every iteration into registers that it then spills.
// The LDS pointers are formed here, from the kernel's LDS array, so that
// their accesses stay LDS instructions.
template <int KP>
__device__ __attribute__((noinline)) void sample_mean(int w, int K, int64_t N, float alpha, float rbar,
                                                      const float *Vs, const double *Lam, const float *lam_mu,
                                                      const int32_t *dcols, const float *dvals, int nnz,
                                                      const int32_t *dq, int nq)
{
    using SH = RowShape<KP>;
    float *u = resident_lds + w * resident_wave_floats<KP>();
    float *rv = u + SH::UNION;
    float *colbuf = rv + 64;
    int *sidx = (int *)(colbuf + 3 * KP);
    const int lane = threadIdx.x & 63;
    // the arguments point to global memory; as plain pointers into a
    // function that is not inlined their loads would be flat loads, each
    // ordered against the wavefront's LDS accesses
    using gfloat = const __attribute__((address_space(1))) float;
    using gint = const __attribute__((address_space(1))) int32_t;
    using gdouble = const __attribute__((address_space(1))) double;
    gfloat *V = (gfloat *)(Vs + (int64_t)w * N * K);
    gdouble *L = (gdouble *)(Lam + (int64_t)w * K * K);
    floatx16 acc[SH::NTILE];
#pragma unroll
    for (int t = 0; t < SH::NTILE; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;
    float bacc = 0.0f;
    gram_f32<KP, WaveSync>((gint *)dcols, (gfloat *)dvals, nnz, V, K, rbar, u, rv, sidx, acc, bacc);
    store_precision<KP>(u, acc, K, alpha, [=](int rr, int cc) { return (float)L[rr * K + cc]; });
    const int ri = lane % KP;
    const float bb = ri < K ? fmaf(alpha, bacc, ((gfloat *)lam_mu)[(int64_t)w * K + ri]) : 0.0f;
    WaveSync::sync();
    bool fail;
    const float m = chol_solve<KP, WaveSync>(u, colbuf, K, bb, 0.0f, fail);
    if (lane < KP) colbuf[lane] = (ri < K) ? (fail ? __builtin_nanf("") : m) : 0.0f;
    WaveSync::sync();
    for (int q = lane; q < nq; q += 64) {
        gfloat *v = V + (int64_t)((gint *)dq)[q] * K;
        float p = 0.0f;
        for (int i = 0; i < K; ++i) p = fmaf(colbuf[i], v[i], p);
        u[q] = p;
    }
}

// Lambda_s mu_s for every stored sample, rounded to FP32 once: a constant of
// the model, formed at server set-up in the order bpmf_foldin forms it (so
// the predictions stay the same bit for bit).
__global__ void resident_lam_mu_kernel(int S, int K, const double *Lam, const double *mu, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * K) return;
    const int64_t s = i / K;
    const int ri = (int)(i - s * K);
    const double *L = Lam + s * K * K;
    const double *m0 = mu + s * K;
    double lm = 0.0;
    for (int c = 0; c < K; ++c) lm = fma(L[ri * K + c], m0[c], lm);
    out[i] = (float)lm;
}

template <int KP>
__global__ __launch_bounds__(1024) void resident_foldin_kernel(int S, int K, int64_t N, float alpha, float rbar,
                                                               const float *Vs, const double *Lam,
                                                               const double *mu, ResidentArgs ra)
{
    __shared__ int s_cmd, s_nnz, s_nq;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, nthr = blockDim.x;
    const int slot = blockIdx.x;
    ResidentSlotHeader *hs = (ResidentSlotHeader *)(ra.slots + (int64_t)slot * ra.slot_bytes);
    const int32_t *hcols = (const int32_t *)((char *)hs + RESIDENT_HEADER_BYTES);
    const float *hvals = (const float *)(hcols + ra.max_nnz);
    const int32_t *hq = (const int32_t *)(hvals + ra.max_nnz);
    float *hout = (float *)(hq + ra.max_q);
    int32_t *dcols = ra.dev_cols + (int64_t)slot * ra.max_nnz;
    float *dvals = ra.dev_vals + (int64_t)slot * ra.max_nnz;
    int32_t *dq = ra.dev_q + (int64_t)slot * ra.max_q;

    int my_done = 0, seen = 0;
    if (tid == 0) {
        my_done = __hip_atomic_load(&hs->done_seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
        seen = __hip_atomic_load(ra.stop + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    for (;;) {
        if (tid == 0) {
            int cmd = 2;
            for (int64_t idle = 0; idle < ra.idle_polls; ++idle) {
                // relaxed polls; the acquire fence follows a change only (an acquire
                // per poll would invalidate the caches the other slots compute from)
                const int rs = __hip_atomic_load(&hs->req_seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                if (rs != my_done) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                    my_done = rs;
                    s_nnz = hs->nnz;
                    s_nq = hs->nq;
                    cmd = 1;
                    break;
                }
                if ((idle & 63) == 63) {
                    if (__hip_atomic_load(ra.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0) break;
                    const int act = __hip_atomic_load(ra.stop + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    if (act != seen) {
                        seen = act;
                        idle = 0;
                    }
                }
                __builtin_amdgcn_s_sleep(8);
            }
            s_cmd = cmd;
        }
        __syncthreads();
        if (s_cmd != 1) break;
        // sizes were checked by the host; clamped again so no index leaves the slot
        const int nnz = min(max(s_nnz, 0), ra.max_nnz), nq = min(max(s_nq, 0), ra.max_q);
        for (int i = tid; i < nnz; i += nthr) {
            dcols[i] = hcols[i];
            dvals[i] = hvals[i];
        }
        for (int i = tid; i < nq; i += nthr) dq[i] = hq[i];
        __syncthreads();
        if (w < S) sample_mean<KP>(w, K, N, alpha, rbar, Vs, Lam, ra.lam_mu, dcols, dvals, nnz, dq, nq);
        __syncthreads();
        if (w == 0) {
            for (int q = lane; q < nq; q += 64) {
                float a = 0.0f;
                for (int t = 0; t < S; ++t) a += resident_lds[t * resident_wave_floats<KP>() + q];
                hout[q] = rbar + a / (float)S;
            }
            // lane 0's release orders this wavefront's stores before done_seq
            if (lane == 0) __hip_atomic_store(&hs->done_seq, my_done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

}  // namespace

size_t resident_lds_bytes(int K, int S)
{
    return (size_t)S * (K <= 32 ? resident_wave_floats<32>() : resident_wave_floats<64>()) * sizeof(float);
}

hipError_t prepare_resident(int S, int K, const double *Lam, const double *mu, float *lam_mu, hipStream_t st)
{
    const int64_t n = (int64_t)S * K;
    hipLaunchKernelGGL(resident_lam_mu_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, S, K, Lam,
                       mu, lam_mu);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int bytes = (int)resident_lds_bytes(K, S);
    return K <= 32 ? hipFuncSetAttribute((const void *)resident_foldin_kernel<32>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, bytes)
                   : hipFuncSetAttribute((const void *)resident_foldin_kernel<64>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t resident_max_slots(int K, int S, int *max_slots)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t lds = resident_lds_bytes(K, S);
    e = K <= 32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, resident_foldin_kernel<32>, 64 * S, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, resident_foldin_kernel<64>, 64 * S, lds);
    if (e != hipSuccess) return e;
    *max_slots = per_cu * cus;
    return hipSuccess;
}

hipError_t launch_resident(int n_slots, int S, int K, int64_t N, double alpha, double rbar, const float *Vs,
                           const double *Lam, const double *mu, const ResidentArgs &ra, hipStream_t st)
{
    if (n_slots <= 0 || S < 1 || S > 16 || K < 1 || K > 64) return hipErrorInvalidValue;
    const dim3 grid((unsigned)n_slots), block((unsigned)(64 * S));
    const size_t lds = resident_lds_bytes(K, S);
    const float fa = (float)alpha, fr = (float)rbar;
    if (K <= 32)
        hipLaunchKernelGGL(resident_foldin_kernel<32>, grid, block, lds, st, S, K, N, fa, fr, Vs, Lam, mu, ra);
    else
        hipLaunchKernelGGL(resident_foldin_kernel<64>, grid, block, lds, st, S, K, N, fa, fr, Vs, Lam, mu, ra);
    return hipGetLastError();
}

}  // namespace bpmf
