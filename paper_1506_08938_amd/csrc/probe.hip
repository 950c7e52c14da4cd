// nmf_probe_gather: a measurement aid, not a step of the method.  It moves
// the bytes of the sparse data products' row gathers (Section 4.2: one row
// of the fixed factor per stored entry) in a given order with nothing else
// in the way -- no values, no multiply, almost no writes -- and with as many
// loads in flight per lane as the loop allows, so its rate is what this GPU
// can gather in that order: the ceiling the products are measured against.
//
// The index list is flattened into (entry, 16-byte segment) items;
// consecutive lanes take consecutive segments of one row (a row is read as
// contiguous 16-byte pieces across lanes) and each lane keeps U such
// gathers, of U different entries, in flight.  Every lane adds what it read
// and writes one float4 at the end, so nothing it loads is dead.
#include "nmf_internal.h"

using namespace nmfi;

namespace {

constexpr int kProbeBlocks = 2048, kProbeThreads = 256, kProbeU = 8;
static_assert(NMF_PROBE_GATHER_OUT_FLOATS == kProbeBlocks * kProbeThreads * 4, "output size");

__global__ __launch_bounds__(kProbeThreads) void k_gather_probe(const uint4 *__restrict__ table, int64_t rows,
                                                                 uint32_t segs, const int32_t *__restrict__ idx,
                                                                 uint32_t items, float4 *__restrict__ out) {
    const uint32_t tid = blockIdx.x * kProbeThreads + threadIdx.x;
    const uint32_t stride = kProbeBlocks * kProbeThreads;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (uint32_t b = tid; b < items; b += kProbeU * stride) {
        uint4 v[kProbeU];
#pragma unroll
        for (int u = 0; u < kProbeU; u++) {
            const uint32_t it = b + (uint32_t)u * stride;
            v[u] = make_uint4(0u, 0u, 0u, 0u);
            if (it < items) {
                const uint32_t e = it / segs, s = it - e * segs;
                int64_t row = idx[e];
                row = row < 0 ? 0 : (row >= rows ? rows - 1 : row);  // never outside the table
                v[u] = table[row * segs + s];
            }
        }
#pragma unroll
        for (int u = 0; u < kProbeU; u++) {
            acc.x += __uint_as_float(v[u].x);
            acc.y += __uint_as_float(v[u].y);
            acc.z += __uint_as_float(v[u].z);
            acc.w += __uint_as_float(v[u].w);
        }
    }
    out[tid] = acc;
}

}  // namespace

extern "C" int nmf_probe_gather(const void *table, int64_t rows, int32_t row_bytes, const int32_t *idx,
                                int64_t n, float *out, void *stream) {
    if (!table || !out || (!idx && n > 0)) return fail(NMF_E_INVAL, "table, idx and out must be non-NULL");
    if (rows < 1) return fail(NMF_E_INVAL, "rows must be >= 1");
    if (row_bytes < 16 || row_bytes % 16) return fail(NMF_E_INVAL, "row_bytes must be a positive multiple of 16");
    if (n < 0) return fail(NMF_E_INVAL, "n must be >= 0");
    const int64_t segs = row_bytes / 16;
    if (n * segs >= ((int64_t)1 << 32) - (int64_t)kProbeU * kProbeBlocks * kProbeThreads)
        return fail(NMF_E_INVAL, "n * row_bytes / 16 is too large for one probe");
    hipLaunchKernelGGL(k_gather_probe, dim3(kProbeBlocks), dim3(kProbeThreads), 0, (hipStream_t)stream,
                       (const uint4 *)table, rows, (uint32_t)segs, idx, (uint32_t)(n * segs), (float4 *)out);
    NMF_HIP(hipGetLastError());
    return NMF_OK;
}
