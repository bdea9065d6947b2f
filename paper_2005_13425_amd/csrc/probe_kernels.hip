// probe_kernels.hip -- HBM bandwidth probes for the measured roofline.
//
// Sec. V measures the bandwidth a CG iteration could reach by replacing its
// computation with device copies of every load and store.  The probes here do
// the same with one streaming kernel over R read streams of n doubles, stream
// k starting at src + k * stride:
//   * write form: dst[i] = sum over k < R of stream_k[i] (R reads, one write
//     stream; R = 1 is a copy, R = 7 the 7:1 read:write byte mix of the FP64
//     local operator: u and six geometric factors in, w out);
//   * read-only form: every workgroup writes one partial sum, so only the
//     read streams touch HBM.
// With NT the loads and stores carry the non-temporal (streaming) hint, as the
// plain FP64 operator's do.  BLK interleaves the streams in blocks of one
// workgroup's pass (NEK_PROBE_BLOCK doubles), so that a workgroup reads one
// contiguous run, as the operator reads an element's u and factor planes.
// The stride lets the caller stagger the streams:
// when they sit a large power of two apart, the lanes' R loads of one
// iteration share their low address bits and can fall on the same HBM
// channels, which a layout like the operator's (six factor planes of one
// element 8 n^3 bytes apart) does not do.
#include "nek_internal.h"
#include "reduce.h"

namespace nek {
namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_PAIRS = 4;

typedef double dvec2 __attribute__((ext_vector_type(2)));

constexpr int64_t PROBE_CHUNK = (int64_t)PROBE_THREADS * PROBE_PAIRS;   // pairs per workgroup pass
static_assert(2 * PROBE_CHUNK == NEK_PROBE_BLOCK, "a probe block is one workgroup pass");

template <int R, bool NT, bool RO, bool BLK>
__global__ void __launch_bounds__(PROBE_THREADS)
probe_kernel(int64_t n, const double *__restrict__ src, int64_t stride, double *__restrict__ dst) {
    const int64_t npairs = n >> 1;
    const int64_t chunk = PROBE_CHUNK;
    dvec2 tot = dvec2{0.0, 0.0};
    for (int64_t base = blockIdx.x * chunk; base < npairs; base += (int64_t)gridDim.x * chunk) {
        dvec2 acc[PROBE_PAIRS];
#pragma unroll
        for (int m = 0; m < PROBE_PAIRS; ++m) acc[m] = dvec2{0.0, 0.0};
#pragma unroll
        for (int k = 0; k < R; ++k) {
            // pair q of stream k: at q in a stream of its own, or at q - base
            // in block base / chunk of the interleaved layout
            const dvec2 *s2 = BLK ? (const dvec2 *)src + ((base / chunk) * R + k) * chunk
                                  : (const dvec2 *)(src + (int64_t)k * stride) + base;
            // every lane loads (a lane past the end reads the last pair again):
            // no load in a branch, so all R * PROBE_PAIRS loads are in flight
            // together instead of one at a time
#pragma unroll
            for (int m = 0; m < PROBE_PAIRS; ++m) {
                const int64_t o = threadIdx.x + (int64_t)m * PROBE_THREADS;
                const int64_t oc = base + o < npairs ? o : npairs - 1 - base;
                const dvec2 v = NT ? __builtin_nontemporal_load(&s2[oc]) : s2[oc];
                acc[m] += base + o < npairs ? v : dvec2{0.0, 0.0};
            }
        }
#pragma unroll
        for (int m = 0; m < PROBE_PAIRS; ++m) {
            const int64_t q = base + threadIdx.x + (int64_t)m * PROBE_THREADS;
            if constexpr (RO) {
                tot += acc[m];
            } else if (q < npairs) {
                if (NT) __builtin_nontemporal_store(acc[m], &((dvec2 *)dst)[q]);
                else ((dvec2 *)dst)[q] = acc[m];
            }
        }
    }
    if constexpr (RO) {
        __shared__ double red[PROBE_THREADS / 64];
        const double s = block_sum<PROBE_THREADS>(tot.x + tot.y, red);
        if (threadIdx.x == 0) dst[blockIdx.x] = s;
    } else if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        // the odd last value: block npairs / chunk, position 2 * (npairs % chunk)
        double a = 0.0;
        for (int k = 0; k < R; ++k)
            a += BLK ? src[(((npairs / chunk) * R + k) * chunk + npairs % chunk) * 2]
                     : src[(int64_t)k * stride + n - 1];
        dst[n - 1] = a;
    }
}

template <int R, bool BLK>
void launch_rb(int64_t blocks, int64_t n, const double *src, int64_t stride, double *dst, bool nt, bool ro,
               hipStream_t s) {
    const dim3 grid((unsigned)blocks), block(PROBE_THREADS);
    if (ro) {
        if (nt) hipLaunchKernelGGL((probe_kernel<R, true, true, BLK>), grid, block, 0, s, n, src, stride, dst);
        else hipLaunchKernelGGL((probe_kernel<R, false, true, BLK>), grid, block, 0, s, n, src, stride, dst);
    } else {
        if (nt) hipLaunchKernelGGL((probe_kernel<R, true, false, BLK>), grid, block, 0, s, n, src, stride, dst);
        else hipLaunchKernelGGL((probe_kernel<R, false, false, BLK>), grid, block, 0, s, n, src, stride, dst);
    }
}

template <int R>
void launch_r(int64_t blocks, int64_t n, const double *src, int64_t stride, double *dst, bool nt, bool ro,
              bool blk, hipStream_t s) {
    if (blk) launch_rb<R, true>(blocks, n, src, stride, dst, nt, ro, s);
    else launch_rb<R, false>(blocks, n, src, stride, dst, nt, ro, s);
}

}  // namespace

int64_t probe_blocks(int64_t n, int grid_cap) {
    const int64_t per = (int64_t)PROBE_THREADS * PROBE_PAIRS * 2;
    int64_t blocks = (n + per - 1) / per;
    if (grid_cap > 0 && blocks > grid_cap) blocks = grid_cap;
    return blocks < 1 ? 1 : blocks;
}

hipError_t launch_probe(int64_t n, int nread, const double *src, int64_t stride, double *dst, int grid_cap,
                        bool streaming, bool read_only, bool blocked, hipStream_t s) {
    const int64_t blocks = probe_blocks(n, grid_cap);
    switch (nread) {
#define NEK_PROBE(R) \
    case R: launch_r<R>(blocks, n, src, stride, dst, streaming, read_only, blocked, s); break;
        NEK_PROBE(1) NEK_PROBE(2) NEK_PROBE(3) NEK_PROBE(4) NEK_PROBE(5) NEK_PROBE(6) NEK_PROBE(7)
        NEK_PROBE(8)
#undef NEK_PROBE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nek
