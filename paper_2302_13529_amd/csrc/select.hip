// select.hip -- device-side round selection of the greedy drivers (Algorithm 3, lines
// choosing x = argmax Delta; Algorithm 4, the same over CB or over V \ B), plus fills.
// Ties go to the smallest vertex id, which makes the argmax order-independent.
#include "imin_internal.h"

#include <algorithm>

namespace imin {
namespace {

constexpr int kSelBlock = 1024;

__global__ void fill_u64_kernel(unsigned long long *p, int64_t count, unsigned long long value)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t count, uint32_t value)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// (d, i) beats (bd, bi) when d is larger, or equal with a smaller id; i = -1 is "none".
__device__ __forceinline__ void better(unsigned long long &bd, int &bi, unsigned long long d, int i)
{
    if (i < 0) return;
    if (bi < 0 || d > bd || (d == bd && i < bi)) {
        bd = d;
        bi = i;
    }
}

__device__ void block_best(unsigned long long &bd, int &bi)
{
    __shared__ unsigned long long sd[kSelBlock];
    __shared__ int si[kSelBlock];
    sd[threadIdx.x] = bd;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = kSelBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            unsigned long long d = sd[threadIdx.x];
            int i = si[threadIdx.x];
            better(d, i, sd[threadIdx.x + s], si[threadIdx.x + s]);
            sd[threadIdx.x] = d;
            si[threadIdx.x] = i;
        }
        __syncthreads();
    }
    bd = sd[0];
    bi = si[0];
}

__global__ void argmax_partial_kernel(const unsigned long long *D, const uint32_t *bits, int mode,
                                      int32_t n, unsigned long long *part_d, int32_t *part_i)
{
    unsigned long long bd = 0;
    int bi = -1;
    for (int64_t v = blockIdx.x * (int64_t)kSelBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kSelBlock) {
        const bool bit = (bits[v >> 5] >> (v & 31)) & 1u;
        const bool cand = mode == 0 ? !bit : bit;
        if (cand) better(bd, bi, D[v], (int)v);
    }
    block_best(bd, bi);
    if (threadIdx.x == 0) {
        part_d[blockIdx.x] = bd;
        part_i[blockIdx.x] = bi;
    }
}

// Threshold 0 for every in-edge of v, by the threads of one workgroup.
__device__ __forceinline__ void mask_in_edges(uint32_t *thr, const int32_t *in_ptr,
                                              const int32_t *in_edge, int v)
{
    for (int32_t k = in_ptr[v] + threadIdx.x; k < in_ptr[v + 1]; k += blockDim.x)
        thr[in_edge[k]] = 0u;
}

__global__ void argmax_final_kernel(const unsigned long long *part_d, const int32_t *part_i,
                                    int32_t parts, uint32_t *inelig, uint32_t *cand, int32_t *B,
                                    int32_t slot, int32_t *out_x, uint32_t *thr,
                                    const int32_t *in_ptr, const int32_t *in_edge)
{
    unsigned long long bd = 0;
    int bi = -1;
    for (int p = threadIdx.x; p < parts; p += kSelBlock) better(bd, bi, part_d[p], part_i[p]);
    block_best(bd, bi);
    if (threadIdx.x == 0) {
        if (bi >= 0) {
            inelig[bi >> 5] |= 1u << (bi & 31);
            if (cand) cand[bi >> 5] &= ~(1u << (bi & 31));
            B[slot] = bi;
        }
        *out_x = bi;
    }
    if (bi >= 0) mask_in_edges(thr, in_ptr, in_edge, bi);
}

__global__ void set_bit_kernel(uint32_t *bits, int32_t v, int value)
{
    if (value) bits[v >> 5] |= 1u << (v & 31);
    else bits[v >> 5] &= ~(1u << (v & 31));
}

// In-edge thresholds of list[blockIdx.x ...] (grid-stride over the list): 0, or restored.
__global__ void mask_list_kernel(uint32_t *thr, const uint32_t *thr_orig, const int32_t *in_ptr,
                                 const int32_t *in_edge, const int32_t *list, int32_t count,
                                 int restore)
{
    for (int32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const int32_t v = list[i];
        for (int32_t k = in_ptr[v] + threadIdx.x; k < in_ptr[v + 1]; k += kSelBlock) {
            const int32_t e = in_edge[k];
            thr[e] = restore ? thr_orig[e] : 0u;
        }
    }
}

__global__ void mask_vertex_kernel(uint32_t *thr, const uint32_t *thr_orig, const int32_t *in_ptr,
                                   const int32_t *in_edge, int32_t v, const int32_t *v_dev,
                                   int restore)
{
    const int32_t x = v_dev ? *v_dev : v;
    if (x < 0) return;
    for (int64_t k = in_ptr[x] + blockIdx.x * (int64_t)kSelBlock + threadIdx.x; k < in_ptr[x + 1];
         k += (int64_t)gridDim.x * kSelBlock) {
        const int32_t e = in_edge[k];
        thr[e] = restore ? thr_orig[e] : 0u;
    }
}

__global__ void batch_zero_kernel(const InstanceDesc *inst)
{
    const InstanceDesc &I = inst[blockIdx.y];
    for (int64_t v = blockIdx.x * (int64_t)kSelBlock + threadIdx.x; v < I.n;
         v += (int64_t)gridDim.x * kSelBlock)
        I.D[v] = 0ull;
}

// Workgroup blockIdx.x scans share blockIdx.x % kArgParts of instance blockIdx.x / kArgParts
// (a multiple of 4 vertices); each thread takes 4 vertices at a time so that several loads
// are in flight. The candidates are the instance's CB in GreedyReplace's first phase, else
// the vertices whose seed/blocked bit is clear.
__global__ void batch_argmax_part_kernel(const InstanceDesc *inst, int32_t round,
                                         unsigned long long *part_d, int32_t *part_i)
{
    const InstanceDesc &I = inst[blockIdx.x / kArgParts];
    const int32_t k = (int32_t)(blockIdx.x % kArgParts);
    unsigned long long bd = 0;
    int bi = -1;
    if (I.ctrl[kCtrlDone] == 0u) {
        const int32_t step = I.step + round;
        const bool in_cb = I.gr_k >= 0 && step < I.gr_k;
        const uint32_t *bits = in_cb ? I.cand : I.inelig;
        const uint32_t flip = in_cb ? 0xFFFFFFFFu : 0u;  // candidates: bit set in CB, clear else
        const int32_t per = (((I.n + kArgParts - 1) / kArgParts) + 3) & ~3;
        const int32_t lo = k * per;
        const int32_t hi = min(I.n, lo + per);
        constexpr int kStep = 4 * kSelBlock;
        for (int32_t base = lo + 4 * (int32_t)threadIdx.x; base < hi; base += kStep) {
            unsigned long long d[4];
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t v = base + q;
                d[q] = v < hi ? I.D[v] : 0ull;
                w[q] = v < hi ? (bits[v >> 5] ^ flip) : 0xFFFFFFFFu;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t v = base + q;
                if (v < hi && !((w[q] >> (v & 31)) & 1u)) better(bd, bi, d[q], (int)v);
            }
        }
    }
    block_best(bd, bi);
    if (threadIdx.x == 0) {
        part_d[blockIdx.x] = bd;
        part_i[blockIdx.x] = bi;
    }
}

// One workgroup per instance: the best of its kArgParts shares, applied. It also ends the
// instance's round for the wavefront-level kernels: when one of them handed over more than
// half of the instance's samples, later rounds send them straight past it.
__global__ void batch_argmax_apply_kernel(const InstanceDesc *inst,
                                          const unsigned long long *part_d,
                                          const int32_t *part_i, int32_t round,
                                          uint32_t *done_count)
{
    const InstanceDesc &I = inst[blockIdx.x];
    unsigned long long bd = 0;
    int bi = -1;
    if (threadIdx.x < kArgParts)
        better(bd, bi, part_d[blockIdx.x * kArgParts + threadIdx.x],
               part_i[blockIdx.x * kArgParts + threadIdx.x]);
    block_best(bd, bi);
    __shared__ int s_go;
    if (threadIdx.x == 0) {
        if (2ull * I.ctrl[kCtrlWaveHanded] > (unsigned long long)I.theta)
            I.ctrl[kCtrlSkipWave] = 1u;
        I.ctrl[kCtrlWaveHanded] = 0u;
        if (2ull * I.ctrl[kCtrlPackHanded] > (unsigned long long)I.theta)
            I.ctrl[kCtrlSkipPack] = 1u;
        I.ctrl[kCtrlPackHanded] = 0u;
        s_go = 0;
        if (I.ctrl[kCtrlDone] == 0u) {
            const int32_t step = I.step + round;
            int32_t slot = step;
            bool last = false;
            int32_t u = -1;
            if (I.gr_k >= 0 && step >= I.gr_k) {
                slot = 2 * I.gr_k - 1 - step;
                u = I.B[slot];
                last = slot == 0;
            } else if (I.gr_k >= 0) {
                if (bi >= 0) I.cand[bi >> 5] &= ~(1u << (bi & 31));
                last = false;
            }
            if (bi >= 0) {
                I.inelig[bi >> 5] |= 1u << (bi & 31);
                I.B[slot] = bi;
                s_go = 1;
            }
            *I.x = bi;
            if (I.gr_k >= 0 && step >= I.gr_k && (bi == u || bi < 0 || last)) {
                I.ctrl[kCtrlDone] = 1u;
                if (done_count) atomicAdd(done_count, 1u);
            }
        }
    }
    __syncthreads();
    if (s_go) mask_in_edges(reinterpret_cast<uint32_t *>(I.thr4), I.in_ptr, I.in_edge, bi);
}

// One workgroup per instance in GreedyReplace's replacement pass: unblock the blocker u of
// this round's slot before the round's samples are drawn.
__global__ void batch_gr_prepare_kernel(const InstanceDesc *inst, int32_t round)
{
    const InstanceDesc &I = inst[blockIdx.x];
    if (I.gr_k < 0 || I.ctrl[kCtrlDone] != 0u) return;
    const int32_t step = I.step + round;
    if (step < I.gr_k || step >= 2 * I.gr_k) return;
    const int32_t u = I.B[2 * I.gr_k - 1 - step];
    if (threadIdx.x == 0) I.inelig[u >> 5] &= ~(1u << (u & 31));
    uint32_t *thr = reinterpret_cast<uint32_t *>(I.thr4);
    const uint32_t *orig = reinterpret_cast<const uint32_t *>(I.thr_orig);
    for (int32_t k = I.in_ptr[u] + threadIdx.x; k < I.in_ptr[u + 1]; k += kSelBlock)
        thr[I.in_edge[k]] = orig[I.in_edge[k]];
}

__global__ void batch_done_kernel(const InstanceDesc *inst, int32_t ninst, uint32_t *out)
{
    const int32_t i = blockIdx.x * kSelBlock + threadIdx.x;
    if (i < ninst) out[i] = inst[i].ctrl[kCtrlDone];
}

__global__ void batch_setup_kernel(const InstanceDesc *inst, const BatchStage *st,
                                   const int32_t *stage)
{
    const InstanceDesc &I = inst[blockIdx.x];
    const BatchStage &S = st[blockIdx.x];
    int32_t *seeds = const_cast<int32_t *>(I.seeds);
    for (int32_t k = threadIdx.x; k < I.nseeds; k += kSelBlock) seeds[k] = stage[S.seeds + k];
    for (int32_t k = threadIdx.x; k < S.words; k += kSelBlock)
        I.inelig[k] = (uint32_t)stage[S.bits + k];
    if (S.cand >= 0)
        for (int32_t k = threadIdx.x; k < S.words; k += kSelBlock)
            I.cand[k] = (uint32_t)stage[S.cand + k];
    if (threadIdx.x < kGatherStats) I.stats[threadIdx.x] = 0ull;
    if (threadIdx.x < kCtrlWords) I.ctrl[threadIdx.x] = 0u;
    uint32_t *thr = reinterpret_cast<uint32_t *>(I.thr4);
    const uint32_t *orig = reinterpret_cast<const uint32_t *>(I.thr_orig);
    if (S.nprev < 0) {
        for (int64_t e = threadIdx.x; e < (int64_t)I.nquads * 4; e += kSelBlock) thr[e] = orig[e];
    } else {
        for (int32_t i = 0; i < S.nprev; ++i) {
            const int32_t v = stage[S.prev + i];
            for (int32_t k = I.in_ptr[v] + threadIdx.x; k < I.in_ptr[v + 1]; k += kSelBlock)
                thr[I.in_edge[k]] = orig[I.in_edge[k]];
        }
    }
    __syncthreads();
    for (int32_t i = 0; i < S.nnow; ++i) mask_in_edges(thr, I.in_ptr, I.in_edge, stage[S.now + i]);
}

__global__ void batch_gather_kernel(const InstanceDesc *inst, const int32_t *rounds, int32_t *out,
                                    int32_t stride)
{
    const InstanceDesc &I = inst[blockIdx.x];
    int32_t *o = out + (int64_t)blockIdx.x * stride;
    for (int32_t k = threadIdx.x; k < rounds[blockIdx.x]; k += kSelBlock) o[kGatherB + k] = I.B[k];
    if (threadIdx.x < kGatherStats) {
        const unsigned long long v = I.stats[threadIdx.x];
        o[2 * threadIdx.x] = (int32_t)(uint32_t)v;
        o[2 * threadIdx.x + 1] = (int32_t)(uint32_t)(v >> 32);
    }
    if (threadIdx.x == 0) o[kGatherErr] = (int32_t)I.ctrl[kCtrlError];
}

int grid_for(int64_t count)
{
    int64_t g = (count + kSelBlock - 1) / kSelBlock;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

}  // namespace

hipError_t launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long value,
                           hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(count)), dim3(kSelBlock), 0, stream, p,
                       count, value);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t value, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(count)), dim3(kSelBlock), 0, stream, p,
                       count, value);
    return hipGetLastError();
}

hipError_t launch_argmax_apply(const unsigned long long *D, const uint32_t *bits, int mode,
                               int32_t n, unsigned long long *part_d, int32_t *part_i,
                               int32_t parts, uint32_t *inelig, uint32_t *cand, int32_t *B,
                               int32_t slot, int32_t *out_x, uint32_t *thr,
                               const int32_t *in_ptr, const int32_t *in_edge,
                               hipStream_t stream)
{
    int g = grid_for(n);
    if (g > parts) g = parts;
    hipLaunchKernelGGL(argmax_partial_kernel, dim3(g), dim3(kSelBlock), 0, stream, D, bits, mode,
                       n, part_d, part_i);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(argmax_final_kernel, dim3(1), dim3(kSelBlock), 0, stream, part_d, part_i, g,
                       inelig, cand, B, slot, out_x, thr, in_ptr, in_edge);
    return hipGetLastError();
}

hipError_t launch_set_bit(uint32_t *bits, int32_t v, int value, hipStream_t stream)
{
    hipLaunchKernelGGL(set_bit_kernel, dim3(1), dim3(1), 0, stream, bits, v, value);
    return hipGetLastError();
}

hipError_t launch_mask_list(uint32_t *thr, const uint32_t *thr_orig, const int32_t *in_ptr,
                            const int32_t *in_edge, const int32_t *list, int32_t count,
                            int restore, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(mask_list_kernel, dim3(std::min<int32_t>(count, 4096)), dim3(kSelBlock), 0,
                       stream, thr, thr_orig, in_ptr, in_edge, list, count, restore);
    return hipGetLastError();
}

hipError_t launch_mask_vertex(uint32_t *thr, const uint32_t *thr_orig, const int32_t *in_ptr,
                              const int32_t *in_edge, int32_t v, const int32_t *v_dev,
                              int restore, hipStream_t stream)
{
    hipLaunchKernelGGL(mask_vertex_kernel, dim3(16), dim3(kSelBlock), 0, stream, thr, thr_orig,
                       in_ptr, in_edge, v, v_dev, restore);
    return hipGetLastError();
}

hipError_t launch_batch_zero(const InstanceDesc *inst, int32_t ninst, hipStream_t stream)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_zero_kernel, dim3(64, ninst), dim3(kSelBlock), 0, stream, inst);
    return hipGetLastError();
}

hipError_t launch_batch_argmax(const InstanceDesc *inst, int32_t ninst, int32_t round,
                               unsigned long long *part_d, int32_t *part_i, uint32_t *done_count,
                               hipStream_t stream)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_argmax_part_kernel, dim3(ninst * kArgParts), dim3(kSelBlock), 0,
                       stream, inst, round, part_d, part_i);
    hipLaunchKernelGGL(batch_argmax_apply_kernel, dim3(ninst), dim3(kSelBlock), 0, stream, inst,
                       part_d, part_i, round, done_count);
    return hipGetLastError();
}

hipError_t launch_batch_gr_prepare(const InstanceDesc *inst, int32_t ninst, int32_t round,
                                   hipStream_t stream)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_gr_prepare_kernel, dim3(ninst), dim3(kSelBlock), 0, stream, inst,
                       round);
    return hipGetLastError();
}

hipError_t launch_batch_done(const InstanceDesc *inst, int32_t ninst, uint32_t *out,
                             hipStream_t stream)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_done_kernel, dim3((ninst + kSelBlock - 1) / kSelBlock),
                       dim3(kSelBlock), 0, stream, inst, ninst, out);
    return hipGetLastError();
}

hipError_t launch_batch_setup(const InstanceDesc *inst, const BatchStage *st,
                              const int32_t *stage, int32_t ninst, hipStream_t stream)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_setup_kernel, dim3(ninst), dim3(kSelBlock), 0, stream, inst, st,
                       stage);
    return hipGetLastError();
}

hipError_t launch_batch_gather(const InstanceDesc *inst, const int32_t *rounds, int32_t *out,
                               int32_t stride, int32_t ninst, hipStream_t stream)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_gather_kernel, dim3(ninst), dim3(kSelBlock), 0, stream, inst, rounds,
                       out, stride);
    return hipGetLastError();
}

}  // namespace imin
