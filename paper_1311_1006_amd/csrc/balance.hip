// balance.hip -- near-field work split by source count.
//
// A leaf's near field sums over every source of its strong list; on
// clustered inputs a few lists hold orders of magnitude more sources than
// the rest, and one wavefront per leaf would leave the device idle while
// those few finish.  So every near-field work item (a leaf's group of
// targets) is cut into chunks of chunk_entries(n) consecutive entries of its
// strong list (n: the leaf's point count), at most kChunkSrc sources each.  A chunk of an item that has one chunk
// writes its targets directly; the chunks of a split item write partial sums
// that a combine pass adds in chunk order, so the result stays deterministic.
//
// Plan time: per item its chunk count, an exclusive scan, the expanded
// offsets of every launch class (read by the host at the plan's
// synchronisation), then the (item, chunk) list.
#include "fmm_internal.h"
#include "p2p_common.h"
#include "plan_extra.h"

namespace fmm {

struct BalItem {
    int32_t leaf, t0, tn, pad;
};

// chunks of every item: its leaf's strong-list entries over chunk_entries
__global__ void k_item_chunks(const BalItem* __restrict__ items, int n, const int32_t* __restrict__ s_cnt,
                              const int32_t* __restrict__ bcount, int32_t* icnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int leaf = items[i].leaf;
    const int ne = s_cnt[leaf], ce = chunk_entries(bcount[leaf]);
    icnt[i] = ne > ce ? (ne + ce - 1) / ce : 1;
}

// exclusive scan of icnt into ioff[0..n] (ioff[n] = total), blocks of 1024
__global__ void __launch_bounds__(1024)
k_iscan_reduce(const int32_t* __restrict__ v, int n, int32_t* bsum)
{
    __shared__ int sh[16];
    const int i = blockIdx.x * 1024 + threadIdx.x;
    int x = i < n ? v[i] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < 16; ++w) t += sh[w];
        bsum[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(1024)
k_iscan_apply(const int32_t* __restrict__ v, int n, const int32_t* __restrict__ bsum, int32_t* out)
{
    __shared__ int sh[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int base = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += 1024) base += bsum[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) base += __shfl_xor(base, o, 64);
    if (lane == 0) sh[wid] = base;
    __syncthreads();
    base = 0;
    for (int w = 0; w < 16; ++w) base += sh[w];
    __syncthreads();
    const int i = blockIdx.x * 1024 + threadIdx.x;
    const int x0 = i < n ? v[i] : 0;
    int x = x0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wid) pre += sh[w];
        tot += sh[w];
    }
    if (i < n) out[i] = base + pre + x - x0;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = base + tot;
}

// exclusive scan of n int32 values into out[0..n] (out[n] = total); bsum
// holds (n + 1023) / 1024 block sums
void launch_exclusive_scan(const int32_t* v, int n, int32_t* bsum, int32_t* out, hipStream_t s)
{
    const int nb = (n + 1023) / 1024;
    k_iscan_reduce<<<nb, 1024, 0, s>>>(v, n, bsum);
    k_iscan_apply<<<nb, 1024, 0, s>>>(v, n, bsum, out);
    check_launch("exclusive scan");
}

// expanded offsets of the launch classes: out[c] = ioff[base[c]]
__global__ void k_class_offsets(const int32_t* __restrict__ ioff, const int64_t* __restrict__ base, int ncls,
                                int64_t* out)
{
    const int c = threadIdx.x;
    if (c <= ncls) out[c] = ioff[base[c]];
}

__global__ void k_item_expand(int n, const int32_t* __restrict__ icnt, const int32_t* __restrict__ ioff, int2* x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = icnt[i], o = ioff[i];
    for (int k = 0; k < c; ++k) x[o + k] = make_int2(i, k);
}

// partial sums of split items, added in chunk order: one wavefront per item,
// lane = target, `vals` values per target
__global__ void __launch_bounds__(256)
k_item_combine(const BalItem* __restrict__ items, int n, const int32_t* __restrict__ icnt,
               const int32_t* __restrict__ ioff, const int32_t* __restrict__ bstart, const double* __restrict__ part,
               int vals, double* out)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int c = icnt[i];
    if (c <= 1) return;
    const BalItem it = items[i];
    if (lane >= it.tn) return;
    const int64_t o = ioff[i];
    const int64_t dst = (int64_t)bstart[it.leaf] + it.t0 + lane;
    for (int q = 0; q < vals; ++q) {
        // the values of sixteen chunks are loaded together, then added in
        // chunk order (one memory round trip per sixteen chunks instead of per
        // chunk)
        const double* pq = part + (o * kItemTargets + lane) * vals + q;
        const int64_t step = (int64_t)kItemTargets * vals;
        double s = 0.0;
        int k = 0;
        for (; k + 16 <= c; k += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = pq[(k + u) * step];
#pragma unroll
            for (int u = 0; u < 16; ++u) s += v[u];
        }
        for (; k < c; ++k) s += pq[k * step];
        out[dst * vals + q] = s;
    }
}

// Before the plan's synchronisation: chunk counts, offsets and the class
// offsets; the copy of the class offsets into b.cls completes with the
// caller's synchronisation.
void balance_launch(Plan::Balance& b, const void* items, int n, const std::vector<P2PClass>& cls,
                    const int32_t* s_cnt, const int32_t* bcount, hipStream_t s)
{
    const int ncls = (int)cls.size();
    b.icnt.alloc(std::max(n, 1), s);
    b.ioff.alloc(n + 1, s);
    const int nb = (n + 1023) / 1024;
    b.bsum.alloc(std::max(nb, 1), s);
    b.h_base.assign(ncls + 1, 0);
    for (int c = 0; c < ncls; ++c) b.h_base[c] = cls[c].off;
    b.h_base[ncls] = n;
    b.d_base.alloc(ncls + 1, s);
    FMM_HIP(hipMemcpyAsync(b.d_base.p, b.h_base.data(), sizeof(int64_t) * (ncls + 1), hipMemcpyHostToDevice, s));
    b.d_cls.alloc(ncls + 1, s);
    b.cls.assign(ncls + 1, 0);
    if (n > 0) {
        k_item_chunks<<<(n + 255) / 256, 256, 0, s>>>((const BalItem*)items, n, s_cnt, bcount, b.icnt.p);
        k_iscan_reduce<<<nb, 1024, 0, s>>>(b.icnt.p, n, b.bsum.p);
        k_iscan_apply<<<nb, 1024, 0, s>>>(b.icnt.p, n, b.bsum.p, b.ioff.p);
        k_class_offsets<<<1, 64, 0, s>>>(b.ioff.p, b.d_base.p, ncls, b.d_cls.p);
        check_launch("balance");
        FMM_HIP(hipMemcpyAsync(b.cls.data(), b.d_cls.p, sizeof(int64_t) * (ncls + 1), hipMemcpyDeviceToHost, s));
    }
}

// After the synchronisation: the (item, chunk) list and the partial buffer.
void balance_finish(Plan::Balance& b, int n, int vals, hipStream_t s)
{
    b.total = b.cls.empty() ? 0 : b.cls.back();
    b.vals = vals;
    b.xitems.alloc(std::max<int64_t>(b.total, 1), s);
    if (n > 0) {
        k_item_expand<<<(n + 255) / 256, 256, 0, s>>>(n, b.icnt.p, b.ioff.p, b.xitems.p);
        check_launch("balance expand");
    }
    // partial sums only for the chunks of split items; sized for all chunks
    // when any item is split
    if (b.total > n) b.partial.alloc((size_t)b.total * kItemTargets * vals, s);
}

void combine_chunks(const Plan::Balance& b, const void* items, int n, const int32_t* bstart, double* out,
                    hipStream_t s)
{
    if (b.total <= n || n == 0) return;     // no item is split
    k_item_combine<<<(n + 3) / 4, 256, 0, s>>>((const BalItem*)items, n, b.icnt.p, b.ioff.p, bstart, b.partial.p,
                                               b.vals, out);
    check_launch("combine chunks");
}

// M2L chunks per box from the weak-list length
__global__ void k_box_chunks(int64_t nbox, const int32_t* __restrict__ w_cnt, int32_t* icnt)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nbox) return;
    const int n = w_cnt[i];
    icnt[i] = n > kChunkPairs ? (n + kChunkPairs - 1) / kChunkPairs : 1;
}

// Work chunks of a plan, after the list build.  Without long lists (the
// one-pass list build flags them) every item is one chunk and nothing is
// launched: the kernels then take item i as chunk (i, 0).
void plan_balance(Plan& pl, hipStream_t s)
{
    PlanExtra& ex = *pl.ex;
    TreeSchedule& sc = *pl.tree->sched;
    int n = 0;
    for (auto& c : ex.p2p_class) n = std::max<int>(n, (int)(c.off + c.n));
    const int nbx = (int)sc.nbox;
    Plan::Balance& bp = pl.bal;
    Plan::Balance& bm = pl.bal_m2l;
    if (!pl.split_p2p) {
        bp.xitems.release();
        bp.icnt.release();
        bp.cls.clear();
        for (auto& c : ex.p2p_class) bp.cls.push_back(c.off);
        bp.cls.push_back(n);
        bp.total = n;
    } else {
        balance_launch(bp, ex.p2p_items.p, n, ex.p2p_class, pl.s_cnt.p, sc.d_box_count.p, s);
    }
    if (!pl.split_m2l) {
        bm.xitems.release();
        bm.icnt.release();
        bm.cls.assign({0, (int64_t)nbx});
        bm.total = nbx;
    } else {
        bm.icnt.alloc(nbx, s);
        bm.ioff.alloc(nbx + 1, s);
        const int nb = (nbx + 1023) / 1024;
        bm.bsum.alloc(std::max(nb, 1), s);
        k_box_chunks<<<(unsigned)((nbx + 255) / 256), 256, 0, s>>>(nbx, pl.w_cnt.p, bm.icnt.p);
        k_iscan_reduce<<<nb, 1024, 0, s>>>(bm.icnt.p, nbx, bm.bsum.p);
        k_iscan_apply<<<nb, 1024, 0, s>>>(bm.icnt.p, nbx, bm.bsum.p, bm.ioff.p);
        check_launch("m2l balance");
        bm.h32 = 0;
        FMM_HIP(hipMemcpyAsync(&bm.h32, bm.ioff.p + nbx, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    if (!pl.split_p2p && !pl.split_m2l) return;
    FMM_HIP(hipStreamSynchronize(s));
    if (pl.split_p2p) balance_finish(bp, n, 2, s);
    if (pl.split_m2l) {
        bm.cls.assign({0, (int64_t)bm.h32});
        bm.total = bm.h32;
        bm.xitems.alloc(std::max<int64_t>(bm.total, 1), s);
        k_item_expand<<<(unsigned)((nbx + 255) / 256), 256, 0, s>>>(nbx, bm.icnt.p, bm.ioff.p, bm.xitems.p);
        check_launch("m2l balance expand");
        if (bm.total > nbx) bm.partial.alloc((size_t)bm.total * pl.p * 2, s);
    }
}

}  // namespace fmm
