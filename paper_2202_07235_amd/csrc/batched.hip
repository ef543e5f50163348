// Host side of the persistent multi-job launch: job table, item order, launch.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "batched.h"

namespace radsvd {

// Job table and queues of align_pairs_batched_noalloc, for callers that cannot
// allocate: one copy per GPU for the life of the process.  Host code never
// uses this name as an address (on the host it is only a stand-in for the
// symbol); it uses the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static_assert(sizeof(fastk::BatchHeader) <= 256 &&
                  256 + (RADSVD_NOALLOC_MAX_JOBS * sizeof(fastk::BatchJob) + 255) / 256 * 256 <= kNoAllocScratchBytes,
              "the no-allocation scratch holds the header and the job table of the maximum job count");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

namespace fastk {

// copies one chunk of the job table (passed by value) into the workspace;
// the first chunk also resets the queue
__global__ void k_batch_table(TableChunk c, BatchHeader *hdr, BatchJob *jobs) {
    const int i = threadIdx.x;
    if (i < c.n) jobs[c.first + i] = c.jobs[i];
    if (c.first == 0 && i < 8 * kBatchClasses) {
        hdr->count[i >> 3][i & 7] = c.count[i >> 3][i & 7];
        hdr->next[i >> 3][i & 7] = 0u;
        if (i < kBatchClasses) hdr->base[i] = c.base[i];
        if (i == 0) {
            hdr->n_jobs = c.n_jobs;
            hdr->total = c.total;
        }
    }
}

}  // namespace fastk

namespace {

int batch_q_index(int Q) {
    for (int i = 0; i < 5; ++i)
        if (fastk::kBatchQ[i] == Q) return i;
    return -1;
}

int plan_kind(const radsvd_plan *p) {
    if (p->prec == RADSVD_FP32) return 0;
    if (p->prec == RADSVD_BF16) return 1;
    return p->products == 3 ? 2 : 3;
}

int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

}  // namespace

size_t batched_bytes(int n_jobs) {
    return align_up(sizeof(fastk::BatchHeader), 256) + align_up((size_t)n_jobs * sizeof(fastk::BatchJob), 256);
}

bool batched_supported(const radsvd_plan *p) {
    return fast_path_supported(p, RADSVD_OUT_BEST) && batch_q_index(p->Q) >= 0 && p->H8 >= 8 && p->H8 <= 32;
}

hipError_t launch_pairs_batched(const radsvd_plan *const *plans, int n_jobs, const radsvd_job_out *outs,
                                void *ws, hipStream_t s) {
    using namespace fastk;
    const int kind = plan_kind(plans[0]);
    // item order: class (four-wave tiles at two workgroups per CU, at one, then
    // eight-wave), then decreasing cost per item (translations x angles x work
    // per angle)
    std::vector<int> order(n_jobs), cls(n_jobs);
    std::vector<double> cost(n_jobs);
    size_t lds[2] = {0, 0};   // LDS per workgroup of classes 0 and 1
    for (int i = 0; i < n_jobs; ++i) {
        const radsvd_plan *p = plans[i];
        order[i] = i;
        cls[i] = wide_plan(p->prec, p->products, p->herm, p->Q) ? 2 : (fast_plan_wpc(p) == 2 ? 0 : 1);
        cost[i] = (double)p->T * p->Q * (std::log2((double)p->Q) + 0.25 * p->H8);
        if (cls[i] < 2) {
            // staging buffers (one at Q = 256 with two workgroups per CU) + parked Z values
            const int nstage = (cls[i] == 0 && p->Q == 256) ? 1 : 2;
            lds[cls[i]] = std::max(lds[cls[i]], (size_t)(nstage * 16 * 128 + (p->Q / 8) * 256) * sizeof(cx<float>));
        }
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return cls[x] != cls[y] ? cls[x] < cls[y] : cost[x] > cost[y]; });
    std::vector<BatchJob> jobs(n_jobs);
    int total = 0, n_cls[kBatchClasses] = {0, 0, 0};
    for (int k = 0; k < n_jobs; ++k) {
        const int i = order[k];
        const radsvd_plan *p = plans[i];
        BatchJob &J = jobs[k];
        memset(&J, 0, sizeof(J));
        Args &a = J.a;
        a.Af = p->Af;
        a.Bf = p->Bf;
        a.n_img = p->n_img;
        a.n_tgt = p->n_tgt;
        a.T = p->T;
        a.nTA = p->na_pad / kFastTA;
        a.nTB = p->nb_pad / kFastTB;
        a.band = p->band ? p->band : kDefaultBand;
        a.H8 = p->H8;
        a.nplanes = p->nplanes_a;
        a.flags = RADSVD_OUT_BEST;
        a.inv_s2 = 1.f;
        a.best_score = outs[i].best_score;
        a.best_m = outs[i].best_m;
        a.best_t = outs[i].best_t;
        a.lse_pair = nullptr;
        J.qi = batch_q_index(p->Q);
        J.hi = p->H8 / 8 - 1;
        // group cheap tiles: about the work of one Q = 256, T = 9, rank-16 tile per item
        const double ref = 9.0 * 256 * (8.0 + 4.0);
        J.group = std::max(1, std::min(16, (int)std::lround(ref / cost[i])));
        J.item0 = total;
        const int items = (a.nTA * a.nTB + J.group - 1) / J.group;
        total += items;
        n_cls[cls[i]] += items;   // jobs are in class order: class c starts after the items of classes < c
    }
    const int base[kBatchClasses] = {0, n_cls[0], n_cls[0] + n_cls[1]};
    // items of each XCD queue of a class: chunks x, x + 8, x + 16, ... of kChunk items
    int count[kBatchClasses][8] = {};
    for (int q = 0; q < kBatchClasses; ++q)
        for (int c = 0; (long)c * kChunk < n_cls[q]; ++c) count[q][c & 7] += std::min(kChunk, n_cls[q] - c * kChunk);
    char *w = reinterpret_cast<char *>(ws);
    BatchHeader *hdr = reinterpret_cast<BatchHeader *>(w);
    BatchJob *djobs = reinterpret_cast<BatchJob *>(w + align_up(sizeof(BatchHeader), 256));
    for (int first = 0; first < n_jobs; first += kTableChunk) {
        TableChunk c;
        memset(&c, 0, sizeof(c));
        c.first = first;
        c.n = std::min(kTableChunk, n_jobs - first);
        c.n_jobs = n_jobs;
        c.total = total;
        for (int q = 0; q < kBatchClasses; ++q) {
            c.base[q] = base[q];
            for (int x = 0; x < 8; ++x) c.count[q][x] = count[q][x];
        }
        for (int k = 0; k < c.n; ++k) c.jobs[k] = jobs[first + k];
        hipLaunchKernelGGL(k_batch_table, dim3(1), dim3(kTableChunk), 0, s, c, hdr, djobs);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int cus = device_cus();
    if (n_cls[0] > 0) {   // two workgroups per CU
        const int grid = std::max(1, std::min(n_cls[0], 2 * cus));
        switch (kind) {
        case 0: e = launch_batched2_fp32(hdr, djobs, grid, lds[0], s); break;
        case 1: e = launch_batched2_bf16(hdr, djobs, grid, lds[0], s); break;
        case 2: e = launch_batched2_bf16x3(hdr, djobs, grid, lds[0], s); break;
        default: e = launch_batched2_bf16x3_6(hdr, djobs, grid, lds[0], s); break;
        }
        if (e != hipSuccess) return e;
    }
    if (n_cls[1] > 0) {
        const int grid = std::max(1, std::min(n_cls[1], cus));
        switch (kind) {
        case 0: e = launch_batched_fp32(hdr, djobs, grid, lds[1], s); break;
        case 1: e = launch_batched_bf16(hdr, djobs, grid, lds[1], s); break;
        case 2: e = launch_batched_bf16x3(hdr, djobs, grid, lds[1], s); break;
        default: e = launch_batched_bf16x3_6(hdr, djobs, grid, lds[1], s); break;
        }
        if (e != hipSuccess) return e;
    }
    if (n_cls[2] > 0) e = launch_batched_wide(hdr, djobs, std::max(1, std::min(n_cls[2], cus)), s);
    return e;
}

}  // namespace radsvd
