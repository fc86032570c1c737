// gen.hip -- the synthetic streams of frames.py, one thread per pixel on the
// GPU.  Same hash (MurmurHash3 fmix32), same palette, drift, bimodal pixels,
// noise table and foreground objects; frames.py computes the per-frame
// numbers (frame hash, drift scale, object positions) and this kernel only
// evaluates the per-pixel integer formula, so both give identical bytes.
// Inputs only: none of the method's arithmetic is here.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace {

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

constexpr int kMaxObj = 6;
constexpr int kFrameInts = 4 + 8 * kMaxObj;   // per-frame record, int32 fields

struct StreamConst {
    int32_t width, height;
    int64_t row_pitch, frame_pitch;
    uint32_t kp;          // palette key
    uint32_t kb;          // bimodal key
    uint32_t bthr;        // bimodal threshold on a 32-bit hash
    int32_t bimodal;      // 0/1
    int32_t period;       // bimodal period in frames
    int32_t block, n_palette;
    uint32_t t0, t1, t2;  // palette pick thresholds on a 16-bit draw
};

// frame record: [0] frame index, [1] frame hash, [2] drift scale (Q16),
// [3] number of objects, then per object: kind (0 rect, 1 ellipse), x, y, a,
// b, R, G, B
// The 16 pixels x0 = 16*gx .. x0+15 of row y of one frame (fewer at the row
// end), written as 48 bytes with three 16-byte stores when the group is whole.
template <typename NT>
__device__ __forceinline__ void gen_group(const StreamConst &sc, const int32_t *__restrict__ r,
                                          const NT *__restrict__ ntab, uint8_t *__restrict__ fo, int y, int gx) {
    const int f = r[0];
    const uint32_t hf = (uint32_t)r[1];
    const int32_t scale = r[2];
    const int nobj = r[3];
    const int x0 = gx * 16;
    const int nv = min(16, sc.width - x0);
    const int nbx = (sc.width + sc.block - 1) / sc.block;
    const uint32_t prow = (uint32_t)y * (uint32_t)sc.width;
    const uint32_t brow = (uint32_t)(y / sc.block) * (uint32_t)nbx;
    int bx = x0 / sc.block, br = x0 - bx * sc.block;
    // objects that reach this row
    uint32_t rowhit = 0;
    for (int o = 0; o < nobj; ++o) {
        const int32_t *ob = r + 4 + 8 * o;
        const int py = ob[2], b = ob[4];
        const bool hit = ob[0] == 0 ? (y >= py && y < py + b) : (y - py <= b && py - y <= b);
        rowhit |= (hit ? 1u : 0u) << o;
    }
    uint32_t w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = 0;
#pragma unroll
    for (int p = 0; p < 16; ++p) {
        if (p < nv) {
            const int x = x0 + p;
            const uint32_t pix = prow + (uint32_t)x;
            const uint32_t base = fmix32(pix ^ hf);
            const uint32_t u = base & 0xFFFFu;
            uint32_t ci = (u >= sc.t0) + (u >= sc.t1) + (u >= sc.t2);
            if (sc.bimodal) {
                const uint32_t hb = fmix32(pix ^ sc.kb);
                if (hb < sc.bthr) {
                    const uint32_t phase = fmix32(hb ^ 0x5851F42Du) % (uint32_t)sc.period;
                    ci = ((uint32_t)(f + phase) % (uint32_t)sc.period >= 4u) ? 1u : 0u;
                }
            }
            const uint32_t idx = (brow + (uint32_t)bx) * (uint32_t)sc.n_palette + ci;
            uint32_t h = fmix32(idx ^ sc.kp);
            h = fmix32(h + 0x632BE5ABu);
            int c0 = (int)(h & 255u), c1 = (int)((h >> 8) & 255u), c2 = (int)((h >> 16) & 255u);
            if (scale != 65536) {
                c0 = min((c0 * scale + 32768) >> 16, 255);
                c1 = min((c1 * scale + 32768) >> 16, 255);
                c2 = min((c2 * scale + 32768) >> 16, 255);
            }
            const uint32_t h2 = fmix32(base ^ 0x68E31DA4u);
            const uint32_t h3 = fmix32(base ^ 0xB5297A4Du);
            c0 = min(max(c0 + (int)ntab[h2 & 0xFFFFu], 0), 255);
            c1 = min(max(c1 + (int)ntab[h2 >> 16], 0), 255);
            c2 = min(max(c2 + (int)ntab[h3 & 0xFFFFu], 0), 255);
            for (uint32_t m = rowhit; m; m &= m - 1) {
                const int32_t *ob = r + 4 + 8 * __builtin_ctz(m);
                const int px = ob[1], py = ob[2], a = ob[3], b = ob[4];
                bool in;
                if (ob[0] == 0) {
                    in = x >= px && x < px + a;
                } else if (x - px > a || px - x > a) {
                    in = false;
                } else {
                    const int64_t dx = (int64_t)(x - px) * b, dy = (int64_t)(y - py) * a;
                    const int64_t ab = (int64_t)a * b;
                    in = dx * dx + dy * dy <= ab * ab;
                }
                if (in) {
                    c0 = ob[5];
                    c1 = ob[6];
                    c2 = ob[7];
                }
            }
            const uint32_t v = (uint32_t)c0 | ((uint32_t)c1 << 8) | ((uint32_t)c2 << 16);
            // bytes 3p .. 3p+2 of the group
            const int b0 = 3 * p, k0 = b0 >> 2, s0 = (b0 & 3) * 8;   // constants once unrolled
            w[k0] |= v << s0;
            if (s0 > 8) w[k0 + 1] |= v >> (32 - s0);
        }
        if (++br == sc.block) {
            br = 0;
            ++bx;
        }
    }
    uint8_t *q = fo + (int64_t)y * sc.row_pitch + 48 * (int64_t)gx;
    if (nv == 16) {
        uint4 *q4 = reinterpret_cast<uint4 *>(q);
        q4[0] = make_uint4(w[0], w[1], w[2], w[3]);
        q4[1] = make_uint4(w[4], w[5], w[6], w[7]);
        q4[2] = make_uint4(w[8], w[9], w[10], w[11]);
    } else {
        for (int bidx = 0; bidx < 3 * nv; ++bidx) q[bidx] = (uint8_t)(w[bidx >> 2] >> ((bidx & 3) * 8));
    }
}

// One stream, several frames: blockIdx.y = frame of `recs`.
__global__ __launch_bounds__(256) void gen_kernel(StreamConst sc, const int32_t *__restrict__ recs, int n_frames,
                                                  const int16_t *__restrict__ ntab, uint8_t *__restrict__ out) {
    const int fi = blockIdx.y;
    if (fi >= n_frames) return;
    const int ngx = (sc.width + 15) / 16;
    const uint32_t groups = (uint32_t)sc.height * (uint32_t)ngx;
    const int32_t *r = recs + (int64_t)fi * kFrameInts;
    uint8_t *fo = out + (int64_t)fi * sc.frame_pitch;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += gridDim.x * blockDim.x) {
        const int y = (int)(g / (uint32_t)ngx);
        gen_group(sc, r, ntab, fo, y, (int)(g - (uint32_t)y * ngx));
    }
}

struct IngestJob {
    StreamConst sc;
    const int32_t *rec;
    uint8_t *out;
    int64_t g0;              // first 16-pixel group of this frame in the launch
};

constexpr int kGenBlock = 1024;
constexpr int64_t kGenLdsMinGroups = 1 << 19;   // about 8 Mpx: below, the direct kernel is quicker

// Frames of many streams, one job per blockIdx.y, noise looked up in HBM: for
// small batches, where filling an LDS table would cost more than it saves.
__global__ __launch_bounds__(256) void gen_jobs_kernel(const IngestJob *__restrict__ jobs, int n_jobs,
                                                       const int16_t *__restrict__ ntab) {
    const int j = blockIdx.y;
    if (j >= n_jobs) return;
    const IngestJob &job = jobs[j];
    const StreamConst sc = job.sc;
    const int ngx = (sc.width + 15) / 16;
    const uint32_t groups = (uint32_t)sc.height * (uint32_t)ngx;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += gridDim.x * blockDim.x) {
        const int y = (int)(g / (uint32_t)ngx);
        gen_group(sc, job.rec, ntab, job.out, y, (int)(g - (uint32_t)y * ngx));
    }
}

// Frames of many streams: their 16-pixel groups numbered end to end, equal
// runs per workgroup.  The noise table (|values| <= 127) is copied to LDS as
// bytes once per workgroup: its per-pixel lookups are scattered.
__global__ __launch_bounds__(kGenBlock) __attribute__((amdgpu_waves_per_eu(8))) void gen_batch_kernel(const IngestJob *__restrict__ jobs, int n_jobs,
                                                              int64_t n_groups, int64_t chunk,
                                                              const int16_t *__restrict__ ntab) {
    __shared__ int8_t nt[65536];
    for (int i = threadIdx.x; i < 65536; i += kGenBlock) nt[i] = (int8_t)ntab[i];
    __syncthreads();
    const int64_t gb = (int64_t)blockIdx.x * chunk;
    const int64_t ge = min(gb + chunk, n_groups);
    int j = -1;
    for (int64_t g = gb + threadIdx.x; g < ge; g += kGenBlock) {
        if (j < 0) {
            int lo = 0, hi = n_jobs - 1;      // last job whose first group is <= g
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].g0 <= g) lo = mid; else hi = mid - 1;
            }
            j = lo;
        }
        while (j + 1 < n_jobs && jobs[j + 1].g0 <= g) ++j;
        const IngestJob &job = jobs[j];
        const int ngx = (job.sc.width + 15) / 16;
        const uint32_t local = (uint32_t)(g - job.g0);
        const int y = (int)(local / (uint32_t)ngx);
        gen_group(job.sc, job.rec, nt, job.out, y, (int)(local - (uint32_t)y * ngx));
    }
}

struct IngestCtx {
    int n_streams;
    StreamConst *consts;         // host copy
    const int32_t *d_recs;       // device: all records
    int64_t *rec_base;           // host: first record of each stream
    int32_t *n_recs;             // host: records per stream
    const int16_t *d_ntab;
    IngestJob *h_jobs;           // pinned staging, one slot of kMaxJobs per in-flight batch
    IngestJob *d_jobs;
    hipEvent_t *slot_done;       // per slot: its last use has run on the device
    bool *slot_used;
    int slots, next_slot;
    int cus;
};

constexpr int kMaxJobs = 4096;

}  // namespace

// Matches obg_ingest_item of the serving API (stream, frame, device buffer).
struct SynthIngestItem {
    int32_t stream;
    int32_t frame;
    uint8_t *dst;
};

extern "C" void synth_ingest_destroy(void *ctx);

extern "C" void *synth_ingest_create(int32_t n_streams, const int32_t *params, const int32_t *d_recs,
                                     const int64_t *rec_base, const int32_t *n_recs, const int16_t *d_ntab,
                                     int32_t slots) {
    // params: per stream 12 int32: width, height, row_pitch, kp, kb, bthr, bimodal, period, block,
    // n_palette, pad, pad (pick thresholds are fixed)
    if (n_streams < 1 || !params || !d_recs || !rec_base || !n_recs || !d_ntab || slots < 1) return nullptr;
    IngestCtx *c = new IngestCtx();
    c->n_streams = n_streams;
    c->consts = new StreamConst[n_streams];
    c->rec_base = new int64_t[n_streams];
    c->n_recs = new int32_t[n_streams];
    for (int s = 0; s < n_streams; ++s) {
        const int32_t *p = params + 12 * s;
        StreamConst sc{p[0], p[1], p[2], (int64_t)p[1] * p[2], (uint32_t)p[3], (uint32_t)p[4], (uint32_t)p[5],
                       p[6], p[7], p[8], p[9], 45875u, 58982u, 63570u};
        c->consts[s] = sc;
        c->rec_base[s] = rec_base[s];
        c->n_recs[s] = n_recs[s];
    }
    c->d_recs = d_recs;
    c->d_ntab = d_ntab;
    c->slots = slots;
    c->next_slot = 0;
    c->slot_done = new hipEvent_t[slots]();
    c->slot_used = new bool[slots]();
    bool ok = hipHostMalloc((void **)&c->h_jobs, sizeof(IngestJob) * kMaxJobs * slots, hipHostMallocDefault) == hipSuccess &&
              hipMalloc((void **)&c->d_jobs, sizeof(IngestJob) * kMaxJobs * slots) == hipSuccess;
    for (int i = 0; ok && i < slots; ++i)
        ok = hipEventCreateWithFlags(&c->slot_done[i], hipEventDisableTiming) == hipSuccess;
    // the batch kernel keeps the noise table in LDS as bytes
    if (ok) {
        std::vector<int16_t> h(65536);
        ok = hipMemcpy(h.data(), d_ntab, 65536 * sizeof(int16_t), hipMemcpyDeviceToHost) == hipSuccess;
        for (int i = 0; ok && i < 65536; ++i) ok = h[i] >= -127 && h[i] <= 127;
    }
    c->cus = 256;
    int dev = 0, ncu = 0;
    if (ok && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        c->cus = ncu;
    if (!ok) {
        synth_ingest_destroy(c);
        return nullptr;
    }
    return c;
}

extern "C" void synth_ingest_destroy(void *ctx) {
    IngestCtx *c = (IngestCtx *)ctx;
    if (!c) return;
    for (int i = 0; i < c->slots; ++i)
        if (c->slot_done && c->slot_done[i]) {
            (void)hipEventSynchronize(c->slot_done[i]);
            (void)hipEventDestroy(c->slot_done[i]);
        }
    if (c->h_jobs) (void)hipHostFree(c->h_jobs);
    if (c->d_jobs) (void)hipFree(c->d_jobs);
    delete[] c->slot_done;
    delete[] c->slot_used;
    delete[] c->consts; delete[] c->rec_base; delete[] c->n_recs;
    delete c;
}

// Generate the listed frames into their device buffers, enqueued on `stream`.
// The staging slots rotate; before a slot is refilled, the host waits until
// the work of its previous use has run, so calls may finish in any order.
extern "C" int synth_ingest(void *ctx, const SynthIngestItem *items, int32_t n, hipStream_t stream) {
    IngestCtx *c = (IngestCtx *)ctx;
    if (!c || n < 0 || n > kMaxJobs) return -1;
    if (n == 0) return 0;
    const int slot = c->next_slot;
    c->next_slot = (c->next_slot + 1) % c->slots;
    if (c->slot_used[slot] && hipEventSynchronize(c->slot_done[slot]) != hipSuccess) return -3;
    IngestJob *hj = c->h_jobs + (size_t)slot * kMaxJobs;
    IngestJob *dj = c->d_jobs + (size_t)slot * kMaxJobs;
    int64_t n_groups = 0;
    for (int i = 0; i < n; ++i) {
        const int s = items[i].stream, f = items[i].frame;
        if (s < 0 || s >= c->n_streams || f < 0 || f >= c->n_recs[s] || !items[i].dst ||
            (uintptr_t)items[i].dst % 16 || c->consts[s].row_pitch % 16)
            return -1;
        hj[i].sc = c->consts[s];
        hj[i].rec = c->d_recs + (c->rec_base[s] + f) * kFrameInts;
        hj[i].out = items[i].dst;
        hj[i].g0 = n_groups;
        n_groups += (int64_t)hj[i].sc.height * ((hj[i].sc.width + 15) / 16);
    }
    if (hipMemcpyAsync(dj, hj, sizeof(IngestJob) * n, hipMemcpyHostToDevice, stream) != hipSuccess) return -3;
    if (n_groups < kGenLdsMinGroups) {
        int64_t most = 0;
        for (int i = 0; i < n; ++i) most = std::max<int64_t>(most, (int64_t)hj[i].sc.height * ((hj[i].sc.width + 15) / 16));
        const int gx = (int)std::min<int64_t>((most + 255) / 256, 1024);
        hipLaunchKernelGGL(gen_jobs_kernel, dim3(gx, n), dim3(256), 0, stream, (const IngestJob *)dj, n, c->d_ntab);
        if (hipGetLastError() != hipSuccess || hipEventRecord(c->slot_done[slot], stream) != hipSuccess) return -3;
        c->slot_used[slot] = true;
        return 0;
    }
    // equal runs of groups, at least 8 per thread, at most two workgroups per CU
    int64_t grid = std::min<int64_t>((n_groups + 8 * kGenBlock - 1) / (8 * kGenBlock), 2 * (int64_t)c->cus);
    grid = std::max<int64_t>(grid, 1);
    const int64_t chunk = (n_groups + grid - 1) / grid;
    grid = (n_groups + chunk - 1) / chunk;
    hipLaunchKernelGGL(gen_batch_kernel, dim3((unsigned)grid), dim3(kGenBlock), 0, stream, (const IngestJob *)dj, n,
                       n_groups, chunk, c->d_ntab);
    if (hipGetLastError() != hipSuccess || hipEventRecord(c->slot_done[slot], stream) != hipSuccess) return -3;
    c->slot_used[slot] = true;
    return 0;
}

extern "C" int synth_generate(int32_t width, int32_t height, int64_t row_pitch, int64_t frame_pitch,
                              uint32_t kp, uint32_t kb, uint32_t bthr, int32_t bimodal, int32_t period,
                              int32_t block, int32_t n_palette, uint32_t t0, uint32_t t1, uint32_t t2,
                              const int32_t *recs, int32_t n_frames, const int16_t *ntab, uint8_t *out,
                              hipStream_t stream) {
    if (width < 1 || height < 1 || n_frames < 0 || row_pitch < 3LL * width || frame_pitch < height * row_pitch)
        return -1;
    if (!recs || !ntab || !out || period < 1 || block < 1 || n_palette < 1) return -1;
    if (row_pitch % 16 || frame_pitch % 16 || (uintptr_t)out % 16) return -1;   // 16-byte stores
    if (n_frames == 0) return 0;
    if ((int64_t)width * height > 0xFFFFFFFFLL || n_frames > 65535) return -1;
    StreamConst sc{width, height, row_pitch, frame_pitch, kp, kb, bthr, bimodal, period, block, n_palette, t0, t1, t2};
    const int64_t groups = (int64_t)height * ((width + 15) / 16);
    int gx = (int)((groups + 255) / 256);
    if (gx > 4096) gx = 4096;
    hipLaunchKernelGGL(gen_kernel, dim3(gx, n_frames), dim3(256), 0, stream, sc, recs, n_frames, ntab, out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
