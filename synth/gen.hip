// gen.hip -- the synthetic streams of frames.py, one thread per pixel on the
// GPU.  Same hash (MurmurHash3 fmix32), same palette, drift, bimodal pixels,
// noise table and foreground objects; frames.py computes the per-frame
// numbers (frame hash, drift scale, object positions) and this kernel only
// evaluates the per-pixel integer formula, so both give identical bytes.
// Inputs only: none of the method's arithmetic is here.
#include <hip/hip_runtime.h>
#include <stdint.h>

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
__global__ void gen_kernel(StreamConst sc, const int32_t *__restrict__ recs, int n_frames,
                           const int16_t *__restrict__ ntab, uint8_t *__restrict__ out) {
    const int64_t npx = (int64_t)sc.width * sc.height;
    const int fi = blockIdx.y;
    if (fi >= n_frames) return;
    const int32_t *r = recs + (int64_t)fi * kFrameInts;
    const int f = r[0];
    const uint32_t hf = (uint32_t)r[1];
    const int32_t scale = r[2];
    const int nobj = r[3];
    uint8_t *fo = out + (int64_t)fi * sc.frame_pitch;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npx; p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / sc.width), x = (int)(p - (int64_t)y * sc.width);
        const uint32_t pix = (uint32_t)p;
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
        const int nbx = (sc.width + sc.block - 1) / sc.block;
        const uint32_t idx = (uint32_t)(((y / sc.block) * nbx + x / sc.block) * sc.n_palette) + ci;
        uint32_t h = fmix32(idx ^ sc.kp);
        h = fmix32(h + 0x632BE5ABu);
        int c[3] = {(int)(h & 255u), (int)((h >> 8) & 255u), (int)((h >> 16) & 255u)};
        if (scale != 65536) {
            for (int k = 0; k < 3; ++k) {
                const int64_t v = ((int64_t)c[k] * scale + 32768) >> 16;
                c[k] = (int)(v > 255 ? 255 : v);
            }
        }
        const uint32_t h2 = fmix32(base ^ 0x68E31DA4u);
        const uint32_t h3 = fmix32(base ^ 0xB5297A4Du);
        const int n[3] = {ntab[h2 & 0xFFFFu], ntab[h2 >> 16], ntab[h3 & 0xFFFFu]};
        for (int k = 0; k < 3; ++k) {
            int v = c[k] + n[k];
            c[k] = v < 0 ? 0 : (v > 255 ? 255 : v);
        }
        for (int o = 0; o < nobj; ++o) {
            const int32_t *ob = r + 4 + 8 * o;
            const int64_t px = ob[1], py = ob[2], a = ob[3], b = ob[4];
            bool in;
            if (ob[0] == 0) {
                in = x >= px && x < px + a && y >= py && y < py + b;
            } else {
                const int64_t dx = (x - px) * b, dy = (y - py) * a;
                in = dx * dx + dy * dy <= (a * b) * (a * b);
            }
            if (in) { c[0] = ob[5]; c[1] = ob[6]; c[2] = ob[7]; }
        }
        uint8_t *q = fo + (int64_t)y * sc.row_pitch + 3 * x;
        q[0] = (uint8_t)c[0];
        q[1] = (uint8_t)c[1];
        q[2] = (uint8_t)c[2];
    }
}

// One frame of a batch of frames from many streams.
struct IngestJob {
    StreamConst sc;
    const int32_t *rec;
    uint8_t *out;
};

__global__ void gen_batch_kernel(const IngestJob *__restrict__ jobs, int n_jobs, const int16_t *__restrict__ ntab) {
    const int j = blockIdx.y;
    if (j >= n_jobs) return;
    const IngestJob job = jobs[j];
    const StreamConst &sc = job.sc;
    const int64_t npx = (int64_t)sc.width * sc.height;
    const int32_t *r = job.rec;
    const int f = r[0];
    const uint32_t hf = (uint32_t)r[1];
    const int32_t scale = r[2];
    const int nobj = r[3];
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npx; p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / sc.width), x = (int)(p - (int64_t)y * sc.width);
        const uint32_t pix = (uint32_t)p;
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
        const int nbx = (sc.width + sc.block - 1) / sc.block;
        const uint32_t idx = (uint32_t)(((y / sc.block) * nbx + x / sc.block) * sc.n_palette) + ci;
        uint32_t h = fmix32(idx ^ sc.kp);
        h = fmix32(h + 0x632BE5ABu);
        int c[3] = {(int)(h & 255u), (int)((h >> 8) & 255u), (int)((h >> 16) & 255u)};
        if (scale != 65536) {
            for (int k = 0; k < 3; ++k) {
                const int64_t v = ((int64_t)c[k] * scale + 32768) >> 16;
                c[k] = (int)(v > 255 ? 255 : v);
            }
        }
        const uint32_t h2 = fmix32(base ^ 0x68E31DA4u);
        const uint32_t h3 = fmix32(base ^ 0xB5297A4Du);
        const int n[3] = {ntab[h2 & 0xFFFFu], ntab[h2 >> 16], ntab[h3 & 0xFFFFu]};
        for (int k = 0; k < 3; ++k) {
            int v = c[k] + n[k];
            c[k] = v < 0 ? 0 : (v > 255 ? 255 : v);
        }
        for (int o = 0; o < nobj; ++o) {
            const int32_t *ob = r + 4 + 8 * o;
            const int64_t px = ob[1], py = ob[2], a = ob[3], b = ob[4];
            bool in;
            if (ob[0] == 0) {
                in = x >= px && x < px + a && y >= py && y < py + b;
            } else {
                const int64_t dx = (x - px) * b, dy = (y - py) * a;
                in = dx * dx + dy * dy <= (a * b) * (a * b);
            }
            if (in) { c[0] = ob[5]; c[1] = ob[6]; c[2] = ob[7]; }
        }
        uint8_t *q = job.out + (int64_t)y * sc.row_pitch + 3 * x;
        q[0] = (uint8_t)c[0];
        q[1] = (uint8_t)c[1];
        q[2] = (uint8_t)c[2];
    }
}

// Ingest context for a serving run: every stream's constants and the frame
// records of every frame that may arrive, resident on the device.
struct IngestCtx {
    int n_streams;
    StreamConst *consts;         // host copy
    const int32_t *d_recs;       // device: all records
    int64_t *rec_base;           // host: first record of each stream
    int32_t *n_recs;             // host: records per stream
    const int16_t *d_ntab;
    IngestJob *h_jobs;           // pinned staging, one slot of kMaxJobs per in-flight batch
    IngestJob *d_jobs;
    int slots, next_slot;
};

constexpr int kMaxJobs = 4096;

}  // namespace

// Matches obg_ingest_item of the serving API (stream, frame, device buffer).
struct SynthIngestItem {
    int32_t stream;
    int32_t frame;
    uint8_t *dst;
};

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
    if (hipHostMalloc((void **)&c->h_jobs, sizeof(IngestJob) * kMaxJobs * slots, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&c->d_jobs, sizeof(IngestJob) * kMaxJobs * slots) != hipSuccess) {
        delete[] c->consts; delete[] c->rec_base; delete[] c->n_recs; delete c;
        return nullptr;
    }
    return c;
}

extern "C" void synth_ingest_destroy(void *ctx) {
    IngestCtx *c = (IngestCtx *)ctx;
    if (!c) return;
    hipHostFree(c->h_jobs);
    hipFree(c->d_jobs);
    delete[] c->consts; delete[] c->rec_base; delete[] c->n_recs;
    delete c;
}

// Generate the listed frames into their device buffers, enqueued on `stream`.
// The staging slots rotate; a slot is reused only after `slots` later calls,
// so the caller keeps at most `slots` calls in flight.
extern "C" int synth_ingest(void *ctx, const SynthIngestItem *items, int32_t n, hipStream_t stream) {
    IngestCtx *c = (IngestCtx *)ctx;
    if (!c || n < 0 || n > kMaxJobs) return -1;
    if (n == 0) return 0;
    const int slot = c->next_slot;
    c->next_slot = (c->next_slot + 1) % c->slots;
    IngestJob *hj = c->h_jobs + (size_t)slot * kMaxJobs;
    IngestJob *dj = c->d_jobs + (size_t)slot * kMaxJobs;
    int64_t maxpx = 0;
    for (int i = 0; i < n; ++i) {
        const int s = items[i].stream, f = items[i].frame;
        if (s < 0 || s >= c->n_streams || f < 0 || f >= c->n_recs[s] || !items[i].dst) return -1;
        hj[i].sc = c->consts[s];
        hj[i].rec = c->d_recs + (c->rec_base[s] + f) * kFrameInts;
        hj[i].out = items[i].dst;
        const int64_t px = (int64_t)hj[i].sc.width * hj[i].sc.height;
        if (px > maxpx) maxpx = px;
    }
    if (hipMemcpyAsync(dj, hj, sizeof(IngestJob) * n, hipMemcpyHostToDevice, stream) != hipSuccess) return -3;
    int gx = (int)((maxpx + 255) / 256);
    if (gx > 1024) gx = 1024;
    hipLaunchKernelGGL(gen_batch_kernel, dim3(gx, n), dim3(256), 0, stream, (const IngestJob *)dj, n, c->d_ntab);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

extern "C" int synth_generate(int32_t width, int32_t height, int64_t row_pitch, int64_t frame_pitch,
                              uint32_t kp, uint32_t kb, uint32_t bthr, int32_t bimodal, int32_t period,
                              int32_t block, int32_t n_palette, uint32_t t0, uint32_t t1, uint32_t t2,
                              const int32_t *recs, int32_t n_frames, const int16_t *ntab, uint8_t *out,
                              hipStream_t stream) {
    if (width < 1 || height < 1 || n_frames < 0 || row_pitch < 3LL * width || frame_pitch < height * row_pitch)
        return -1;
    if (!recs || !ntab || !out || period < 1 || block < 1 || n_palette < 1) return -1;
    if (n_frames == 0) return 0;
    if ((int64_t)width * height > 0xFFFFFFFFLL || n_frames > 65535) return -1;
    StreamConst sc{width, height, row_pitch, frame_pitch, kp, kb, bthr, bimodal, period, block, n_palette, t0, t1, t2};
    const int64_t npx = (int64_t)width * height;
    int gx = (int)((npx + 255) / 256);
    if (gx > 4096) gx = 4096;
    hipLaunchKernelGGL(gen_kernel, dim3(gx, n_frames), dim3(256), 0, stream, sc, recs, n_frames, ntab, out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
