// Host-to-device copies out of pageable home buffers.
//
// A host-backed array may live in pageable memory (the caller's own buffer).
// The copy engine cannot read pageable memory directly; hipMemcpy*Async then
// stages it through the runtime's buffers, copying on the issuing thread and
// holding the copy engine meanwhile.  Here the box is instead packed by a
// small pool of host threads into a ring of pinned bounce buffers, and each
// buffer goes to the device with an ordinary asynchronous copy on the H2D
// stream.  Packing the next piece overlaps the copy of the previous one; a
// bounce buffer is reused once the event recorded after its copy has fired.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "lt_internal.h"

namespace lt {

// Runs fn(0) .. fn(parts - 1) on the pool's threads and the caller's, and
// returns when all are done.
class HostPool {
   public:
    explicit HostPool(int n) {
        for (int i = 0; i < n; ++i) threads_.emplace_back([this] { loop(); });
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : threads_) t.join();
    }
    void run(int parts, const std::function<void(int)> &fn) {
        {
            std::lock_guard<std::mutex> g(mu_);
            fn_ = &fn;
            parts_ = parts;
            next_ = 0;
            done_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> l(mu_);
        done_cv_.wait(l, [this] { return done_ == parts_; });
        fn_ = nullptr;
    }

   private:
    void work() {
        for (;;) {
            int i;
            const std::function<void(int)> *fn;
            {
                std::lock_guard<std::mutex> g(mu_);
                if (!fn_ || next_ >= parts_) return;
                i = next_++;
                fn = fn_;
            }
            (*fn)(i);
            std::lock_guard<std::mutex> g(mu_);
            if (++done_ == parts_) done_cv_.notify_all();
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> l(mu_);
                cv_.wait(l, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            work();
        }
    }
    std::vector<std::thread> threads_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *fn_ = nullptr;
    int parts_ = 0, next_ = 0, done_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

struct BounceRing {
    struct Buf {
        char *p = nullptr;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    std::vector<Buf> bufs;
    int next = 0;
    HostPool pool{BOUNCE_THREADS - 1};
};

void bounce_release(Ctx *ctx) {
    BounceRing *r = ctx->bounce;
    if (!r) return;
    for (auto &b : r->bufs) {
        if (b.ev) {
            (void)hipEventSynchronize(b.ev);
            (void)hipEventDestroy(b.ev);
        }
        if (b.p) (void)hipHostFree(b.p);
    }
    delete r;
    ctx->bounce = nullptr;
}

static lt_status ring_get(Ctx *ctx, BounceRing::Buf **out) {
    if (!ctx->bounce) {
        ctx->bounce = new BounceRing();
        ctx->bounce->bufs.reserve(BOUNCE_BUFS);  // entries never move
    }
    BounceRing &r = *ctx->bounce;
    if ((int)r.bufs.size() < BOUNCE_BUFS) {
        BounceRing::Buf b;
        hipError_t e = hipHostMalloc((void **)&b.p, BOUNCE_BYTES, hipHostMallocDefault);
        if (e != hipSuccess) return set_err(ctx, LT_ERR_OOM, "pinned bounce buffer: %s", hipGetErrorString(e));
        e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipHostFree(b.p);
            return hip_fail(ctx, e, "hipEventCreate(bounce)");
        }
        r.bufs.push_back(b);
        *out = &r.bufs.back();
        return LT_OK;
    }
    BounceRing::Buf &b = r.bufs[r.next];
    r.next = (r.next + 1) % BOUNCE_BUFS;
    if (b.pending) {
        // its previous copy must have read it
        hipError_t e = hipEventSynchronize(b.ev);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize(bounce)");
        b.pending = false;
    }
    *out = &b;
    return LT_OK;
}

lt_status bounce_h2d(Ctx *ctx, int stream, char *dst, const int64_t *ds, const char *src, const int64_t *ss,
                     const int64_t *ext, int nd, int esz) {
    // merge axes contiguous on both sides (outermost first afterwards), as
    // copy_box does
    int64_t e[MAXD], d[MAXD], s[MAXD];
    int n = 0;
    for (int a = nd - 1; a >= 0; --a) {
        if (ext[a] <= 0) return LT_OK;
        if (n > 0 && ds[a] == e[n - 1] * d[n - 1] && ss[a] == e[n - 1] * s[n - 1]) {
            e[n - 1] *= ext[a];
            continue;
        }
        e[n] = ext[a];
        d[n] = ds[a];
        s[n] = ss[a];
        ++n;
    }
    for (int i = 0; i < n / 2; ++i) {
        std::swap(e[i], e[n - 1 - i]);
        std::swap(d[i], d[n - 1 - i]);
        std::swap(s[i], s[n - 1 - i]);
    }
    const int64_t width = e[n - 1] * esz;  // bytes per row
    // rows: (plane, row) pairs of the outer axes, planes outermost
    const int64_t rows_per_plane = n >= 2 ? e[n - 2] : 1;
    const int64_t planes = n == 3 ? e[0] : 1;
    if (n >= 2 && width > BOUNCE_BYTES)
        return copy_box(ctx, stream, dst, ds, src, ss, ext, nd, esz, hipMemcpyHostToDevice);
    int64_t total = 0;
    hipStream_t h = ctx->streams[stream].h;
    for (int64_t pl = 0; pl < planes; ++pl) {
        const char *sp = src + (n == 3 ? pl * s[0] * esz : 0);
        char *dp = dst + (n == 3 ? pl * d[0] * esz : 0);
        const int64_t spitch = n >= 2 ? s[n - 2] * esz : 0, dpitch = n >= 2 ? d[n - 2] * esz : 0;
        // pieces: whole rows (n >= 2), or byte ranges of the one row (n == 1)
        const int64_t per = n >= 2 ? std::max<int64_t>(1, BOUNCE_BYTES / width) : BOUNCE_BYTES;
        const int64_t count = n >= 2 ? rows_per_plane : width;
        for (int64_t r0 = 0; r0 < count; r0 += per) {
            const int64_t r1 = std::min(count, r0 + per);
            BounceRing::Buf *b;
            lt_status st = ring_get(ctx, &b);
            if (st) return st;
            // pack on the pool: BOUNCE_THREADS parts of whole rows / bytes
            const int64_t units = r1 - r0;
            const int parts = (int)std::min<int64_t>(BOUNCE_THREADS, n >= 2 ? units : (units + 65535) / 65536);
            std::function<void(int)> pack = [&](int k) {
                const int64_t u0 = r0 + units * k / parts, u1 = r0 + units * (k + 1) / parts;
                if (n >= 2) {
                    for (int64_t r = u0; r < u1; ++r) memcpy(b->p + (r - r0) * width, sp + r * spitch, (size_t)width);
                } else {
                    memcpy(b->p + (u0 - r0), sp + u0, (size_t)(u1 - u0));
                }
            };
            ctx->bounce->pool.run(parts, pack);
            hipEvent_t pa = nullptr;
            st = prof_begin(ctx, stream, "copy_h2d", &pa);
            if (st) return st;
            hipError_t r;
            if (n >= 2)
                r = hipMemcpy2DAsync(dp + r0 * dpitch, dpitch, b->p, width, width, units, hipMemcpyHostToDevice, h);
            else
                r = hipMemcpyAsync(dp + r0, b->p, units, hipMemcpyHostToDevice, h);
            if (r != hipSuccess) return hip_fail(ctx, r, "hipMemcpyAsync(bounce)");
            st = prof_end(ctx, stream, "copy_h2d", pa);
            if (st) return st;
            r = hipEventRecord(b->ev, h);
            if (r != hipSuccess) return hip_fail(ctx, r, "hipEventRecord(bounce)");
            b->pending = true;
            total += n >= 2 ? units * width : units;
        }
    }
    ctx->stats.bytes_h2d += (uint64_t)total;
    ctx->stats.copies_h2d++;
    return LT_OK;
}

}  // namespace lt
