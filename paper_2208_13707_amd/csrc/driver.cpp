// Native multi-threaded program runner (see include/mpixs_driver.h).
#include <hip/hip_runtime.h>

#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "../../include/mpixs_driver.h"

namespace {

using clk = std::chrono::steady_clock;

struct ThreadOut {
    clk::time_point start, end, enq_end;
    int err = 0;
    int64_t err_op = -1;
    std::vector<hipEvent_t> marks;
};

int run_ops(const mpixs_drv_thread &t, int mode, std::vector<mpixs_request> &reqs,
            ThreadOut &out) {
    hipStream_t hs = static_cast<hipStream_t>(t.hip_stream);
    for (int64_t i = 0; i < t.nops; ++i) {
        const mpixs_drv_op &o = t.ops[i];
        mpixs_comm c = (o.comm >= 0 && o.comm < t.ncomms) ? t.comms[o.comm] : nullptr;
        int rc = MPIXS_SUCCESS;
        switch (o.kind) {
        case MPIXS_DRV_SEND:
            rc = mode ? mpixs_send(reinterpret_cast<const void *>(o.buf), o.count, o.datatype,
                                   o.peer, o.tag, c)
                      : mpixs_send_enqueue(reinterpret_cast<const void *>(o.buf), o.count,
                                           o.datatype, o.peer, o.tag, c);
            break;
        case MPIXS_DRV_ISEND:
            rc = mpixs_isend_enqueue(reinterpret_cast<const void *>(o.buf), o.count, o.datatype,
                                     o.peer, o.tag, c, &reqs[size_t(o.req)]);
            break;
        case MPIXS_DRV_RECV:
            rc = mode ? mpixs_recv(reinterpret_cast<void *>(o.buf), o.count, o.datatype, o.peer,
                                   o.tag, c, reinterpret_cast<mpixs_status *>(o.status))
                      : mpixs_recv_enqueue(reinterpret_cast<void *>(o.buf), o.count, o.datatype,
                                           o.peer, o.tag, c,
                                           reinterpret_cast<mpixs_status *>(o.status));
            break;
        case MPIXS_DRV_IRECV:
            rc = mpixs_irecv_enqueue(reinterpret_cast<void *>(o.buf), o.count, o.datatype, o.peer,
                                     o.tag, c, &reqs[size_t(o.req)]);
            break;
        case MPIXS_DRV_WAITALL:
            rc = mpixs_waitall_enqueue(o.nreq, &reqs[size_t(o.req)],
                                       reinterpret_cast<mpixs_status *>(o.status));
            break;
        case MPIXS_DRV_ALLREDUCE: {
            const void *sb = o.buf == 1 ? MPIXS_IN_PLACE : reinterpret_cast<const void *>(o.buf);
            rc = mode ? mpixs_allreduce(sb, reinterpret_cast<void *>(o.buf2), o.count, o.datatype,
                                        o.op, c)
                      : mpixs_allreduce_enqueue(sb, reinterpret_cast<void *>(o.buf2), o.count,
                                                o.datatype, o.op, c);
            break;
        }
        case MPIXS_DRV_GROUP_START: rc = mpixs_group_start(c); break;
        case MPIXS_DRV_GROUP_END: rc = mpixs_group_end(c); break;
        case MPIXS_DRV_STREAM_SEND:
            rc = mpixs_stream_send_enqueue(reinterpret_cast<const void *>(o.buf), o.count,
                                           o.datatype, o.peer, o.tag, c, o.op, o.pad);
            break;
        case MPIXS_DRV_STREAM_ISEND:
            rc = mpixs_stream_isend_enqueue(reinterpret_cast<const void *>(o.buf), o.count,
                                            o.datatype, o.peer, o.tag, c, o.op, o.pad,
                                            &reqs[size_t(o.req)]);
            break;
        case MPIXS_DRV_STREAM_RECV:
            rc = mpixs_stream_recv_enqueue(reinterpret_cast<void *>(o.buf), o.count, o.datatype,
                                           o.peer, o.tag, c, o.op, o.pad,
                                           reinterpret_cast<mpixs_status *>(o.status));
            break;
        case MPIXS_DRV_STREAM_IRECV:
            rc = mpixs_stream_irecv_enqueue(reinterpret_cast<void *>(o.buf), o.count, o.datatype,
                                            o.peer, o.tag, c, o.op, o.pad, &reqs[size_t(o.req)]);
            break;
        case MPIXS_DRV_GROUP_INIT:
        case MPIXS_DRV_GROUP_INIT_STATIC:
        case MPIXS_DRV_BATCH_START:
        case MPIXS_DRV_BATCH_FREE:
            if (!t.batches || o.req < 0 || o.req >= t.nbatches) {
                rc = MPIXS_ERR_ARG;
            } else if (o.kind == MPIXS_DRV_GROUP_INIT) {
                rc = mpixs_group_end_init(c, &t.batches[o.req]);
            } else if (o.kind == MPIXS_DRV_GROUP_INIT_STATIC) {
                rc = mpixs_group_end_init_static(c, &t.batches[o.req]);
            } else if (o.kind == MPIXS_DRV_BATCH_START) {
                rc = mpixs_batch_start_enqueue(t.batches[o.req]);
            } else {
                rc = mpixs_batch_free(&t.batches[o.req]);
            }
            break;
        case MPIXS_DRV_MARK:
            if (o.req >= 0 && size_t(o.req) < out.marks.size())
                rc = hipEventRecord(out.marks[size_t(o.req)], hs) == hipSuccess ? 0 : MPIXS_ERR_GPU;
            break;
        default: rc = MPIXS_ERR_ARG;
        }
        if (rc) {
            out.err = rc;
            out.err_op = i;
            return rc;
        }
    }
    return MPIXS_SUCCESS;
}

}  // namespace

extern "C" int mpixs_drv_run(mpixs_world world, int nthreads, const mpixs_drv_thread *threads,
                             int mode, mpixs_drv_result *result, double *marks_ms) {
    if (!world || nthreads <= 0 || !threads || !result) return MPIXS_ERR_ARG;
    for (int i = 0; i < nthreads; ++i)
        if (threads[i].ncomms < 0 || threads[i].ncomms > 16) return MPIXS_ERR_ARG;
    std::vector<ThreadOut> outs(static_cast<size_t>(nthreads));
    int max_marks = 0;
    for (int i = 0; i < nthreads; ++i) {
        max_marks = std::max(max_marks, threads[i].nmarks);
        outs[size_t(i)].marks.resize(size_t(std::max(threads[i].nmarks, 0)));
        for (auto &e : outs[size_t(i)].marks)
            if (hipEventCreate(&e) != hipSuccess) return MPIXS_ERR_GPU;
    }
    std::atomic<int> ready{0};
    std::atomic<int> go{0};
    clk::time_point t_go;
    std::vector<std::thread> th;
    th.reserve(size_t(nthreads));
    for (int i = 0; i < nthreads; ++i) {
        th.emplace_back([&, i] {
            const mpixs_drv_thread &t = threads[i];
            ThreadOut &out = outs[size_t(i)];
            std::vector<mpixs_request> reqs(size_t(std::max(t.max_reqs, 1)), nullptr);
            ready.fetch_add(1);
            while (!go.load(std::memory_order_acquire)) _mm_pause();
            out.start = clk::now();
            if (run_ops(t, mode, reqs, out)) mpixs_world_abort(world);
            out.enq_end = clk::now();
            if (hipStreamSynchronize(static_cast<hipStream_t>(t.hip_stream)) != hipSuccess &&
                !out.err)
                out.err = MPIXS_ERR_GPU;
            out.end = clk::now();
        });
    }
    while (ready.load() < nthreads) std::this_thread::yield();
    t_go = clk::now();
    go.store(1, std::memory_order_release);
    for (auto &x : th) x.join();
    clk::time_point end = t_go, enq_end = t_go;
    result->first_error = 0;
    result->error_thread = -1;
    result->error_op = -1;
    for (int i = 0; i < nthreads; ++i) {
        end = std::max(end, outs[size_t(i)].end);
        enq_end = std::max(enq_end, outs[size_t(i)].enq_end);
        if (outs[size_t(i)].err && !result->first_error) {
            result->first_error = outs[size_t(i)].err;
            result->error_thread = i;
            result->error_op = outs[size_t(i)].err_op;
        }
    }
    result->seconds = std::chrono::duration<double>(end - t_go).count();
    result->enqueue_seconds = std::chrono::duration<double>(enq_end - t_go).count();
    if (marks_ms && max_marks > 0 && !outs[0].marks.empty()) {
        for (int i = 0; i < nthreads; ++i) {
            for (int m = 0; m < max_marks; ++m) {
                double v = -1;
                if (size_t(m) < outs[size_t(i)].marks.size()) {
                    float ms = 0;
                    if (hipEventElapsedTime(&ms, outs[0].marks[0], outs[size_t(i)].marks[size_t(m)]) ==
                        hipSuccess)
                        v = ms;
                }
                marks_ms[size_t(i) * size_t(max_marks) + size_t(m)] = v;
            }
        }
    }
    for (auto &o : outs)
        for (auto &e : o.marks) (void)hipEventDestroy(e);
    return result->first_error;
}
