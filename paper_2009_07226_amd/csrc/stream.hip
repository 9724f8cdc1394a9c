// Slice streaming on one GPU: projection / backprojection of slice batches
// that live in host memory, in chunks whose host-to-device copies, SpMM and
// device-to-host copies run on three streams, so the copies of one chunk
// overlap the products of its neighbours (the single-GPU form of the
// paper's minibatch pipelining, Sec. III-A/III-D: slices move in batches
// while earlier batches are processed).
#include <algorithm>

#include "common.hpp"

namespace xct {

static size_t align256s(size_t b) { return (b + 255) & ~(size_t)255; }

struct StreamWs {
    char *in[2], *out[2];
    void *spmm;
};

// Two input and two output chunk buffers, then the SpMM workspace.
static size_t stream_ws_layout(const xct_matrix *m, int dir, int chunk, xct_dtype io, char *base, StreamWs *w) {
    const int64_t n_vol = (int64_t)m->n * m->n, n_sino = (int64_t)m->M * m->C;
    const int64_t n_in = dir ? n_sino : n_vol, n_out = dir ? n_vol : n_sino;
    const size_t in_b = align256s((size_t)chunk * n_in * elem_bytes(io));
    const size_t out_b = align256s((size_t)chunk * n_out * elem_bytes(io));
    if (w) {
        w->in[0] = base;
        w->in[1] = base + in_b;
        w->out[0] = base + 2 * in_b;
        w->out[1] = base + 2 * in_b + out_b;
        w->spmm = base + 2 * in_b + 2 * out_b;
    }
    return 2 * in_b + 2 * out_b + spmm_workspace(m, chunk);
}

static int streamed(const xct_matrix *m, int dir, const void *src_host, void *dst_host, int batch, int chunk,
                    xct_dtype io, void *workspace, void *compute, void *h2d, void *d2h) {
    if (!m || !src_host || !dst_host || !workspace) return fail(XCT_ERR_INVALID, "NULL argument");
    if (batch < 1) return fail(XCT_ERR_INVALID, "batch must be >= 1");
    if (chunk < 1) return fail(XCT_ERR_INVALID, "chunk must be >= 1");
    if (!valid_dtype(io)) return fail(XCT_ERR_INVALID, "bad io dtype");
    if (((uintptr_t)workspace & 255) != 0) return fail(XCT_ERR_INVALID, "workspace must be 256-byte aligned");
    chunk = std::min(chunk, batch);
    StreamWs w;
    stream_ws_layout(m, dir, chunk, io, (char *)workspace, &w);
    const int64_t n_vol = (int64_t)m->n * m->n, n_sino = (int64_t)m->M * m->C;
    const size_t in_slice = (size_t)(dir ? n_sino : n_vol) * elem_bytes(io);
    const size_t out_slice = (size_t)(dir ? n_vol : n_sino) * elem_bytes(io);
    hipStream_t sc = (hipStream_t)compute, si = (hipStream_t)h2d, so = (hipStream_t)d2h;
    // Any failure stops the enqueueing; the streams are then drained before
    // returning, so no copy into or out of the caller's buffers is left running.
    int rc = XCT_OK;
    auto chk = [&](hipError_t e, const char *what) -> bool {
        if (e != hipSuccess && rc == XCT_OK) rc = fail(XCT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
        return rc == XCT_OK;
    };
    // per buffer slot: input copied in (0, 1), product done (2, 3), output
    // copied out (4, 5); 6: the compute stream's earlier work.  The handle
    // keeps them from its first streamed call on.
    std::lock_guard<std::mutex> lock(const_cast<xct_matrix *>(m)->stream_mu);
    hipEvent_t *ev = const_cast<xct_matrix *>(m)->stream_ev;
    for (int q = 0; q < 7; ++q)
        if (!ev[q] && !chk(hipEventCreateWithFlags(&ev[q], hipEventDisableTiming), "hipEventCreateWithFlags"))
            return rc;
    // The workspace is ordered on the compute stream (its previous user may
    // still be running there): both copy streams start after that work.
    if (!chk(hipEventRecord(ev[6], sc), "hipEventRecord") ||
        !chk(hipStreamWaitEvent(si, ev[6], 0), "hipStreamWaitEvent") ||
        !chk(hipStreamWaitEvent(so, ev[6], 0), "hipStreamWaitEvent"))
        return rc;
    const int nc = (batch + chunk - 1) / chunk;
    auto slices = [&](int c) { return std::min(chunk, batch - c * chunk); };
    auto copy_in = [&](int c) -> bool {
        const int slot = c & 1;
        // the product of chunk c - 2 has finished reading this input buffer
        if (c >= 2 && !chk(hipStreamWaitEvent(si, ev[2 + slot], 0), "hipStreamWaitEvent")) return false;
        return chk(hipMemcpyAsync(w.in[slot], (const char *)src_host + (size_t)c * chunk * in_slice,
                                  (size_t)slices(c) * in_slice, hipMemcpyHostToDevice, si),
                   "hipMemcpyAsync") &&
               chk(hipEventRecord(ev[slot], si), "hipEventRecord");
    };
    copy_in(0);
    for (int c = 0; c < nc && rc == XCT_OK; ++c) {
        const int slot = c & 1;
        if (c + 1 < nc && !copy_in(c + 1)) break;
        if (!chk(hipStreamWaitEvent(sc, ev[slot], 0), "hipStreamWaitEvent")) break;
        // the copy-out of chunk c - 2 has finished reading this output buffer
        if (c >= 2 && !chk(hipStreamWaitEvent(sc, ev[4 + slot], 0), "hipStreamWaitEvent")) break;
        const int r = spmm_call(m, dir, w.in[slot], w.out[slot], slices(c), io, w.spmm, sc);
        if (r) {
            rc = r;
            break;
        }
        if (!chk(hipEventRecord(ev[2 + slot], sc), "hipEventRecord") ||
            !chk(hipStreamWaitEvent(so, ev[2 + slot], 0), "hipStreamWaitEvent") ||
            !chk(hipMemcpyAsync((char *)dst_host + (size_t)c * chunk * out_slice, w.out[slot],
                                (size_t)slices(c) * out_slice, hipMemcpyDeviceToHost, so),
                 "hipMemcpyAsync") ||
            !chk(hipEventRecord(ev[4 + slot], so), "hipEventRecord"))
            break;
    }
    // everything enqueued completes before the events are released
    chk(hipStreamSynchronize(so), "hipStreamSynchronize");
    chk(hipStreamSynchronize(sc), "hipStreamSynchronize");
    chk(hipStreamSynchronize(si), "hipStreamSynchronize");
    return rc;
}

}  // namespace xct

using namespace xct;

extern "C" size_t xct_stream_workspace_bytes(const xct_matrix *m, int which, int chunk, xct_dtype io) {
    if (!m || (which != 0 && which != 1) || chunk < 1 || !valid_dtype(io)) return 0;
    return stream_ws_layout(m, which, chunk, io, nullptr, nullptr);
}

extern "C" int xct_project_streamed(const xct_matrix *m, const void *x_host, void *y_host, int batch, int chunk,
                                    xct_dtype io, void *workspace, void *compute_stream, void *h2d_stream,
                                    void *d2h_stream) {
    return streamed(m, 0, x_host, y_host, batch, chunk, io, workspace, compute_stream, h2d_stream, d2h_stream);
}

extern "C" int xct_backproject_streamed(const xct_matrix *m, const void *y_host, void *x_host, int batch, int chunk,
                                        xct_dtype io, void *workspace, void *compute_stream, void *h2d_stream,
                                        void *d2h_stream) {
    return streamed(m, 1, y_host, x_host, batch, chunk, io, workspace, compute_stream, h2d_stream, d2h_stream);
}
