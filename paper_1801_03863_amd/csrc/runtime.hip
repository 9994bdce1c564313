// runtime.hip -- host side of the C ABI declared in include/lbm.h: parameter
// checks, device memory, the two population buffers, step launches (plain
// or replayed from a captured HIP graph), the launch-shape autotuner, status
// words and host read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "kernels.hpp"

#ifndef LBM_SOURCE_ID
#define LBM_SOURCE_ID "dev"
#endif

using lbm::DevStatus;
using lbm::Inst;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, const char *what = "")
{
    std::snprintf(g_err, sizeof(g_err), fmt, what);
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    std::snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
    return LBM_EHIP;
}

#define HIPCHK(expr)                                \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

constexpr int64_t kAlignElems = 64;  // plane alignment (elements)
// Single-lattice planes of at least 1 MiB carry a pad of 0..8 KiB after their
// nodes, chosen by the autotuner: the nine plane streams of a tile row start
// at offsets that differ by the plane stride, and a stride that is a large
// power of two puts them all on the same memory-channel offset.  Buffers
// are sized for the largest pad, so the pad can change in place.
constexpr int64_t kPadMinPlaneBytes = 1 << 20;
constexpr int32_t kPadMaxBytes = 8192;
constexpr int32_t kPadDefaultBytes = 2048;
constexpr int32_t kPadCandidates[] = {0, 1024, 2048, 4096, 8192};
constexpr int64_t kMaxBatchNodes = int64_t(1) << 22;
// D2Q9 rows are stored at a pitch of whole lines of this many bytes, so every
// row's first element starts a cache line: a row read by a wave then touches
// the fewest lines, and row writes fill whole lines.  Lattices of arbitrary
// width (a batch's instances) would otherwise start most rows mid-line.
constexpr int64_t kRowLineBytes = 128;

size_t elem_bytes(int precision)
{
    switch (precision) {
    case LBM_FP64: return 8;
    case LBM_FP32_NEWTON64:
    case LBM_FP32: return 4;
    case LBM_FP16DEV: return 2;
    default: return 0;
    }
}

int storage_of(int precision)
{
    switch (precision) {
    case LBM_FP64: return lbm::ST_F64;
    case LBM_FP32_NEWTON64: return lbm::ST_F32N64;
    case LBM_FP32: return lbm::ST_F32;
    default: return lbm::ST_F16DEV;
    }
}

// Row stride of an instance in elements: D2Q9 rows rounded up to whole
// lines of kRowLineBytes; a D1Q3 lattice is one row.
int64_t row_pitch(const lbm_params_t &q)
{
    if (q.lattice == LBM_D1Q3) return q.nx;
    const int64_t line = kRowLineBytes / (int64_t)elem_bytes(q.precision);
    return ((int64_t)q.nx + line - 1) / line * line;
}

int check_params(const lbm_params_t *p)
{
    if (!p) return fail(LBM_EINVAL, "null parameters");
    if (p->lattice != LBM_D1Q3 && p->lattice != LBM_D2Q9) return fail(LBM_EINVAL, "lattice must be D1Q3 or D2Q9");
    if (p->collision < LBM_MINXENT4 || p->collision > LBM_MRT) return fail(LBM_EINVAL, "unknown collision rule");
    if (p->bc < LBM_BC_PERIODIC || p->bc > LBM_BC_BOX) return fail(LBM_EINVAL, "unknown boundary kind");
    if (p->precision < LBM_FP64 || p->precision > LBM_FP16DEV) return fail(LBM_EINVAL, "unknown precision form");
    if (p->nx < 3) return fail(LBM_EINVAL, "nx must be >= 3");
    if (p->lattice == LBM_D2Q9 && p->ny < 3) return fail(LBM_EINVAL, "ny must be >= 3 for D2Q9");
    if (p->lattice == LBM_D1Q3 && p->ny != 1) return fail(LBM_EINVAL, "ny must be 1 for D1Q3");
    if ((int64_t)p->nx * (int64_t)p->ny > (int64_t)0x7fffffff / 2)
        return fail(LBM_EINVAL, "lattice too large for one instance (nx*ny must be < 2^30)");
    if (p->lattice == LBM_D2Q9 && row_pitch(*p) * (int64_t)p->ny > (int64_t)0x7fffffff)
        return fail(LBM_EINVAL, "lattice too large for one instance (its rows, stored at a pitch of whole "
                                "128-byte lines, must hold fewer than 2^31 elements)");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_EINVAL, "tau must be finite and > 1/2");
    if (p->tau2 > 0.0 && !(p->tau2 > 0.5 && std::isfinite(p->tau2)))
        return fail(LBM_EINVAL, "tau2 must be finite and > 1/2 (or <= 0 for the default)");
    if (!std::isfinite(p->u_lid)) return fail(LBM_EINVAL, "u_lid must be finite");
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return fail(LBM_EINVAL, "rho0 must be finite and > 0");
    if (p->fp16_exp < 0 || p->fp16_exp > 24) return fail(LBM_EINVAL, "fp16_exp must be in [0, 24]");
    if (p->reserved != 0) return fail(LBM_EINVAL, "reserved field must be 0");
    return LBM_OK;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Polynomial equilibrium in double (lid values handed to the kernels).
void feq9(double rho, double ux, double uy, double *out)
{
    static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    for (int a = 0; a < 9; ++a) {
        const double w = a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        const double cu = cx[a] * ux + cy[a] * uy;
        out[a] = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy));
    }
}

}  // namespace

struct lbm_ctx {
    lbm_params_t p{};
    int b = 9;
    int storage = 0;
    int batch = 0;
    int n = 1;
    std::vector<Inst> inst;
    std::vector<int64_t> node_prefix;  // host offsets of each instance's fields
    Inst *d_inst = nullptr;
    int32_t *d_tile_inst = nullptr;
    int32_t *d_tile_first = nullptr;
    int ntiles = 0;
    int tile_nodes = 0;  // nodes per tile of the current batched variant
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    char *buf[2] = {nullptr, nullptr};
    int cur = 0;
    size_t elem = 8;
    int64_t elems = 0;  // elements per buffer
    int64_t nodes = 0;
    int64_t steps_done = 0;
    DevStatus *d_status = nullptr;
    DevStatus *d_status_scratch = nullptr;
    int64_t *d_step_base = nullptr;
    bool base_synced = false;
    int variant = 0;
    int graph_chunk = 0;
    int32_t pad = -1;        // plane pad in bytes; -1: the context takes none
    int64_t plane_base = 0;  // plane length before the pad (elements)
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    float scale = 1.0f, iscale = 1.0f;
    std::string arch;
    int lds_variant = -1;  // batched D2Q9: index of the LDS-resident shape, -1 if it does not fit
    size_t lds_bytes = 0;
    int lds_block = 0;
};

namespace {

// Whether a single lattice of these parameters takes a plane pad.
bool paddable(const lbm_params_t &q, int batch)
{
    const int64_t elems = row_pitch(q) * (q.lattice == LBM_D1Q3 ? 1 : q.ny);
    return !batch && round_up(elems, kAlignElems) * (int64_t)elem_bytes(q.precision) >= kPadMinPlaneBytes;
}

int layout(const lbm_params_t *p, int32_t n, int batch, int b, std::vector<Inst> *inst, int64_t *elems,
           int64_t *nodes)
{
    int64_t off = 0, nn = 0;
    for (int i = 0; i < n; ++i) {
        const lbm_params_t &q = p[i];
        Inst in{};
        in.nx = q.nx;
        in.ny = q.lattice == LBM_D1Q3 ? 1 : q.ny;
        in.pitch = (int32_t)row_pitch(q);
        in.offset = off;
        in.stop = INT64_MAX;
        in.plane = round_up((int64_t)in.pitch * in.ny, kAlignElems);
        int64_t room = in.plane;  // elements reserved per plane
        if (paddable(q, batch)) {
            const int64_t eb = (int64_t)elem_bytes(q.precision);
            room = in.plane + kPadMaxBytes / eb;
            in.plane += kPadDefaultBytes / eb;
        }
        in.omega = 1.0 / q.tau;
        const double tau2 = (q.tau2 > 0.0) ? q.tau2 : (8.0 * q.tau - 1.0) / (2.0 * q.tau - 1.0);
        in.omega2 = 1.0 / tau2;
        in.u_lid = q.u_lid;
        in.rho0 = q.rho0;
        feq9(q.rho0, q.u_lid, 0.0, in.lid);
        off += b * room;
        nn += (int64_t)in.nx * in.ny;
        if (inst) inst->push_back(in);
    }
    *elems = off;
    *nodes = nn;
    return LBM_OK;
}

size_t buffer_bytes(int64_t elems, size_t elem) { return (size_t)round_up((int64_t)(elems * elem), 256); }

int check_batch(const lbm_params_t *p, int32_t n)
{
    if (!p || n < 1) return fail(LBM_EINVAL, "need at least one instance");
    for (int i = 0; i < n; ++i) {
        int rc = check_params(&p[i]);
        if (rc) return rc;
        if (p[i].lattice != p[0].lattice || p[i].collision != p[0].collision || p[i].bc != p[0].bc ||
            p[i].precision != p[0].precision || p[i].fp16_exp != p[0].fp16_exp)
            return fail(LBM_EINVAL, "batch instances must share lattice, collision, bc, precision and fp16_exp");
        if ((int64_t)p[i].nx * (p[i].lattice == LBM_D1Q3 ? 1 : p[i].ny) > kMaxBatchNodes)
            return fail(LBM_EINVAL, "batched instances are limited to 2^22 nodes each");
    }
    return LBM_OK;
}

int build_tiles(lbm_ctx *c, int tile_nodes)
{
    std::vector<int32_t> ti, tf;
    if (tile_nodes < 0) {
        // Two-step shapes: tiles of bx x rows nodes, row-major within each
        // instance, recorded as the tile's index ty * tiles_x + tx.
        const int bx = -tile_nodes / 4096, rows = -tile_nodes % 4096;
        for (int i = 0; i < c->n; ++i) {
            const int64_t nt = (int64_t)((c->inst[i].nx + bx - 1) / bx) * ((c->inst[i].ny + rows - 1) / rows);
            for (int64_t k = 0; k < nt; ++k) {
                ti.push_back(i);
                tf.push_back((int32_t)k);
            }
        }
    } else {
        for (int i = 0; i < c->n; ++i) {
            const int64_t nn = (int64_t)c->inst[i].nx * c->inst[i].ny;
            for (int64_t s = 0; s < nn; s += tile_nodes) {
                ti.push_back(i);
                tf.push_back((int32_t)s);
            }
        }
    }
    if (c->d_tile_inst) (void)hipFree(c->d_tile_inst);
    if (c->d_tile_first) (void)hipFree(c->d_tile_first);
    c->d_tile_inst = nullptr;
    c->d_tile_first = nullptr;
    c->ntiles = (int)ti.size();
    HIPCHK(hipMalloc(&c->d_tile_inst, ti.size() * sizeof(int32_t)));
    HIPCHK(hipMalloc(&c->d_tile_first, tf.size() * sizeof(int32_t)));
    HIPCHK(hipMemcpy(c->d_tile_inst, ti.data(), ti.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_tile_first, tf.data(), tf.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    c->tile_nodes = tile_nodes;
    return LBM_OK;
}


void drop_graphs(lbm_ctx *c)
{
    for (int k = 0; k < 2; ++k)
        if (c->gexec[k]) {
            (void)hipGraphExecDestroy(c->gexec[k]);
            c->gexec[k] = nullptr;
        }
}

// Move the state to a plane pad of `pad` bytes: each plane's nodes are
// copied from the current buffer into the other one at the new stride, which
// then becomes current (both buffers have room for the largest pad).
int set_pad(lbm_ctx *c, int32_t pad)
{
    if (pad == c->pad) return LBM_OK;
    if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
    else HIPCHK(hipDeviceSynchronize());
    drop_graphs(c);
    const int64_t eb = (int64_t)c->elem;
    const int64_t old_plane = c->inst[0].plane;
    const int64_t new_plane = c->plane_base + pad / eb;
    const size_t width = (size_t)c->inst[0].pitch * (size_t)c->inst[0].ny * (size_t)eb;
    const char *src = c->buf[c->cur];
    char *dst = c->buf[c->cur ^ 1];
    for (int q = 0; q < c->b; ++q)
        HIPCHK(hipMemcpyAsync(dst + q * new_plane * eb, src + q * old_plane * eb, width, hipMemcpyDeviceToDevice,
                              c->stream));
    if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
    else HIPCHK(hipDeviceSynchronize());
    c->cur ^= 1;
    c->inst[0].plane = new_plane;
    c->pad = pad;
    return LBM_OK;
}

lbm::StepArgs step_args(const lbm_ctx *c, DevStatus *status, int64_t step, const int64_t *base)
{
    lbm::StepArgs a{};
    a.inst = c->d_inst;
    a.one = c->inst[0];
    a.status = status;
    a.step_base = base;
    a.tile_inst = c->d_tile_inst;
    a.tile_first = c->d_tile_first;
    a.step = step;
    a.bc = c->p.bc;
    a.ntiles = c->ntiles;
    a.xcd_swizzle = 0;  // launch order; each launcher sets its own
    a.fp16_scale = c->scale;
    a.fp16_iscale = c->iscale;
    a.max_steps = 2;  // launchers of multi-step shapes set the count they need
    return a;
}

hipError_t launch_step(const lbm_ctx *c, int variant, const void *src, void *dst, const lbm::StepArgs &a,
                       hipStream_t s)
{
    if (c->b == 9) {
        if (c->batch) return lbm::launch_d2q9_batch_step(c->storage, c->p.collision, variant, src, dst, a, s);
        return lbm::launch_d2q9_step(c->storage, c->p.collision, variant, src, dst, a, s);
    }
    if (c->batch) return lbm::launch_d1q3_batch_step(c->storage, variant, src, dst, a, s);
    return lbm::launch_d1q3_step(c->storage, variant, src, dst, a, s);
}

// Steps one launch of shape v takes at most: 2 for the temporally blocked
// D2Q9 shapes, up to 256 for the K-step D1Q3 shapes, else 1.
int launch_steps(const lbm_ctx *c, int v)
{
    if (c->b != 9) return c->batch ? lbm::batch_variant_steps(3, v) : lbm::d1q3_variant_steps(v);
    if (c->batch) return v == c->lds_variant ? 1 : lbm::batch_variant_steps(9, v);
    return lbm::d2q9_variant_steps(c->p.collision, v);
}

// Launch `n` steps (at most the shape's steps per launch) of shape v from
// buf[cur]: the state ends in buf[cur ^ 1] whatever n is.
hipError_t launch_steps_from(const lbm_ctx *c, int v, int n, int cur, const lbm::StepArgs &a, hipStream_t s)
{
    lbm::StepArgs b = a;
    b.max_steps = n;
    return launch_step(c, v, c->buf[cur], c->buf[cur ^ 1], b, s);
}

// Launches that replay `steps` steps with shape v, which sets how often the
// two buffers swap.
int64_t launches_for(const lbm_ctx *c, int v, int64_t steps)
{
    const int64_t k = launch_steps(c, v);
    return (steps + k - 1) / k;
}

int variant_count(const lbm_ctx *c)
{
    if (c->batch) return lbm::batch_variant_count(c->b, c->p.collision) + (c->lds_variant >= 0 ? 1 : 0);
    return c->b == 9 ? lbm::d2q9_variant_count(c->p.collision) : lbm::d1q3_variant_count();
}

// LDS-resident batch: n steps in one launch; the state moves to
// buf[cur ^ (n & 1)] as with n single-step launches.
hipError_t launch_lds(lbm_ctx *c, DevStatus *status, int64_t step, int nsteps, int dst_parity_flip)
{
    lbm::StepArgs a = step_args(c, status, step, nullptr);
    a.ntiles = c->n;
    return lbm::launch_d2q9_lds(c->storage, c->p.collision, c->buf[c->cur], c->buf[c->cur ^ dst_parity_flip], a,
                                nsteps, c->lds_block, c->lds_bytes, c->stream);
}

int capture_graph(lbm_ctx *c, int parity)
{
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int cur = parity;
    hipError_t err = hipSuccess;
    const int spl = launch_steps(c, c->variant);
    for (int k = 0; k < c->graph_chunk && err == hipSuccess;) {
        const int n = std::min(spl, c->graph_chunk - k);
        lbm::StepArgs a = step_args(c, c->d_status, k, c->d_step_base);
        err = launch_steps_from(c, c->variant, n, cur, a, c->cap_stream);
        cur ^= 1;
        k += n;
    }
    if (err == hipSuccess) err = lbm::launch_add_step_base(c->d_step_base, c->graph_chunk, c->cap_stream);
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(err, "graph capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipError_t e3 = hipGraphInstantiate(&c->gexec[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return hip_fail(e3, "hipGraphInstantiate");
    return LBM_OK;
}

void destroy(lbm_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->d_status) (void)hipFree(c->d_status);
    if (c->d_status_scratch) (void)hipFree(c->d_status_scratch);
    if (c->d_step_base) (void)hipFree(c->d_step_base);
    if (c->d_inst) (void)hipFree(c->d_inst);
    if (c->d_tile_inst) (void)hipFree(c->d_tile_inst);
    if (c->d_tile_first) (void)hipFree(c->d_tile_first);
    delete c;
}

int check_device(std::string *arch)
{
    int dev = 0, count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) return fail(LBM_ENODEV, "no HIP device visible");
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    *arch = prop.gcnArchName;
    if (arch->find("gfx950") == std::string::npos)
        return fail(LBM_ENODEV, "device is %s; this library is built for gfx950 only", prop.gcnArchName);
    return LBM_OK;
}

// Upload the fields (or populations) of every instance and write the
// pre-shifted state into buf[cur].
int load_state(lbm_ctx *c, const double *rho, const double *ux, const double *uy, const double *f)
{
    const int64_t total = c->nodes;
    double *d = nullptr;
    const size_t per = f ? (size_t)c->b : 3;
    HIPCHK(hipMalloc(&d, sizeof(double) * per * (size_t)total));
    int rc = LBM_OK;
    hipError_t e = hipSuccess;
    if (f) {
        e = hipMemcpyAsync(d, f, sizeof(double) * per * total, hipMemcpyHostToDevice, c->stream);
    } else {
        e = hipMemcpyAsync(d, rho, sizeof(double) * total, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(d + total, ux, sizeof(double) * total, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && uy && c->b == 9)
            e = hipMemcpyAsync(d + 2 * total, uy, sizeof(double) * total, hipMemcpyHostToDevice, c->stream);
        else if (e == hipSuccess)
            e = hipMemsetAsync(d + 2 * total, 0, sizeof(double) * total, c->stream);
    }
    for (int i = 0; i < c->n && e == hipSuccess; ++i) {
        const int64_t o = c->node_prefix[i];
        if (f)
            e = lbm::launch_init(c->b, c->storage, c->inst[i], c->p.bc, nullptr, nullptr, nullptr, d + per * o,
                                 c->buf[c->cur], c->scale, c->stream);
        else
            e = lbm::launch_init(c->b, c->storage, c->inst[i], c->p.bc, d + o, d + total + o, d + 2 * total + o,
                                 nullptr, c->buf[c->cur], c->scale, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = hip_fail(e, "state upload");
    (void)hipFree(d);
    return rc;
}

int create(const lbm_params_t *p, int32_t n, int batch, const double *rho, const double *ux, const double *uy,
           void *ws, size_t ws_bytes, void *stream, lbm_ctx_t **out)
{
    if (!out) return fail(LBM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!rho || !ux) return fail(LBM_EINVAL, "rho and ux are required");
    if (p[0].lattice == LBM_D2Q9 && !uy) return fail(LBM_EINVAL, "uy is required for D2Q9");
    std::string arch;
    int rc = check_device(&arch);
    if (rc) return rc;
    lbm_ctx *c = new lbm_ctx();
    c->p = p[0];
    c->arch = arch;
    c->b = p[0].lattice == LBM_D1Q3 ? 3 : 9;
    c->storage = storage_of(p[0].precision);
    c->elem = elem_bytes(p[0].precision);
    c->batch = batch;
    c->n = n;
    c->stream = (hipStream_t)stream;
    const int k = p[0].fp16_exp ? p[0].fp16_exp : 14;
    c->scale = std::ldexp(1.0f, k);
    c->iscale = std::ldexp(1.0f, -k);
    layout(p, n, batch, c->b, &c->inst, &c->elems, &c->nodes);
    if (paddable(p[0], batch)) {
        c->pad = kPadDefaultBytes;
        c->plane_base = round_up((int64_t)c->inst[0].pitch * c->inst[0].ny, kAlignElems);
    }
    int64_t acc = 0;
    for (int i = 0; i < n; ++i) {
        c->node_prefix.push_back(acc);
        acc += (int64_t)c->inst[i].nx * c->inst[i].ny;
    }
    const size_t bb = buffer_bytes(c->elems, c->elem);
    if (ws) {
        if (ws_bytes < 2 * bb) {
            destroy(c);
            return fail(LBM_ENOMEM, "workspace too small");
        }
        if (((uintptr_t)ws & 255) != 0) {
            destroy(c);
            return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
        }
        c->ws = (char *)ws;
        c->ws_bytes = ws_bytes;
    } else {
        hipError_t e = hipMalloc(&c->ws, 2 * bb);
        if (e != hipSuccess) {
            destroy(c);
            return fail(LBM_ENOMEM, "hipMalloc of %s failed", "the population buffers");
        }
        c->own_ws = true;
        c->ws_bytes = 2 * bb;
    }
    c->buf[0] = c->ws;
    c->buf[1] = c->ws + bb;
#define CK(expr)                                   \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) {                    \
            int r_ = hip_fail(e_, #expr);          \
            destroy(c);                            \
            return r_;                             \
        }                                          \
    } while (0)
    CK(hipMalloc(&c->d_status, sizeof(DevStatus) * n));
    CK(hipMalloc(&c->d_status_scratch, sizeof(DevStatus) * n));
    CK(hipMalloc(&c->d_step_base, sizeof(int64_t)));
    if (batch && c->b == 9) {
        int64_t maxn = 0;
        for (int i = 0; i < n; ++i) maxn = std::max<int64_t>(maxn, (int64_t)c->inst[i].nx * c->inst[i].ny);
        int dev = 0, smem = 0;
        CK(hipGetDevice(&dev));
        CK(hipDeviceGetAttribute(&smem, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const size_t need = 2 * 9 * (size_t)maxn * c->elem;
        if (need <= (size_t)smem) {
            c->lds_variant = lbm::batch_variant_count(9, c->p.collision);
            c->lds_bytes = need;
            c->lds_block = (int)std::min<int64_t>(1024, std::max<int64_t>(64, (maxn + 63) / 64 * 64));
        }
    }
    if (batch) {
        CK(hipMalloc(&c->d_inst, sizeof(Inst) * n));
        CK(hipMemcpy(c->d_inst, c->inst.data(), sizeof(Inst) * n, hipMemcpyHostToDevice));
        rc = build_tiles(c, lbm::batch_tile_nodes(c->b, 0));
        if (rc) {
            destroy(c);
            return rc;
        }
    }
    CK(lbm::launch_clear_status(c->d_status, n, c->stream));
    CK(lbm::launch_clear_status(c->d_status_scratch, n, c->stream));
    CK(lbm::launch_set_step_base(c->d_step_base, 0, c->stream));
#undef CK
    rc = load_state(c, rho, ux, uy, nullptr);
    if (rc) {
        destroy(c);
        return rc;
    }
    *out = c;
    return LBM_OK;
}

// Device memory of the no-allocation entry point lbm_run_noalloc: a status
// record (the first 256 bytes) and the two population buffers of a lattice
// that fits.  Each GPU the library runs on holds its own copy until the
// process ends.  Host code never uses this name as an address: it takes the
// per-device address from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[LBM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current (after checking that the device is a
// gfx950, so later calls on it skip the property query).
int scratch_address(void **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_ENODEV, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        std::string arch;
        int rc = check_device(&arch);
        if (rc) return rc;
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(LBM_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace

extern "C" {

static int ws_bytes(const lbm_params_t *p, int32_t n, int batch, size_t *bytes)
{
    if (!bytes) return fail(LBM_EINVAL, "null output pointer");
    int64_t elems, nodes;
    layout(p, n, batch, p[0].lattice == LBM_D1Q3 ? 3 : 9, nullptr, &elems, &nodes);
    *bytes = 2 * buffer_bytes(elems, elem_bytes(p[0].precision));
    return LBM_OK;
}

int lbm_workspace_bytes(const lbm_params_t *p, size_t *bytes)
{
    int rc = check_params(p);
    if (rc) return rc;
    return ws_bytes(p, 1, 0, bytes);
}

int lbm_workspace_bytes_batch(const lbm_params_t *p, int32_t n, size_t *bytes)
{
    int rc = check_batch(p, n);
    if (rc) return rc;
    return ws_bytes(p, n, 1, bytes);
}

int lbm_init(const lbm_params_t *p, const double *rho, const double *ux, const double *uy, void *ws,
             size_t ws_bytes, void *stream, lbm_ctx_t **out)
{
    int rc = check_params(p);
    if (rc) return rc;
    return create(p, 1, 0, rho, ux, uy, ws, ws_bytes, stream, out);
}

int lbm_init_batch(const lbm_params_t *p, int32_t n, const double *rho, const double *ux, const double *uy,
                   void *ws, size_t ws_bytes, void *stream, lbm_ctx_t **out)
{
    int rc = check_batch(p, n);
    if (rc) return rc;
    return create(p, n, 1, rho, ux, uy, ws, ws_bytes, stream, out);
}

int lbm_step(lbm_ctx_t *c, int64_t nsteps)
{
    if (!c || nsteps < 0) return fail(LBM_EINVAL, "bad context or step count");
    if (c->batch && c->variant == c->lds_variant && c->lds_variant >= 0) {
        // Persistent LDS-resident shape: no graph needed, one launch per chunk.
        int64_t left = nsteps;
        while (left > 0) {
            const int chunk = (int)std::min<int64_t>(left, 1 << 20);
            HIPCHK(launch_lds(c, c->d_status, c->steps_done, chunk, chunk & 1));
            c->cur ^= chunk & 1;
            c->steps_done += chunk;
            left -= chunk;
        }
        c->base_synced = false;
        return LBM_OK;
    }
    int64_t i = 0;
    while (i < nsteps) {
        if (c->graph_chunk > 0 && nsteps - i >= c->graph_chunk) {
            if (!c->gexec[c->cur]) {
                int rc = capture_graph(c, c->cur);
                if (rc) return rc;
            }
            if (!c->base_synced) {
                HIPCHK(lbm::launch_set_step_base(c->d_step_base, c->steps_done, c->stream));
                c->base_synced = true;
            }
            HIPCHK(hipGraphLaunch(c->gexec[c->cur], c->stream));
            c->steps_done += c->graph_chunk;
            if (launches_for(c, c->variant, c->graph_chunk) & 1) c->cur ^= 1;
            i += c->graph_chunk;
            continue;
        }
        const int n = (int)std::min<int64_t>(launch_steps(c, c->variant), nsteps - i);
        lbm::StepArgs a = step_args(c, c->d_status, c->steps_done, nullptr);
        HIPCHK(launch_steps_from(c, c->variant, n, c->cur, a, c->stream));
        c->cur ^= 1;
        c->steps_done += n;
        c->base_synced = false;
        i += n;
    }
    return LBM_OK;
}

int lbm_set_graph_chunk(lbm_ctx_t *c, int32_t chunk)
{
    if (!c || chunk < 0) return fail(LBM_EINVAL, "bad context or chunk");
    if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->graph_chunk = chunk;
    c->base_synced = false;
    return LBM_OK;
}

int lbm_set_variant(lbm_ctx_t *c, int32_t v)
{
    if (!c || v < 0 || v >= variant_count(c)) return fail(LBM_EINVAL, "launch shape index out of range");
    if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
    else HIPCHK(hipDeviceSynchronize());
    drop_graphs(c);
    if (!c->batch && c->b == 9) HIPCHK(lbm::prepare_d2q9_variant(c->storage, c->p.collision, v));
    if (c->batch && c->b == 9 && v != c->lds_variant)
        HIPCHK(lbm::prepare_batch_variant(c->storage, c->p.collision, v));
    if (c->b == 3) HIPCHK(lbm::prepare_d1q3_variant(c->storage, c->batch, v));
    c->variant = v;
    if (c->batch && v != c->lds_variant && lbm::batch_tile_nodes(c->b, v) != c->tile_nodes)
        return build_tiles(c, lbm::batch_tile_nodes(c->b, v));
    return LBM_OK;
}

int lbm_variant_count(const lbm_ctx_t *c) { return c ? variant_count(c) : 0; }

int lbm_variant_steps(const lbm_ctx_t *c, int32_t v)
{
    if (!c || v < 0 || v >= variant_count(c)) return 0;
    return launch_steps(c, v);
}

int lbm_set_plane_pad(lbm_ctx_t *c, int32_t pad_bytes)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    if (c->pad < 0) return fail(LBM_EINVAL, "this context takes no plane pad (batched, or planes under 1 MiB)");
    if (pad_bytes < 0 || pad_bytes > kPadMaxBytes || pad_bytes % 256 != 0)
        return fail(LBM_EINVAL, "plane pad must be a multiple of 256 bytes in [0, 8192]");
    return set_pad(c, pad_bytes);
}

int lbm_set_batch_steps(lbm_ctx_t *c, const int64_t *stop_steps, int32_t n)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    if (!c->batch) return fail(LBM_EINVAL, "step limits apply to batched contexts");
    if (stop_steps && n != c->n) return fail(LBM_EINVAL, "need one step limit per instance");
    if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
    else HIPCHK(hipDeviceSynchronize());
    for (int i = 0; i < c->n; ++i) {
        const int64_t v = stop_steps ? stop_steps[i] : -1;
        c->inst[i].stop = v < 0 ? INT64_MAX : v;
    }
    HIPCHK(hipMemcpy(c->d_inst, c->inst.data(), sizeof(Inst) * c->n, hipMemcpyHostToDevice));
    return LBM_OK;
}

int lbm_get_layout(const lbm_ctx_t *c, int64_t *plane_stride, int32_t *pad_bytes)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    if (plane_stride) *plane_stride = c->inst[0].plane;
    if (pad_bytes) *pad_bytes = c->pad;
    return LBM_OK;
}

const char *lbm_variant_name(const lbm_ctx_t *c, int32_t v)
{
    if (!c) return "?";
    if (c->batch && v == c->lds_variant && v >= 0) return "batch persistent, lattices resident in LDS";
    if (c->batch) return lbm::batch_variant_name(c->b, v);
    return c->b == 9 ? lbm::d2q9_variant_name(v) : lbm::d1q3_variant_name(v);
}

int lbm_autotune(lbm_ctx_t *c, const char *cache_path, int32_t *chosen)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    char key[256];
    std::snprintf(key, sizeof(key), "%s|%s|lat%d|prec%d|coll%d|bc%d|n%d|%dx%d|nodes%lld", LBM_SOURCE_ID,
                  c->arch.c_str(), c->b, c->p.precision, c->p.collision, c->p.bc, c->n, c->inst[0].nx,
                  c->inst[0].ny, (long long)c->nodes);
    if (cache_path) {
        if (FILE *fh = std::fopen(cache_path, "r")) {
            char line[512];
            int found = -1, found_pad = -1;
            while (std::fgets(line, sizeof(line), fh)) {
                char k2[256];
                int v = -1, pd = -1;
                if (std::sscanf(line, "%255s %d %d", k2, &v, &pd) >= 2 && std::strcmp(k2, key) == 0) {
                    found = v;
                    found_pad = pd;
                }
            }
            std::fclose(fh);
            if (found >= 0 && found < variant_count(c)) {
                if (c->pad >= 0 && found_pad >= 0) {
                    int rc = lbm_set_plane_pad(c, found_pad);
                    if (rc) return rc;
                }
                if (chosen) *chosen = found;
                return lbm_set_variant(c, found);
            }
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int nv = variant_count(c);
    // Enough launches per shape to time at least ~2e8 node updates.
    const int reps = (int)std::max<int64_t>(3, std::min<int64_t>(50, 200000000 / std::max<int64_t>(1, c->nodes)));
    // Time `n` launches of shape v (the source buffer is the current state
    // and is never written: the persistent shape runs an odd number of
    // steps, ending in the other buffer); best of `trials`, in ms per `reps`
    // steps (a two-step shape takes two per launch).
    auto time_shape = [&](int v, int n, int trials, float &out) -> int {
        int rc = lbm_set_variant(c, v);
        if (rc) return rc;
        const bool pers = c->batch && v == c->lds_variant;
        const int pn = n | 1;
        const int spl = launch_steps(c, v);
        float best_t = 1e30f;
        for (int trial = 0; trial < trials; ++trial) {
            HIPCHK(hipEventRecord(e0, c->stream));
            if (pers) {
                HIPCHK(launch_lds(c, c->d_status_scratch, 0, pn, 1));
            } else {
                for (int r = 0; r < n; ++r) {
                    lbm::StepArgs a = step_args(c, c->d_status_scratch, 0, nullptr);
                    HIPCHK(launch_steps_from(c, v, spl, c->cur, a, c->stream));
                }
            }
            HIPCHK(hipEventRecord(e1, c->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            ms *= (float)reps / (float)(pers ? pn : n * spl);
            best_t = std::min(best_t, ms);
        }
        out = best_t;
        return LBM_OK;
    };
    // Stage 1: every shape, a short warm-up then the best of three trials.
    std::vector<std::pair<float, int>> t1;
    for (int v = 0; v < nv; ++v) {
        float ms = 0.0f;
        int rc = time_shape(v, 3, 1, ms);
        if (rc == LBM_OK) rc = time_shape(v, reps, 3, ms);
        if (rc) return rc;
        t1.emplace_back(ms, v);
    }
    std::sort(t1.begin(), t1.end());
    // Stage 2: the eight fastest again with four times longer trials, taken
    // in turn so that clock drift affects them alike.
    const int nc = (int)std::min<size_t>(8, t1.size());
    std::vector<float> t2(nc, 1e30f);
    for (int round = 0; round < 6; ++round) {
        for (int k = 0; k < nc; ++k) {
            float ms = 0.0f;
            int rc = time_shape(t1[k].second, 4 * reps, 1, ms);
            if (rc) return rc;
            t2[k] = std::min(t2[k], ms);
        }
    }
    std::vector<std::pair<float, int>> ranked;
    for (int k = 0; k < nc; ++k) ranked.emplace_back(t2[k], t1[k].second);
    std::sort(ranked.begin(), ranked.end());
    int best_v = ranked[0].second;
    // Stage 3, single lattices with large planes: the plane pad, timed with
    // the two fastest shapes (a shape's rank can depend on the pad) in turn
    // over the candidates (the state moves with it); the fastest pair wins.
    if (c->pad >= 0) {
        constexpr int np = (int)(sizeof(kPadCandidates) / sizeof(kPadCandidates[0]));
        const int ns = (int)std::min<size_t>(2, ranked.size());
        float tp[2][np];
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < np; ++k) tp[j][k] = 1e30f;
        for (int round = 0; round < 3; ++round) {
            for (int k = 0; k < np; ++k) {
                int rc = set_pad(c, kPadCandidates[k]);
                if (rc) return rc;
                for (int j = 0; j < ns; ++j) {
                    float ms = 0.0f;
                    rc = time_shape(ranked[j].second, 4 * reps, 1, ms);
                    if (rc) return rc;
                    tp[j][k] = std::min(tp[j][k], ms);
                }
            }
        }
        int jb = 0, kb = 0;
        for (int j = 0; j < ns; ++j)
            for (int k = 0; k < np; ++k)
                if (tp[j][k] < tp[jb][kb]) {
                    jb = j;
                    kb = k;
                }
        best_v = ranked[jb].second;
        int rc = set_pad(c, kPadCandidates[kb]);
        if (rc) return rc;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int rc = lbm_set_variant(c, best_v);
    if (rc) return rc;
    if (cache_path) {
        if (FILE *fh = std::fopen(cache_path, "a")) {
            if (c->pad >= 0) std::fprintf(fh, "%s %d %d\n", key, best_v, c->pad);
            else std::fprintf(fh, "%s %d\n", key, best_v);
            std::fclose(fh);
        }
    }
    if (chosen) *chosen = best_v;
    return LBM_OK;
}

int lbm_moments(lbm_ctx_t *c, double *rho, double *ux, double *uy)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    const int64_t total = c->nodes;
    double *d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(double) * 3 * (size_t)total));
    hipError_t e = hipSuccess;
    for (int i = 0; i < c->n && e == hipSuccess; ++i) {
        const int64_t o = c->node_prefix[i];
        e = lbm::launch_gather(c->b, c->storage, c->inst[i], c->p.bc, c->buf[c->cur], d + o, d + total + o,
                               d + 2 * total + o, nullptr, c->iscale, c->stream);
    }
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, d, sizeof(double) * total, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && ux) e = hipMemcpyAsync(ux, d + total, sizeof(double) * total, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && uy)
        e = hipMemcpyAsync(uy, d + 2 * total, sizeof(double) * total, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "lbm_moments");
    return LBM_OK;
}

int lbm_get_populations(lbm_ctx_t *c, double *f)
{
    if (!c || !f) return fail(LBM_EINVAL, "null argument");
    const size_t count = (size_t)c->b * (size_t)c->nodes;
    double *d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(double) * count));
    hipError_t e = hipSuccess;
    for (int i = 0; i < c->n && e == hipSuccess; ++i)
        e = lbm::launch_gather(c->b, c->storage, c->inst[i], c->p.bc, c->buf[c->cur], nullptr, nullptr, nullptr,
                               d + (size_t)c->b * c->node_prefix[i], c->iscale, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "lbm_get_populations");
    return LBM_OK;
}

int lbm_set_populations(lbm_ctx_t *c, const double *f)
{
    if (!c || !f) return fail(LBM_EINVAL, "null argument");
    return load_state(c, nullptr, nullptr, nullptr, f);
}

int lbm_status_batch(lbm_ctx_t *c, lbm_status_t *out, int32_t n)
{
    if (!c || !out || n < 1 || n > c->n) return fail(LBM_EINVAL, "bad arguments");
    std::vector<DevStatus> h(c->n);
    HIPCHK(hipMemcpyAsync(h.data(), c->d_status, sizeof(DevStatus) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < n; ++i) {
        out[i].flags = h[i].flags;
        out[i].reserved = 0;
        const bool none = h[i].first == ~0ull;
        out[i].first_step = none ? -1 : (int64_t)(h[i].first >> 32);
        out[i].first_node = none ? -1 : (int64_t)(h[i].first & 0xffffffffull);
        out[i].guarded = h[i].guarded;
    }
    return LBM_OK;
}

int lbm_status(lbm_ctx_t *c, lbm_status_t *out)
{
    if (!c || !out) return fail(LBM_EINVAL, "bad arguments");
    std::vector<lbm_status_t> all(c->n);
    int rc = lbm_status_batch(c, all.data(), c->n);
    if (rc) return rc;
    // Over a batch: the earliest step, and at that step the smallest node in
    // the instances' concatenated node order.
    lbm_status_t s{0, 0, -1, -1, 0};
    for (int i = 0; i < c->n; ++i) {
        const lbm_status_t &x = all[i];
        s.flags |= x.flags;
        s.guarded += x.guarded;
        if (x.first_step < 0) continue;
        const int64_t node = c->node_prefix[i] + x.first_node;
        if (s.first_step < 0 || x.first_step < s.first_step || (x.first_step == s.first_step && node < s.first_node)) {
            s.first_step = x.first_step;
            s.first_node = node;
        }
    }
    *out = s;
    return LBM_OK;
}

int lbm_reset_status(lbm_ctx_t *c)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    HIPCHK(lbm::launch_clear_status(c->d_status, c->n, c->stream));
    return LBM_OK;
}

int lbm_info(const lbm_ctx_t *c, int64_t *steps_done, int64_t *nodes, int64_t *bytes_per_step)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    if (steps_done) *steps_done = c->steps_done;
    if (nodes) *nodes = c->nodes;
    if (bytes_per_step) *bytes_per_step = 2 * (int64_t)c->b * c->nodes * (int64_t)c->elem;
    return LBM_OK;
}

void lbm_free(lbm_ctx_t *c) { destroy(c); }

int lbm_run_noalloc(const lbm_params_t *p, const double *rho, const double *ux, const double *uy, int64_t nsteps,
                    double *rho_out, double *ux_out, double *uy_out, lbm_status_t *status, void *hip_stream)
{
    if (!p || !rho || !ux) return fail(LBM_EINVAL, "p, rho and ux are required");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    int rc = check_params(p);
    if (rc) return rc;
    const int b = p->lattice == LBM_D1Q3 ? 3 : 9;
    if (b == 9 && !uy) return fail(LBM_EINVAL, "uy is required for D2Q9");
    // One instance laid out without a plane pad (the pad only moves planes;
    // results do not depend on it).
    std::vector<Inst> inst;
    int64_t elems = 0, nodes = 0;
    layout(p, 1, /*no plane pad=*/1, b, &inst, &elems, &nodes);
    const size_t elem = elem_bytes(p->precision);
    const size_t bb = buffer_bytes(elems, elem);
    const size_t need = 256 + 2 * bb;
    if (need > (size_t)LBM_NOALLOC_SCRATCH_BYTES) {
        std::snprintf(g_err, sizeof(g_err),
                      "lattice needs %zu bytes of scratch; lbm_run_noalloc holds %zu (use lbm_init for larger ones)",
                      need, (size_t)LBM_NOALLOC_SCRATCH_BYTES);
        return LBM_EINVAL;
    }
    void *base = nullptr;
    rc = scratch_address(&base);
    if (rc) return rc;
    DevStatus *st = (DevStatus *)base;
    char *buf[2] = {(char *)base + 256, (char *)base + 256 + bb};
    const int storage = storage_of(p->precision);
    const int k = p->fp16_exp ? p->fp16_exp : 14;
    const float scale = std::ldexp(1.0f, k), iscale = std::ldexp(1.0f, -k);
    hipStream_t s = (hipStream_t)hip_stream;
    // The scratch keeps the previous call's contents: the status record is
    // cleared by a kernel (no memset node under graph capture) and the
    // initial state overwrites the first buffer.
    HIPCHK(lbm::launch_clear_status(st, 1, s));
    HIPCHK(lbm::launch_init(b, storage, inst[0], p->bc, rho, ux, b == 9 ? uy : nullptr, nullptr, buf[0], scale, s));
    lbm::StepArgs a{};
    a.inst = nullptr;
    a.one = inst[0];
    a.status = st;
    a.step_base = nullptr;
    a.bc = p->bc;
    a.fp16_scale = scale;
    a.fp16_iscale = iscale;
    a.max_steps = 1;
    int cur = 0;
    for (int64_t i = 0; i < nsteps; ++i) {
        a.step = i;
        // Shape 0: one step per launch, every node once per step.
        hipError_t e = (b == 9) ? lbm::launch_d2q9_step(storage, p->collision, 0, buf[cur], buf[cur ^ 1], a, s)
                                : lbm::launch_d1q3_step(storage, 0, buf[cur], buf[cur ^ 1], a, s);
        if (e != hipSuccess) return hip_fail(e, "lbm_run_noalloc step");
        cur ^= 1;
    }
    HIPCHK(lbm::launch_gather(b, storage, inst[0], p->bc, buf[cur], rho_out, ux_out, b == 9 ? uy_out : nullptr,
                              nullptr, iscale, s));
    if (status) {
        DevStatus h{};
        HIPCHK(hipMemcpyAsync(&h, st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        status->flags = h.flags;
        status->reserved = 0;
        const bool none = h.first == ~0ull;
        status->first_step = none ? -1 : (int64_t)(h.first >> 32);
        status->first_node = none ? -1 : (int64_t)(h.first & 0xffffffffull);
        status->guarded = h.guarded;
    }
    return LBM_OK;
}

int lbm_copy_kernel(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src || (bytes & 15)) return fail(LBM_EINVAL, "copy needs non-null pointers and bytes % 16 == 0");
    HIPCHK(lbm::launch_copy(dst, src, bytes, (hipStream_t)stream));
    return LBM_OK;
}

const char *lbm_last_error(void) { return g_err; }

const char *lbm_strerror(int code)
{
    switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory or workspace too small";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ENODEV: return "no usable gfx950 device";
    default: return "unknown error";
    }
}

}  // extern "C"
