// Host runtime behind the C ABI: context, lattices, fields, the field cache
// (pool + pinned-host spill), canonical <-> device layout conversion and
// error reporting.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"

using namespace qdpmi;

#define QDP_API_BEGIN try {
#define QDP_API_END(ctx)                                                          \
    }                                                                             \
    catch (const std::bad_alloc&) {                                               \
        return set_error(ctx, QDP_ERR_NOMEM, "host allocation failed");           \
    }                                                                             \
    catch (...) {                                                                 \
        return set_error(ctx, QDP_ERR_STATE, "unexpected internal exception");    \
    }

namespace qdpmi {

bool SmearTuneKey::operator<(const SmearTuneKey& o) const {
    const int32_t a[8] = {L[0], L[1], L[2], L[3], ncols, prec, mode, batch};
    const int32_t b[8] = {o.L[0], o.L[1], o.L[2], o.L[3], o.ncols, o.prec, o.mode, o.batch};
    return std::lexicographical_compare(a, a + 8, b, b + 8);
}

qdp_status set_error(Ctx* ctx, qdp_status code, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return code;
}

qdp_status hip_error(Ctx* ctx, hipError_t err, const char* what) {
    return set_error(ctx, QDP_ERR_HIP, "%s: %s", what, hipGetErrorString(err));
}

qdp_status check_launch(Ctx* ctx, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(ctx, e, what);
    return QDP_OK;
}

bool HipMover::host_area_ready() {
    if (ctx->host_bytes == 0) return false;
    if (!ctx->host_base) {
        void* p = nullptr;
        if (hipHostMalloc(&p, ctx->host_bytes, hipHostMallocDefault) != hipSuccess) return false;
        ctx->host_base = static_cast<char*>(p);
    }
    return true;
}

bool HipMover::d2h(size_t dev_off, size_t host_off, size_t bytes) {
    return hipMemcpyAsync(ctx->host_base + host_off, ctx->pool_base + dev_off, bytes,
                          hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
}

bool HipMover::h2d(size_t host_off, size_t dev_off, size_t bytes) {
    return hipMemcpyAsync(ctx->pool_base + dev_off, ctx->host_base + host_off, bytes,
                          hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
}

bool HipMover::d2d(size_t src_off, size_t dst_off, size_t bytes) {
    return hipMemcpyAsync(ctx->pool_base + dst_off, ctx->pool_base + src_off, bytes,
                          hipMemcpyDeviceToDevice, ctx->stream) == hipSuccess;
}

Field* find_field(Ctx* ctx, uint64_t id) {
    auto it = ctx->fields.find(id);
    return it == ctx->fields.end() ? nullptr : &it->second;
}

Lattice* find_lattice(Ctx* ctx, uint64_t id) {
    auto it = ctx->lattices.find(id);
    return it == ctx->lattices.end() ? nullptr : &it->second;
}

static qdp_status cache_status(Ctx* ctx, qdp_status s, const char* what) {
    if (s == QDP_OK) return s;
    if (s == QDP_ERR_NOMEM)
        return set_error(ctx, s, "%s: device pool and pinned spill area cannot hold the fields",
                         what);
    if (s == QDP_ERR_HIP) return set_error(ctx, s, "%s: HIP copy failed", what);
    return set_error(ctx, s, "%s: invalid field state", what);
}

qdp_status acquire_field(Ctx* ctx, uint64_t id, bool need_contents, char** ptr) {
    if (!find_field(ctx, id)) return set_error(ctx, QDP_ERR_STATE, "unknown field handle %llu",
                                               (unsigned long long)id);
    QDP_CHECK(cache_status(ctx, ctx->cache.acquire(id, need_contents), "field acquire"));
    *ptr = ctx->pool_base + ctx->cache.find(id)->dev_off;
    return QDP_OK;
}

void release_field(Ctx* ctx, uint64_t id) { ctx->cache.release(id); }

qdp_status field_create(Ctx* ctx, uint64_t lattice, int32_t type, int32_t prec, uint64_t* out) {
    Lattice* lat = find_lattice(ctx, lattice);
    if (!lat) return set_error(ctx, QDP_ERR_STATE, "unknown lattice handle");
    if (!valid_type(type)) return set_error(ctx, QDP_ERR_ARG, "invalid field type %d", type);
    if (!valid_prec(prec)) return set_error(ctx, QDP_ERR_ARG, "invalid precision %d", prec);
    Field f;
    f.id = ctx->next_id++;
    f.lattice = lattice;
    f.type = type;
    f.prec = prec;
    f.bytes = field_bytes(lat->geo, type, prec);
    QDP_CHECK(cache_status(ctx, ctx->cache.create(f.id, (size_t)f.bytes), "field allocation"));
    ctx->fields[f.id] = f;
    *out = f.id;
    return QDP_OK;
}

qdp_status field_destroy(Ctx* ctx, uint64_t id) {
    if (!find_field(ctx, id)) return set_error(ctx, QDP_ERR_STATE, "unknown field handle");
    QDP_CHECK(cache_status(ctx, ctx->cache.destroy(id), "field free"));
    ctx->fields.erase(id);
    return QDP_OK;
}

PoolTemp::~PoolTemp() {
    if (ctx_ && id_) {
        ctx_->cache.release(id_);
        ctx_->cache.destroy(id_);
    }
}

qdp_status PoolTemp::alloc(Ctx* ctx, int64_t bytes) {
    ctx_ = ctx;
    id_ = ctx->next_id++;
    QDP_CHECK(cache_status(ctx, ctx->cache.create(id_, (size_t)std::max<int64_t>(bytes, 1)),
                           "scratch allocation"));
    QDP_CHECK(cache_status(ctx, ctx->cache.acquire(id_, false), "scratch allocation"));
    ptr_ = ctx->pool_base + ctx->cache.find(id_)->dev_off;
    return QDP_OK;
}

qdp_status host_result_buffer(Ctx* ctx, size_t bytes, double** out) {
    if (ctx->host_result_bytes < bytes) {
        if (ctx->host_result) {
            QDP_HIP(ctx, hipStreamSynchronize(ctx->stream));
            hipHostFree(ctx->host_result);
            ctx->host_result = nullptr;
            ctx->host_result_bytes = 0;
        }
        void* p = nullptr;
        QDP_HIP(ctx, hipHostMalloc(&p, bytes, hipHostMallocDefault));
        ctx->host_result = static_cast<double*>(p);
        ctx->host_result_bytes = bytes;
    }
    *out = ctx->host_result;
    return QDP_OK;
}

}  // namespace qdpmi

// -------------------------------------------------------------------------
// Canonical host layout <-> device layout
// -------------------------------------------------------------------------

namespace {

size_t host_doubles(const Geometry& g, int32_t type) {
    const TypeShape s = type_shape(type);
    if (type == QDP_REAL) return (size_t)g.V;
    return (size_t)g.V * s.nrec * s.ncomp * 2;
}

// Offset (in doubles) of component (rec, comp) of lexicographic site s.
inline size_t host_index(const Geometry& g, int32_t type, int64_t s, int32_t rec, int32_t comp) {
    const TypeShape sh = type_shape(type);
    if (type == QDP_REAL) return (size_t)s;
    return (((size_t)rec * g.V + s) * sh.ncomp + comp) * 2;
}

// FP16S encoding of one record of n complex values given in FP32.
void encode_f16s(const float* v, int n, _Float16* q, float* scale) {
    float m = 0.f;
    for (int i = 0; i < 2 * n; ++i) m = std::max(m, std::fabs(v[i]));
    int e = 0;
    if (m > 0.f) std::frexp(m, &e);
    *scale = m > 0.f ? std::ldexp(1.0f, e) : kF16sZeroScale;
    for (int i = 0; i < 2 * n; ++i) q[i] = (_Float16)std::ldexp(v[i], -e);
}

void to_device_layout(const Geometry& g, int32_t type, int32_t prec, const double* host,
                      std::vector<char>& dev) {
    const TypeShape sh = type_shape(type);
    dev.assign((size_t)field_bytes(g, type, prec), 0);
    char* base = dev.data();
    std::vector<float> rec(2 * sh.ncomp);
    std::vector<_Float16> q(2 * sh.ncomp);
    for (int32_t t = 0; t < g.L[3]; ++t)
        for (int32_t z = 0; z < g.L[2]; ++z)
            for (int32_t y = 0; y < g.L[1]; ++y)
                for (int32_t x = 0; x < g.L[0]; ++x) {
                    const int64_t s = x + (int64_t)g.L[0] * (y + (int64_t)g.L[1] * (z + (int64_t)g.L[2] * t));
                    const int64_t c = cb_index(g, x, y, z, t);
                    for (int32_t r = 0; r < sh.nrec; ++r) {
                        for (int32_t k = 0; k < sh.ncomp; ++k) {
                            const size_t hi = host_index(g, type, s, r, k);
                            const double re = host[hi];
                            const double im = type == QDP_REAL ? 0.0 : host[hi + 1];
                            char* p = base + comp_offset(sh.nrec, sh.ncomp, prec, r, k, c);
                            if (prec == QDP_F64) {
                                double* d = reinterpret_cast<double*>(p);
                                d[0] = re;
                                d[1] = im;
                            } else if (prec == QDP_F32) {
                                float* d = reinterpret_cast<float*>(p);
                                d[0] = (float)re;
                                d[1] = (float)im;
                            } else {
                                rec[2 * k] = (float)re;
                                rec[2 * k + 1] = (float)im;
                            }
                        }
                        if (prec == QDP_F16S) {
                            float sc;
                            encode_f16s(rec.data(), sh.ncomp, q.data(), &sc);
                            for (int32_t k = 0; k < sh.ncomp; ++k) {
                                _Float16* d = reinterpret_cast<_Float16*>(
                                    base + comp_offset(sh.nrec, sh.ncomp, prec, r, k, c));
                                d[0] = q[2 * k];
                                d[1] = q[2 * k + 1];
                            }
                            *reinterpret_cast<float*>(base + scale_offset(sh.nrec, sh.ncomp, r, c)) = sc;
                        }
                    }
                }
}

// Convert slices t0..t1-1 to the canonical layout of that sub-lattice.
// `at(off)` returns the host address holding device byte offset `off` of the
// field image (only the tiles of the requested slices are read).
template <typename At>
void from_device_layout(const Geometry& g, int32_t type, int32_t prec, At at, double* host, int32_t t0,
                        int32_t t1) {
    const TypeShape sh = type_shape(type);
    const int64_t Vsub = (int64_t)g.L[0] * g.L[1] * g.L[2] * (t1 - t0);
    for (int32_t t = t0; t < t1; ++t)
        for (int32_t z = 0; z < g.L[2]; ++z)
            for (int32_t y = 0; y < g.L[1]; ++y)
                for (int32_t x = 0; x < g.L[0]; ++x) {
                    const int64_t s = x + (int64_t)g.L[0] * (y + (int64_t)g.L[1] * (z + (int64_t)g.L[2] * (t - t0)));
                    const int64_t c = cb_index(g, x, y, z, t);
                    for (int32_t r = 0; r < sh.nrec; ++r) {
                        float sc = 1.f;
                        if (prec == QDP_F16S)
                            sc = *reinterpret_cast<const float*>(at(scale_offset(sh.nrec, sh.ncomp, r, c)));
                        for (int32_t k = 0; k < sh.ncomp; ++k) {
                            const char* p = at(comp_offset(sh.nrec, sh.ncomp, prec, r, k, c));
                            double re, im;
                            if (prec == QDP_F64) {
                                re = reinterpret_cast<const double*>(p)[0];
                                im = reinterpret_cast<const double*>(p)[1];
                            } else if (prec == QDP_F32) {
                                re = reinterpret_cast<const float*>(p)[0];
                                im = reinterpret_cast<const float*>(p)[1];
                            } else {
                                re = (double)((float)reinterpret_cast<const _Float16*>(p)[0] * sc);
                                im = (double)((float)reinterpret_cast<const _Float16*>(p)[1] * sc);
                            }
                            const size_t hi = type == QDP_REAL ? (size_t)s
                                                               : (((size_t)r * Vsub + s) * sh.ncomp + k) * 2;
                            host[hi] = re;
                            if (type != QDP_REAL) host[hi + 1] = im;
                        }
                    }
                }
}

}  // namespace

// -------------------------------------------------------------------------
// C ABI
// -------------------------------------------------------------------------

extern "C" {

qdp_status qdp_init(const qdp_init_opts* opts, qdp_ctx** out) {
    if (!opts || !out) return QDP_ERR_ARG;
    if (opts->pool_bytes < OffsetPool::kAlign) return QDP_ERR_ARG;
    qdp_ctx* ctx = nullptr;
    try {
        ctx = new qdp_ctx();
    } catch (...) {
        return QDP_ERR_NOMEM;
    }
    auto fail = [&](qdp_status s) {
        if (ctx->own_pool && ctx->pool_base) hipFree(ctx->pool_base);
        delete ctx;
        return s;
    };
    ctx->device = opts->device;
    ctx->stream = static_cast<hipStream_t>(opts->hip_stream);
    ctx->flags = opts->flags;
    if (hipSetDevice(opts->device) != hipSuccess) return fail(QDP_ERR_HIP);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, opts->device) ==
            hipSuccess &&
        cus > 0)
        ctx->num_cus = cus;
    if (opts->pool_ptr) {
        if (reinterpret_cast<uintptr_t>(opts->pool_ptr) % OffsetPool::kAlign) return fail(QDP_ERR_ARG);
        ctx->pool_base = static_cast<char*>(opts->pool_ptr);
    } else {
        void* p = nullptr;
        if (hipMalloc(&p, opts->pool_bytes) != hipSuccess) return fail(QDP_ERR_HIP);
        ctx->pool_base = static_cast<char*>(p);
        ctx->own_pool = true;
    }
    ctx->pool_bytes = opts->pool_bytes;
    ctx->host_bytes = opts->host_spill_bytes;
    ctx->mover.ctx = ctx;
    ctx->cache.reset(opts->pool_bytes, opts->host_spill_bytes, &ctx->mover);
    if (const char* env = std::getenv("QDP_FAULT_ALLOC_AFTER")) ctx->cache.fault_after(std::atoll(env));
    build_gamma_tables(ctx);
    if (noalloc_scratch_init(ctx) != QDP_OK) return fail(QDP_ERR_HIP);
    *out = ctx;
    return QDP_OK;
}

qdp_status qdp_finalize(qdp_ctx* ctx) {
    if (!ctx) return QDP_ERR_ARG;
    hipStreamSynchronize(ctx->stream);
    release_graphs(ctx);
    if (ctx->own_pool && ctx->pool_base) hipFree(ctx->pool_base);
    if (ctx->host_base) hipHostFree(ctx->host_base);
    if (ctx->host_result) hipHostFree(ctx->host_result);
    delete ctx;
    return QDP_OK;
}

qdp_status qdp_lattice_create(qdp_ctx* ctx, const int32_t dims[4], qdp_lattice* out) {
    if (!ctx || !dims || !out) return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_API_BEGIN
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 2 || dims[i] % 2)
            return set_error(ctx, QDP_ERR_LATTICE,
                             "lattice extents must be even and >= 2 (got %d %d %d %d)", dims[0],
                             dims[1], dims[2], dims[3]);
    if ((int64_t)dims[0] * dims[1] * dims[2] * dims[3] > (int64_t(1) << 31))
        return set_error(ctx, QDP_ERR_LATTICE, "lattice volume above 2^31 sites");
    Lattice lat;
    lat.geo = make_geometry(dims);
    const uint64_t id = ctx->next_id++;
    ctx->lattices[id] = lat;
    *out = id;
    return QDP_OK;
    QDP_API_END(ctx)
}

qdp_status qdp_field_alloc(qdp_ctx* ctx, qdp_lattice lat, int32_t type, int32_t prec,
                           qdp_field* out) {
    if (!ctx || !out) return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_API_BEGIN
    return field_create(ctx, lat, type, prec, out);
    QDP_API_END(ctx)
}

qdp_status qdp_field_free(qdp_ctx* ctx, qdp_field f) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_API_BEGIN
    return field_destroy(ctx, f);
    QDP_API_END(ctx)
}

qdp_status qdp_field_host_doubles(qdp_ctx* ctx, qdp_field f, size_t* n) {
    if (!ctx || !n) return set_error(ctx, QDP_ERR_ARG, "null argument");
    Field* fd = find_field(ctx, f);
    if (!fd) return set_error(ctx, QDP_ERR_STATE, "unknown field handle");
    *n = host_doubles(find_lattice(ctx, fd->lattice)->geo, fd->type);
    return QDP_OK;
}

qdp_status qdp_field_info(qdp_ctx* ctx, qdp_field f, qdp_field_info_t* out) {
    if (!ctx || !out) return set_error(ctx, QDP_ERR_ARG, "null argument");
    Field* fd = find_field(ctx, f);
    if (!fd) return set_error(ctx, QDP_ERR_STATE, "unknown field handle");
    const CacheEntry* e = ctx->cache.find(f);
    out->type = fd->type;
    out->prec = fd->prec;
    out->lattice = fd->lattice;
    out->bytes = (uint64_t)fd->bytes;
    out->on_device = e && e->on_device ? 1 : 0;
    out->reserved = 0;
    return QDP_OK;
}

qdp_status qdp_field_device_ptr(qdp_ctx* ctx, qdp_field f, void** ptr, uint64_t* bytes) {
    if (!ctx || !ptr || !bytes) return set_error(ctx, QDP_ERR_ARG, "null argument");
    Field* fd = find_field(ctx, f);
    if (!fd) return set_error(ctx, QDP_ERR_STATE, "unknown field handle");
    char* p;
    QDP_CHECK(acquire_field(ctx, f, true, &p));
    release_field(ctx, f);
    *ptr = p;
    *bytes = (uint64_t)fd->bytes;
    return QDP_OK;
}

qdp_status qdp_field_write(qdp_ctx* ctx, qdp_field f, const double* host, size_t n_doubles) {
    if (!ctx || !host) return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_API_BEGIN
    Field* fd = find_field(ctx, f);
    if (!fd) return set_error(ctx, QDP_ERR_STATE, "unknown field handle");
    const Geometry& g = find_lattice(ctx, fd->lattice)->geo;
    if (n_doubles != host_doubles(g, fd->type))
        return set_error(ctx, QDP_ERR_ARG, "field_write: expected %zu doubles, got %zu",
                         host_doubles(g, fd->type), n_doubles);
    std::vector<char> staging;
    to_device_layout(g, fd->type, fd->prec, host, staging);
    char* p;
    QDP_CHECK(acquire_field(ctx, f, false, &p));
    hipError_t e = hipMemcpyAsync(p, staging.data(), staging.size(), hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    release_field(ctx, f);
    if (e != hipSuccess) return hip_error(ctx, e, "field_write copy");
    return QDP_OK;
    QDP_API_END(ctx)
}

qdp_status qdp_field_read(qdp_ctx* ctx, qdp_field f, double* host, size_t n_doubles) {
    if (!ctx || !host) return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_API_BEGIN
    Field* fd = find_field(ctx, f);
    if (!fd) return set_error(ctx, QDP_ERR_STATE, "unknown field handle");
    const Geometry& g = find_lattice(ctx, fd->lattice)->geo;
    if (n_doubles != host_doubles(g, fd->type))
        return set_error(ctx, QDP_ERR_ARG, "field_read: expected %zu doubles, got %zu",
                         host_doubles(g, fd->type), n_doubles);
    std::vector<char> staging((size_t)fd->bytes);
    const CacheEntry* ce = ctx->cache.find(f);
    if (ce && !ce->on_device && ce->on_host) {
        // spilled: read the pinned host copy once the stream has written it
        QDP_HIP(ctx, hipStreamSynchronize(ctx->stream));
        std::memcpy(staging.data(), ctx->host_base + ce->host_off, staging.size());
    } else {
        char* p;
        QDP_CHECK(acquire_field(ctx, f, true, &p));
        hipError_t e = hipMemcpyAsync(staging.data(), p, staging.size(), hipMemcpyDeviceToHost,
                                      ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        release_field(ctx, f);
        if (e != hipSuccess) return hip_error(ctx, e, "field_read copy");
    }
    const char* img = staging.data();
    from_device_layout(g, fd->type, fd->prec, [img](int64_t off) { return img + off; }, host, 0, g.L[3]);
    return QDP_OK;
    QDP_API_END(ctx)
}

qdp_status qdp_field_read_timeslices(qdp_ctx* ctx, qdp_field f, int32_t t_begin, int32_t t_end,
                                     double* host, size_t n_doubles) {
    if (!ctx || !host) return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_API_BEGIN
    Field* fd = find_field(ctx, f);
    if (!fd) return set_error(ctx, QDP_ERR_STATE, "unknown field handle");
    const Geometry& g = find_lattice(ctx, fd->lattice)->geo;
    if (t_begin < 0 || t_end > g.L[3] || t_begin >= t_end)
        return set_error(ctx, QDP_ERR_ARG, "read_timeslices: bad slice range");
    const TypeShape sh = type_shape(fd->type);
    const int64_t Vsub = (int64_t)g.L[0] * g.L[1] * g.L[2] * (t_end - t_begin);
    const size_t need = fd->type == QDP_REAL ? (size_t)Vsub : (size_t)Vsub * sh.nrec * sh.ncomp * 2;
    if (n_doubles != need)
        return set_error(ctx, QDP_ERR_ARG, "read_timeslices: expected %zu doubles, got %zu", need, n_doubles);
    // the slices occupy checkerboard sites [p Vh + t_begin Vsh, p Vh + t_end Vsh) for
    // p = 0, 1: copy the tiles of those two ranges into one compact staging buffer
    const int64_t tb = tile_bytes(sh.nrec, sh.ncomp, fd->prec);
    int64_t a[2], b[2];
    for (int par = 0; par < 2; ++par) {
        a[par] = (par * g.Vh + t_begin * g.Vsh) / 64;
        b[par] = (par * g.Vh + t_end * g.Vsh + 63) / 64;
    }
    if (a[1] < b[0]) a[1] = b[0];  // tiny lattices: the two ranges share a tile
    std::vector<char> staging((size_t)((b[0] - a[0] + b[1] - a[1]) * tb));
    char* p;
    QDP_CHECK(acquire_field(ctx, f, true, &p));
    hipError_t e = hipMemcpyAsync(staging.data(), p + a[0] * tb, (size_t)((b[0] - a[0]) * tb),
                                  hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && b[1] > a[1])
        e = hipMemcpyAsync(staging.data() + (b[0] - a[0]) * tb, p + a[1] * tb, (size_t)((b[1] - a[1]) * tb),
                           hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    release_field(ctx, f);
    if (e != hipSuccess) return hip_error(ctx, e, "read_timeslices copy");
    const char* img = staging.data();
    const int64_t a0 = a[0], b0 = b[0], a1 = a[1];
    auto at = [=](int64_t off) {
        const int64_t tile = off / tb;
        const int64_t within = off - tile * tb;
        const int64_t pos = tile < b0 ? tile - a0 : (b0 - a0) + (tile - a1);
        return img + pos * tb + within;
    };
    from_device_layout(g, fd->type, fd->prec, at, host, t_begin, t_end);
    return QDP_OK;
    QDP_API_END(ctx)
}

qdp_status qdp_cache_stats(qdp_ctx* ctx, qdp_cache_stats_t* out) {
    if (!ctx || !out) return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const CacheCounters& c = ctx->cache.counters();
    out->hits = c.hits;
    out->misses = c.misses;
    out->spills = c.spills;
    out->fills = c.fills;
    out->bytes_spilled = c.bytes_spilled;
    out->bytes_filled = c.bytes_filled;
    out->pool_capacity = ctx->cache.device_pool().capacity();
    out->pool_limit = ctx->cache.device_pool().limit();
    out->pool_used = ctx->cache.device_pool().used_bytes();
    out->pool_high_water = ctx->cache.device_pool().high_water();
    out->host_used = ctx->cache.host_pool().used_bytes();
    out->n_fields = ctx->fields.size();
    out->n_external = ctx->external.size();
    out->external_bytes = ctx->external_bytes;
    return QDP_OK;
}

qdp_status qdp_cache_evict(qdp_ctx* ctx, qdp_field f) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_API_BEGIN
    if (!find_field(ctx, f)) return set_error(ctx, QDP_ERR_STATE, "unknown field handle");
    return cache_status(ctx, ctx->cache.evict(f), "cache_evict");
    QDP_API_END(ctx)
}

qdp_status qdp_cache_evict_all(qdp_ctx* ctx) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_API_BEGIN
    return cache_status(ctx, ctx->cache.evict_all(), "cache_evict_all");
    QDP_API_END(ctx)
}

qdp_status qdp_set_pool_limit(qdp_ctx* ctx, size_t bytes) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_API_BEGIN
    if (bytes > ctx->pool_bytes) return set_error(ctx, QDP_ERR_ARG, "pool limit above capacity");
    return cache_status(ctx, ctx->cache.set_limit(bytes), "set_pool_limit");
    QDP_API_END(ctx)
}

qdp_status qdp_pool_malloc(qdp_ctx* ctx, size_t bytes, void** out) {
    if (!ctx || !out || bytes == 0) return set_error(ctx, QDP_ERR_ARG, "pool_malloc: bad argument");
    QDP_API_BEGIN
    const uint64_t id = ctx->next_id++;
    QDP_CHECK(cache_status(ctx, ctx->cache.create(id, bytes), "pool_malloc"));
    // pinned for the block's whole life: never chosen as a spill victim
    qdp_status s = ctx->cache.acquire(id, false);
    if (s != QDP_OK) {
        ctx->cache.destroy(id);
        return cache_status(ctx, s, "pool_malloc");
    }
    char* p = ctx->pool_base + ctx->cache.find(id)->dev_off;
    ctx->external[reinterpret_cast<uintptr_t>(p)] = id;
    ctx->external_bytes += bytes;
    *out = p;
    return QDP_OK;
    QDP_API_END(ctx)
}

qdp_status qdp_pool_free(qdp_ctx* ctx, void* p) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_API_BEGIN
    auto it = ctx->external.find(reinterpret_cast<uintptr_t>(p));
    if (it == ctx->external.end())
        return set_error(ctx, QDP_ERR_ARG, "pool_free: %p is not a live pool_malloc block", p);
    const uint64_t id = it->second;
    ctx->external_bytes -= ctx->cache.find(id)->bytes;
    ctx->cache.release(id);
    ctx->cache.destroy(id);
    ctx->external.erase(it);
    return QDP_OK;
    QDP_API_END(ctx)
}

qdp_status qdp_fault_alloc_after(qdp_ctx* ctx, int64_t n) {
    if (!ctx || n < 0) return set_error(ctx, QDP_ERR_ARG, "bad argument");
    ctx->cache.fault_after(n);
    return QDP_OK;
}

qdp_status qdp_sync(qdp_ctx* ctx) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return QDP_OK;
}

const char* qdp_last_error(qdp_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

qdp_status qdp_smear_set_shape(qdp_ctx* ctx, const qdp_launch_shape* shape) {
    if (!ctx || !shape) return set_error(ctx, QDP_ERR_ARG, "null argument");
    if (shape->site_waves != 0) {
        const int sw = shape->site_waves, cg = shape->col_groups;
        if (sw < 1 || cg < 1 || cg > 12 || sw * cg > 4 || shape->xcd < 0 || shape->xcd > 2 ||
            !(shape->waves_per_simd == 0 || shape->waves_per_simd == 2 || shape->waves_per_simd == 3) ||
            shape->flat < 0 || shape->flat > 1 || shape->zstack < 0 || shape->zstack > 2 || shape->lds < 0 ||
            shape->lds > 2)
            return set_error(ctx, QDP_ERR_ARG, "launch shape out of range (site_waves * col_groups <= 4, lds <= 2)");
    }
    ctx->forced = *shape;
    return QDP_OK;
}

qdp_status qdp_smear_get_shape(qdp_ctx* ctx, qdp_launch_shape* out) {
    if (!ctx || !out) return set_error(ctx, QDP_ERR_ARG, "null argument");
    *out = ctx->last_shape;
    return QDP_OK;
}

// ---- entry points whose work lives in the kernel translation units ------

static qdp_status copy_handles(qdp_ctx* ctx, const qdp_field* in, int32_t n, std::vector<uint64_t>& out) {
    if (!in || n < 1 || n > 12) return set_error(ctx, QDP_ERR_ARG, "expected 1..12 column handles");
    out.assign(in, in + n);
    return QDP_OK;
}

qdp_status qdp_smear_jacobi(qdp_ctx* ctx, qdp_field gauge, const qdp_field* cols, int32_t ncols,
                            double kappa, int32_t n_iter, int32_t j_decay, int32_t mode) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_API_BEGIN
    std::vector<uint64_t> c;
    QDP_CHECK(copy_handles(ctx, cols, ncols, c));
    return smear_jacobi_impl(ctx, gauge, c.data(), c.data(), ncols, kappa, n_iter, j_decay, mode);
    QDP_API_END(ctx)
}

qdp_status qdp_smear_jacobi_to(qdp_ctx* ctx, qdp_field gauge, const qdp_field* src,
                               const qdp_field* dst, int32_t ncols, double kappa, int32_t n_iter,
                               int32_t j_decay, int32_t mode) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_API_BEGIN
    std::vector<uint64_t> s, d;
    QDP_CHECK(copy_handles(ctx, src, ncols, s));
    QDP_CHECK(copy_handles(ctx, dst, ncols, d));
    return smear_jacobi_impl(ctx, gauge, s.data(), d.data(), ncols, kappa, n_iter, j_decay, mode);
    QDP_API_END(ctx)
}

qdp_status qdp_smear_jacobi_batch(qdp_ctx* ctx, const qdp_smear_job* jobs, int32_t njobs,
                                  double kappa, int32_t n_iter) {
    if (!ctx) return QDP_ERR_ARG;
    if (!jobs || njobs < 1) return set_error(ctx, QDP_ERR_ARG, "no jobs");
    QDP_API_BEGIN
    return smear_batch_impl(ctx, jobs, njobs, kappa, n_iter);
    QDP_API_END(ctx)
}

qdp_status qdp_hadron_contract(qdp_ctx* ctx, const qdp_field* S1, const qdp_field* S2,
                               uint32_t gamma_mask, int32_t t0, int32_t j_decay, double* out) {
    if (!ctx) return QDP_ERR_ARG;
    if (!S1 || !S2 || !out) return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_API_BEGIN
    return hadron_contract_impl(ctx, S1, S2, gamma_mask, t0, j_decay, nullptr, 0, out);
    QDP_API_END(ctx)
}

qdp_status qdp_hadron_contract_noalloc(qdp_ctx* ctx, const qdp_field* S1, const qdp_field* S2,
                                       uint32_t gamma_mask, int32_t t0, int32_t j_decay, double* out_dev) {
    if (!ctx) return QDP_ERR_ARG;
    if (!S1 || !S2 || !out_dev) return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_API_BEGIN
    return hadron_contract_noalloc_impl(ctx, S1, S2, gamma_mask, t0, j_decay, out_dev);
    QDP_API_END(ctx)
}

qdp_status qdp_hadron_contract_mom(qdp_ctx* ctx, const qdp_field* S1, const qdp_field* S2, uint32_t gamma_mask,
                                   const int32_t* moms, int32_t nmom, int32_t t0, int32_t j_decay, double* out) {
    if (!ctx) return QDP_ERR_ARG;
    if (!S1 || !S2 || !out || !moms) return set_error(ctx, QDP_ERR_ARG, "null argument");
    if (nmom < 1) return set_error(ctx, QDP_ERR_ARG, "contract_mom: nmom must be >= 1");
    QDP_API_BEGIN
    return hadron_contract_impl(ctx, S1, S2, gamma_mask, t0, j_decay, moms, nmom, out);
    QDP_API_END(ctx)
}

qdp_status qdp_baryon_contract(qdp_ctx* ctx, const qdp_field* Su, const qdp_field* Sd, int32_t kind,
                               int32_t parity, int32_t t0, int32_t j_decay, double* out) {
    if (!ctx) return QDP_ERR_ARG;
    if (!Su || (!Sd && kind != QDP_BARYON_DELTA_PP) || !out) return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_API_BEGIN
    return baryon_contract_impl(ctx, Su, Sd, kind, parity, t0, j_decay, out);
    QDP_API_END(ctx)
}

qdp_status qdp_eval(qdp_ctx* ctx, const qdp_expr* expr, qdp_field dest, qdp_subset subset,
                    int32_t assign) {
    if (!ctx) return QDP_ERR_ARG;
    if (!expr || !expr->nodes || expr->n < 1) return set_error(ctx, QDP_ERR_ARG, "empty expression");
    QDP_API_BEGIN
    return eval_impl(ctx, expr, dest, subset, assign);
    QDP_API_END(ctx)
}

qdp_status qdp_shift(qdp_ctx* ctx, qdp_field dest, qdp_field src, int32_t mu, int32_t sign,
                     qdp_subset subset) {
    if (!ctx) return QDP_ERR_ARG;
    if (mu < 0 || mu > 3 || (sign != 1 && sign != -1))
        return set_error(ctx, QDP_ERR_ARG, "shift: mu in 0..3 and sign +1/-1");
    qdp_node nodes[2];
    std::memset(nodes, 0, sizeof nodes);
    nodes[0].op = QDP_OP_FIELD;
    nodes[0].field = src;
    nodes[1].op = QDP_OP_SHIFT;
    nodes[1].i0 = mu;
    nodes[1].i1 = sign;
    qdp_expr e{nodes, 2};
    QDP_API_BEGIN
    return eval_impl(ctx, &e, dest, subset, QDP_ASSIGN);
    QDP_API_END(ctx)
}

qdp_status qdp_sum_multi(qdp_ctx* ctx, const qdp_expr* expr, int32_t set, double* out,
                         size_t n_doubles) {
    if (!ctx) return QDP_ERR_ARG;
    if (!expr || !expr->nodes || expr->n < 1 || !out)
        return set_error(ctx, QDP_ERR_ARG, "null argument");
    QDP_API_BEGIN
    return sum_multi_impl(ctx, expr, set, out, n_doubles);
    QDP_API_END(ctx)
}

qdp_status qdp_fill_random(qdp_ctx* ctx, qdp_field f, int32_t kind, uint64_t seed, int32_t column,
                           double scale) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_API_BEGIN
    return fill_random_impl(ctx, f, kind, seed, column, scale);
    QDP_API_END(ctx)
}

qdp_status qdp_fill_point(qdp_ctx* ctx, qdp_field f, int64_t site, int32_t spin, int32_t colour) {
    if (!ctx) return QDP_ERR_ARG;
    QDP_API_BEGIN
    return fill_point_impl(ctx, f, site, spin, colour);
    QDP_API_END(ctx)
}

}  // extern "C"
