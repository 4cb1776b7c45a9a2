// Host-side (FP64) construction of the distance-driven projector tables.
//
// For each view the library stores, in FP32 for the kernels:
//   * the sweep frame (rows when |cos theta| >= |sin theta|, else columns),
//     decided here in FP64;
//   * for every bin boundary b' = 0..B, the along-line position of the
//     boundary ray on sweep line q as X0 + X1 q, in pixel units from the
//     line's first pixel edge (intersections of a straight line with a family
//     of parallel lines are affine in the line index);
//   * for every bin, the path length per sweep line of the bin-centre ray,
//     line spacing / |cos(angle to the line normal)|;
//   * the rational map from a point (K, q), K centred on the image, back to
//     its fractional bin index,
//     used by the pixel-driven back projector to find the bins a pixel sees,
//     and per sweep line its restriction to that line with the factor that
//     turns a residual of the map into the fraction of the bin.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "internal.h"

namespace mbmd {

void validate_geometry(const mbmd_geometry& g) {
    MBMD_REQUIRE(g.kind >= 0 && g.kind <= 2, MBMD_ERR_ARG, "geometry kind must be 0, 1 or 2");
    MBMD_REQUIRE(g.nx > 0 && g.ny > 0 && g.n_views > 0 && g.n_bins > 0, MBMD_ERR_ARG,
                 "geometry sizes must be positive");
    if (g.kind == MBMD_GEOM_IDENTITY) {
        MBMD_REQUIRE(g.nx == g.n_bins && g.ny == g.n_views, MBMD_ERR_SHAPE,
                     "identity geometry needs nx == n_bins and ny == n_views");
        return;
    }
    MBMD_REQUIRE(g.nx <= 8192 && g.ny <= 8192 && g.n_bins <= 65535 && g.n_views <= 65535,
                 MBMD_ERR_SHAPE, "geometry too large");
    MBMD_REQUIRE(g.dx > 0 && g.dy > 0 && g.du > 0, MBMD_ERR_ARG, "pixel and bin sizes must be positive");
    if (g.kind == MBMD_GEOM_FAN_FLAT) {
        const double r = 0.5 * std::hypot(g.nx * g.dx, g.ny * g.dy);
        MBMD_REQUIRE(g.dso > r * 1.0001 && g.dsd > 0, MBMD_ERR_SHAPE,
                     "fan beam: the source must lie outside the image's circumscribed circle");
    }
}

namespace {

struct Ray {
    double px, py, rx, ry;
};

Ray boundary_ray(const mbmd_geometry& g, double c, double s, double u) {
    const double ex = c, ey = s, dxv = -s, dyv = c;
    if (g.kind == MBMD_GEOM_PARALLEL) return {u * ex, u * ey, dxv, dyv};
    const double sx = -g.dso * dxv, sy = -g.dso * dyv;
    const double tx = (g.dsd - g.dso) * dxv + u * ex, ty = (g.dsd - g.dso) * dyv + u * ey;
    return {sx, sy, tx - sx, ty - sy};
}

}  // namespace

void build_geometry_host(const mbmd_geometry& g, GeomHost& h) {
    validate_geometry(g);
    MBMD_REQUIRE(g.kind != MBMD_GEOM_IDENTITY, MBMD_ERR_ARG, "identity geometry has no projector tables");
    const int V = g.n_views, B = g.n_bins;
    std::vector<ViewParams>& vp = h.vp;
    vp.assign(V, ViewParams{});
    std::vector<float2>& bound = h.bound;
    bound.assign((size_t)V * (B + 1), make_float2(0.f, 0.f));
    const int QL = g.nx > g.ny ? g.nx : g.ny;
    std::vector<float4>& line = h.line;
    line.assign((size_t)QL * V * 2 + 2 * kBackMaxU, make_float4(0.f, 0.f, 0.f, 0.f));   // zero padding at the end
    std::vector<float>& path = h.path;
    path.assign((size_t)V * B, 0.0f);
    std::vector<int> views[2];

    // Per-view tables are stored in "slot" order: the views sweeping rows first,
    // then the views sweeping columns; frame_views maps a slot to its view.
    std::vector<int> frame_of(V);
    for (int v = 0; v < V; ++v) {
        const double th = g.theta0 + v * g.dtheta;
        const int frame = std::fabs(std::cos(th)) >= std::fabs(std::sin(th)) ? 0 : 1;
        frame_of[v] = frame;
        views[frame].push_back(v);
    }
    std::vector<int>& fv = h.fv;
    fv = views[0];
    fv.insert(fv.end(), views[1].begin(), views[1].end());
    for (int slot = 0; slot < V; ++slot) {
        const int v = fv[slot];
        const double th = g.theta0 + v * g.dtheta;
        const double c = std::cos(th), s = std::sin(th);
        const int frame = frame_of[v];
        const int ia = frame == 0 ? 1 : 0;        // line-normal axis (y for row sweeps)
        const int it = frame == 0 ? 0 : 1;        // along-line axis
        const double dq = frame == 0 ? g.dy : g.dx;
        const double dp = frame == 0 ? g.dx : g.dy;
        std::vector<double> C0s(B + 1), C1s(B + 1);
        for (int bb = 0; bb <= B; ++bb) {
            const double u = (bb - 0.5 * B) * g.du + g.u_offset;
            const Ray r = boundary_ray(g, c, s, u);
            const double P[2] = {r.px, r.py}, R[2] = {r.rx, r.ry};
            const double rn = std::hypot(R[0], R[1]);
            MBMD_REQUIRE(std::fabs(R[ia]) > 1e-9 * rn, MBMD_ERR_SHAPE,
                         "a bin boundary ray runs parallel to its sweep lines (fan too wide)");
            const double slope = R[it] / R[ia];
            // along-line coordinate on the line at normal coordinate a = qq * dq:
            //   t = P_t + (a - P_a) * slope
            const double C0 = (P[it] - P[ia] * slope) / dp;
            const double C1 = dq * slope / dp;
            const double X0 = C0 + 0.5 * (frame == 0 ? g.nx : g.ny) - C1 * 0.5 * ((frame == 0 ? g.ny : g.nx) - 1);
            bound[(size_t)slot * (B + 1) + bb] = make_float2((float)X0, (float)C1);
            C0s[bb] = C0;
            C1s[bb] = C1;
        }
        // Orientation: the sign of the bin widths K(b+1) - K(b).  They are affine in
        // the line coordinate, so checking the first and last sweep line covers every
        // line; a sign change would need the source inside the slab of sweep lines.
        const double qmax = 0.5 * ((frame == 0 ? g.ny : g.nx) - 1);
        int n_pos = 0, n_neg = 0;
        for (int b = 0; b < B; ++b)
            for (double qq : {-qmax, qmax}) {
                const double w = (C0s[b + 1] - C0s[b]) + (C1s[b + 1] - C1s[b]) * qq;
                n_pos += w > 0.0;
                n_neg += w < 0.0;
            }
        MBMD_REQUIRE(n_pos == 0 || n_neg == 0, MBMD_ERR_SHAPE,
                     "fan beam: the source lies between the sweep lines of a view (source too close)");
        if (n_neg) std::reverse(bound.begin() + (size_t)slot * (B + 1), bound.begin() + (size_t)(slot + 1) * (B + 1));
        for (int b = 0; b < B; ++b) {
            const double u = (b - 0.5 * (B - 1)) * g.du + g.u_offset;
            const Ray r = boundary_ray(g, c, s, u);
            const double R[2] = {r.rx, r.ry};
            path[(size_t)slot * B + b] = (float)(dq * std::hypot(R[0], R[1]) / std::fabs(R[ia]));
        }
        // fractional bin index of the point at along position K (pixels, centred)
        // on line qq: world point with along coordinate K dp and normal qq dq.
        const double e[2] = {c, s}, d[2] = {-s, c};
        const double u0 = -0.5 * B * g.du + g.u_offset;     // left edge of bin 0
        double n0, nK, nq, d0, dK, dqq;
        if (g.kind == MBMD_GEOM_PARALLEL) {
            n0 = -u0 / g.du;
            nK = e[it] * dp / g.du;
            nq = e[ia] * dq / g.du;
            d0 = 1.0;
            dK = 0.0;
            dqq = 0.0;
        } else {
            // u = dsd (e.X) / (d.X + dso);  beta = (u - u0) / du
            n0 = -u0 * g.dso;
            nK = (g.dsd * e[it] - u0 * d[it]) * dp;
            nq = (g.dsd * e[ia] - u0 * d[ia]) * dq;
            d0 = g.du * g.dso;
            dK = g.du * d[it] * dp;
            dqq = g.du * d[ia] * dq;
        }
        ViewParams p{};
        p.n0 = (float)n0;
        p.nK = (float)nK;
        p.nq = (float)nq;
        p.d0 = (float)d0;
        p.dK = (float)dK;
        p.dq = (float)dqq;
        // Per sweep line: with N = n0 + nq qq and D = d0 + dqq qq the bin index is
        // beta(K) = (N + nK K) / (D + dK K).  Boundary b sits at K_b with
        // beta(K_b) = b; the map is projective, so
        //   (K - K_b) / (K_{b+1} - K_b) = (num - b den) (nK - (b+1) dK) / Delta,
        // Delta = D nK - N dK (nonzero: boundaries are distinct and not parallel to
        // the line).  Numerator and denominator are divided by D, so that the
        // denominator is 1 + c K, and the bin origin moves to the detector centre,
        // which bounds the in-range FP32 map values by half the detector and makes
        // the clamp of the bin index symmetric.  For a view whose bins run along -K
        // the map is of the reversed index B - beta (numerator B (D + dK K) -
        // (N + nK K)), matching its detector row, which the back projector stores
        // from the last bin: every row then runs along +K.
        const int Nq = frame == 0 ? g.ny : g.nx;
        const double sh = (double)back_shift(B);
        for (int q = 0; q < Nq; ++q) {
            const double qq = q - 0.5 * (Nq - 1);
            const double D = d0 + dqq * qq;
            const double N = n_neg ? B * D - (n0 + nq * qq) : n0 + nq * qq;
            const double nKl = n_neg ? B * dK - nK : nK;
            const double delta = D * nKl - N * dK;
            MBMD_REQUIRE(std::fabs(delta) > 0.0 && D > 0.0, MBMD_ERR_SHAPE,
                         "degenerate bin map on a sweep line (source too close)");
            float4* L = &line[((size_t)q * V + slot) * 2];
            L[0] = make_float4((float)((N - sh * D) / D), (float)((nKl - sh * dK) / D), (float)(dK / D),
                               (float)(D * (nKl - (sh + 1.0) * dK) / delta));
            L[1] = make_float4((float)(D * dK / delta), 0.0f, 0.0f, 0.0f);
        }
        p.orient = n_neg == 0 ? 1.0f : -1.0f;
        p.view_frame = v | (frame << 16);
        vp[slot] = p;
    }
    h.n_frame_views[0] = (int)views[0].size();
    h.n_frame_views[1] = (int)views[1].size();

    // Forward items of each frame in order of decreasing work: the active lines
    // of the item's half, summed over its wavefronts, from the same hull the
    // kernel computes.  Dispatching the heaviest first balances the CUs (the
    // fan is usually wider than the image, so many items have no lines at all).
    std::vector<int>& order = h.order;
    order.clear();
    {
        const int chunks = fwd_chunks(B);
        for (int f = 0; f < 2; ++f) {
            const int nv = (int)views[f].size(), slot0 = f ? (int)views[0].size() : 0;
            const int Nq = f ? g.nx : g.ny, Np = f ? g.ny : g.nx;
            std::vector<std::pair<long long, int>> w;
            w.reserve((size_t)nv * chunks * 2);
            for (int sl = 0; sl < nv; ++sl)
                for (int c = 0; c < chunks; ++c)
                    for (int h = 0; h < 2; ++h) {
                        long long work = 0;
                        const float2* brow = &bound[(size_t)(slot0 + sl) * (B + 1)];
                        for (int wv = 0; wv < kFwdWaves; ++wv) {
                            const int e0 = (c * kFwdWaves + wv) * kFwdBinsPerWave;
                            if (e0 >= B) break;
                            int lo = 0, hi = -1;
                            active_lines(brow[e0], brow[std::min(e0 + kFwdBinsPerWave, B)], Np, Nq, lo, hi);
                            const int mid = (lo + hi + 1) >> 1;
                            work += std::max(0, h ? hi - mid + 1 : mid - lo);
                        }
                        w.emplace_back(work, (sl * chunks + c) * 2 + h);
                    }
            std::stable_sort(w.begin(), w.end(), [](const std::pair<long long, int>& a,
                                                    const std::pair<long long, int>& b) { return a.first > b.first; });
            for (const auto& e : w) order.push_back(e.second);
        }
    }

}

namespace {
size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

// Byte layout of a geometry's device block: tables, then the scratch of the
// forward (line prefixes) and of the back projection (detector rows, column part).
struct GeomLayout {
    size_t view, bound, path, fv, pre, line, order, det, part;
    size_t total() const { return view + bound + path + fv + pre + line + order + det + part; }
};

static GeomLayout layout_of(const mbmd_geometry& g, int prefix_mat, int back_ch) {
    const size_t V = g.n_views, B = g.n_bins, nj = (size_t)g.nx * g.ny;
    const size_t QL = g.nx > g.ny ? g.nx : g.ny;
    GeomLayout L;
    L.view = al256(sizeof(ViewParams) * V);
    L.bound = al256(sizeof(float2) * V * (B + 1));
    L.path = al256(sizeof(float) * V * B);
    L.fv = al256(sizeof(int) * V);
    L.pre = al256(sizeof(float) * prefix_elems(g.nx, g.ny) * prefix_mat);
    // the back projector's per-line maps, padded for the prefetch of its last group of views
    L.line = back_ch ? al256(sizeof(float4) * (QL * V * 2 + 2 * kBackMaxU)) : 0;
    L.order = al256(sizeof(int) * V * fwd_chunks((int)B) * 2);
    L.det = al256(sizeof(DetEntry) * (size_t)back_ch * V * det_row((int)B));
    L.part = al256(sizeof(float) * (size_t)back_ch * nj);
    return L;
}

size_t geometry_bytes(const mbmd_geometry& g, int prefix_mat, int back_ch) {
    return layout_of(g, prefix_mat, back_ch).total();
}

void place_geometry(const mbmd_geometry& g, const GeomHost& h, GeomTables& t, char* base, int prefix_mat,
                    int back_ch, hipStream_t s) {
    t.g = g;
    t.V = g.n_views;
    t.B = g.n_bins;
    t.nx = g.nx;
    t.ny = g.ny;
    t.n_frame_views[0] = h.n_frame_views[0];
    t.n_frame_views[1] = h.n_frame_views[1];
    const GeomLayout L = layout_of(g, prefix_mat, back_ch);
    MBMD_REQUIRE(h.order.size() * sizeof(int) <= L.order, MBMD_ERR_ARG, "forward item table larger than its layout");
    // the back projector addresses the detector prefix with 32-bit buffer offsets
    MBMD_REQUIRE(L.det < (size_t(1) << 31), MBMD_ERR_SHAPE, "too many views x bins x channels for a back projection");
    MBMD_REQUIRE((reinterpret_cast<uintptr_t>(base) & 255) == 0, MBMD_ERR_ARG, "geometry memory must be 256-byte aligned");
    MBMD_HIP(hipGetDevice(&t.device));
    t.prefix_mat = prefix_mat;
    t.back_ch = back_ch;
    t.back_line_q = g.nx > g.ny ? g.nx : g.ny;
    char* p = base;
    t.view = reinterpret_cast<ViewParams*>(p);
    p += L.view;
    t.bound = reinterpret_cast<float2*>(p);
    p += L.bound;
    t.path = reinterpret_cast<float*>(p);
    p += L.path;
    t.frame_views = reinterpret_cast<int*>(p);
    p += L.fv;
    t.prefix = prefix_mat ? reinterpret_cast<float*>(p) : nullptr;
    p += L.pre;
    t.back_line = back_ch ? reinterpret_cast<float4*>(p) : nullptr;
    p += L.line;
    t.fwd_order = reinterpret_cast<int*>(p);
    p += L.order;
    t.det_prefix = back_ch ? reinterpret_cast<DetEntry*>(p) : nullptr;
    p += L.det;
    t.back_part = back_ch ? reinterpret_cast<float*>(p) : nullptr;
    for (int i = 0; i <= kMaxBackCh; ++i) t.back_variant[i] = -1;
    const char* fv = std::getenv("MBMD_BACK_VARIANT");
    t.forced_back = fv && fv[0] ? std::atoi(fv) : -1;
    // stream-ordered uploads; the caller keeps h alive until the stream has run them
    MBMD_HIP(hipMemcpyAsync(t.view, h.vp.data(), sizeof(ViewParams) * h.vp.size(), hipMemcpyHostToDevice, s));
    MBMD_HIP(hipMemcpyAsync(t.bound, h.bound.data(), sizeof(float2) * h.bound.size(), hipMemcpyHostToDevice, s));
    MBMD_HIP(hipMemcpyAsync(t.path, h.path.data(), sizeof(float) * h.path.size(), hipMemcpyHostToDevice, s));
    MBMD_HIP(hipMemcpyAsync(t.frame_views, h.fv.data(), sizeof(int) * h.fv.size(), hipMemcpyHostToDevice, s));
    if (back_ch)
        MBMD_HIP(hipMemcpyAsync(t.back_line, h.line.data(), sizeof(float4) * h.line.size(), hipMemcpyHostToDevice, s));
    MBMD_HIP(hipMemcpyAsync(t.fwd_order, h.order.data(), sizeof(int) * h.order.size(), hipMemcpyHostToDevice, s));
}

void build_geometry(const mbmd_geometry& g, GeomTables& t, int prefix_mat, int back_ch) {
    GeomHost h;
    build_geometry_host(g, h);
    char* base = nullptr;
    MBMD_HIP(hipMalloc(&base, geometry_bytes(g, prefix_mat, back_ch)));
    t.mem = base;
    try {
        place_geometry(g, h, t, base, prefix_mat, back_ch, nullptr);
        MBMD_HIP(hipStreamSynchronize(nullptr));        // h goes out of scope
    } catch (...) {
        (void)hipFree(base);
        t.mem = nullptr;
        throw;
    }
}

void free_geometry(GeomTables& t) {
    if (t.mem) (void)hipFree(t.mem);
    t.mem = nullptr;
}

namespace {
// Cached tables of the standalone projector calls, one entry per (geometry,
// device, stream): every stream has its own scratch, so calls on different
// streams do not race.  At most kCacheEntries entries; the least recently used
// one is freed first (hipFree waits for the device).
constexpr size_t kCacheEntries = 16;
struct CacheEntry {
    GeomTables* t;
    unsigned long long last_use;
};
std::mutex g_cache_mu;
std::map<std::string, CacheEntry> g_cache;
unsigned long long g_cache_clock = 0;
}  // namespace

GeomTables& cached_geometry(const mbmd_geometry& g, int prefix_mat, int back_ch, hipStream_t s) {
    int dev = 0;
    MBMD_HIP(hipGetDevice(&dev));
    // key from the fields (the struct has padding bytes), the device and the stream
    const double f[] = {(double)g.kind, (double)g.nx, (double)g.ny, g.dx, g.dy, (double)g.n_views,
                        g.theta0, g.dtheta, (double)g.n_bins, g.du, g.u_offset, g.dso, g.dsd,
                        (double)dev};
    const uintptr_t sid = reinterpret_cast<uintptr_t>(s);
    std::string key(reinterpret_cast<const char*>(f), sizeof(f));
    key.append(reinterpret_cast<const char*>(&sid), sizeof(sid));
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end() && it->second.t->prefix_mat >= prefix_mat && it->second.t->back_ch >= back_ch) {
        it->second.last_use = ++g_cache_clock;
        return *it->second.t;
    }
    if (it != g_cache.end()) {
        // a larger scratch is needed: rebuild
        free_geometry(*it->second.t);
        delete it->second.t;
        g_cache.erase(it);
    }
    while (g_cache.size() >= kCacheEntries) {
        auto old = g_cache.begin();
        for (auto e = g_cache.begin(); e != g_cache.end(); ++e)
            if (e->second.last_use < old->second.last_use) old = e;
        free_geometry(*old->second.t);
        delete old->second.t;
        g_cache.erase(old);
    }
    GeomTables* t = new GeomTables();
    try {
        build_geometry(g, *t, prefix_mat < 1 ? 1 : prefix_mat, back_ch < 1 ? 1 : back_ch);
    } catch (...) {
        delete t;
        throw;
    }
    g_cache[key] = CacheEntry{t, ++g_cache_clock};
    return *t;
}

void clear_geometry_cache() {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (auto& e : g_cache) {
        free_geometry(*e.second.t);
        delete e.second.t;
    }
    g_cache.clear();
}

}  // namespace mbmd
