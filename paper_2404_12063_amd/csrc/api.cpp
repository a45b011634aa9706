// Host side of the C ABI declared in include/vpinn.h: argument and mesh
// validation, ownership of device buffers, and dispatch to the kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace vp {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

vpinn_status fail(vpinn_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

// selects the problem's device for the duration of a call
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// mesh checks on the host, before any device work.  det J of the bilinear map
// is affine in (xi, eta), so its minimum over the reference square is attained
// at a corner; at corner c it equals the cross product of the two edges
// leaving vertex c (up to the positive factor 1/4).
static vpinn_status validate_mesh(const vpinn_mesh *m) {
    if (!m || !m->xy || !m->quad) return fail(VPINN_E_INVALID, "mesh or its arrays are null");
    if (m->n_nodes < 4 || m->n_elem < 1) return fail(VPINN_E_INVALID, "mesh needs >= 4 nodes and >= 1 element");
    for (int64_t i = 0; i < 2 * m->n_nodes; ++i)
        if (!std::isfinite(m->xy[i])) return fail(VPINN_E_MESH, "vertex " + std::to_string(i / 2) + " is not finite");
    for (int64_t e = 0; e < m->n_elem; ++e) {
        double x[4], y[4];
        for (int c = 0; c < 4; ++c) {
            const int32_t id = m->quad[4 * e + c];
            if (id < 0 || id >= m->n_nodes)
                return fail(VPINN_E_MESH, "element " + std::to_string(e) + ": vertex id " + std::to_string(id) +
                                              " out of range");
            x[c] = m->xy[2 * (int64_t)id];
            y[c] = m->xy[2 * (int64_t)id + 1];
        }
        for (int c = 0; c < 4; ++c) {
            const int nx = (c + 1) & 3, pv = (c + 3) & 3;
            const double cross = (x[nx] - x[c]) * (y[pv] - y[c]) - (y[nx] - y[c]) * (x[pv] - x[c]);
            if (!(cross > 0.0))
                return fail(VPINN_E_MESH, "element " + std::to_string(e) +
                                              ": det J <= 0 at a corner (vertices must be counter-clockwise and "
                                              "the quadrilateral convex)");
        }
    }
    return VPINN_OK;
}

// True if every element is a translate of element 0 with its vertices in the same
// order: the bilinear map's non-constant coefficients agree (to 1e-12 relative), so
// the Jacobian field, and with it G, is the same for every element.
static bool congruent_elements(const vpinn_mesh *m) {
    auto coeffs = [&](int64_t e, double c[6]) {
        double x[4], y[4];
        for (int k = 0; k < 4; ++k) {
            const int64_t id = m->quad[4 * e + k];
            x[k] = m->xy[2 * id];
            y[k] = m->xy[2 * id + 1];
        }
        c[0] = 0.25 * (-x[0] + x[1] + x[2] - x[3]);
        c[1] = 0.25 * (-x[0] - x[1] + x[2] + x[3]);
        c[2] = 0.25 * (x[0] - x[1] + x[2] - x[3]);
        c[3] = 0.25 * (-y[0] + y[1] + y[2] - y[3]);
        c[4] = 0.25 * (-y[0] - y[1] + y[2] + y[3]);
        c[5] = 0.25 * (y[0] - y[1] + y[2] - y[3]);
    };
    double c0[6], c[6], scale = 0.0;
    coeffs(0, c0);
    for (double v : c0) scale = std::max(scale, std::fabs(v));
    for (int64_t e = 1; e < m->n_elem; ++e) {
        coeffs(e, c);
        for (int i = 0; i < 6; ++i)
            if (std::fabs(c[i] - c0[i]) > 1e-12 * scale) return false;
    }
    return true;
}

// Shared GLL points from the mesh topology: a vertex point is keyed by its vertex id,
// an edge point by the edge's vertex pair and its position counted from the
// lower-numbered vertex (the GLL nodes are symmetric, so both elements place it at
// the same physical point), an element-interior point is its own.  Distinct points
// are numbered in order of first appearance over slots s = e nq + q.
static vpinn_status shared_point_map(const vpinn_mesh *m, int n, std::vector<int32_t> &umap, int64_t &n_uniq) {
    const int nq = n * n;
    const int64_t n_slots = m->n_elem * nq;
    if (n_slots > INT32_MAX) return fail(VPINN_E_UNSUPPORTED, "too many quadrature points for shared points");
    umap.assign((size_t)n_slots, -1);
    std::vector<int32_t> vid((size_t)m->n_nodes, -1);
    std::unordered_map<uint64_t, int64_t> edge_base;  // edge -> first of its n - 2 point ids in edge_ids
    std::vector<int32_t> edge_ids;
    int64_t next = 0;
    // corners of the reference square in vertex order, and the edges (from vertex, to vertex)
    // with the local index walked from the first: bottom (0 -> 1, i), right (1 -> 2, j),
    // top (3 -> 2, i), left (0 -> 3, j)
    for (int64_t e = 0; e < m->n_elem; ++e) {
        const int32_t *v = m->quad + 4 * e;
        for (int q = 0; q < nq; ++q) {
            const int i = q % n, j = q / n;
            const bool xi_end = i == 0 || i == n - 1, eta_end = j == 0 || j == n - 1;
            int32_t *slot = &umap[(size_t)(e * nq + q)];
            if (xi_end && eta_end) {
                const int c = (j == 0) ? (i == 0 ? 0 : 1) : (i == 0 ? 3 : 2);
                int32_t &id = vid[(size_t)v[c]];
                if (id < 0) id = (int32_t)next++;
                *slot = id;
            } else if (xi_end || eta_end) {
                int a, b, pos;
                if (j == 0) a = 0, b = 1, pos = i;
                else if (i == n - 1) a = 1, b = 2, pos = j;
                else if (j == n - 1) a = 3, b = 2, pos = i;
                else a = 0, b = 3, pos = j;
                int64_t va = v[a], vb = v[b];
                if (va > vb) {
                    std::swap(va, vb);
                    pos = n - 1 - pos;
                }
                const uint64_t key = (uint64_t)va * (uint64_t)m->n_nodes + (uint64_t)vb;
                auto it = edge_base.find(key);
                if (it == edge_base.end()) {
                    it = edge_base.emplace(key, (int64_t)edge_ids.size()).first;
                    edge_ids.resize(edge_ids.size() + (size_t)(n - 2), -1);
                }
                int32_t &id = edge_ids[(size_t)(it->second + pos - 1)];
                if (id < 0) id = (int32_t)next++;
                *slot = id;
            } else {
                *slot = (int32_t)next++;
            }
        }
    }
    n_uniq = next;
    return VPINN_OK;
}

static vpinn_status rebuild_points(vpinn_problem *p, const std::vector<float> &bxy, const std::vector<float> &bg,
                                   const std::vector<float> &sxy, const std::vector<float> &sd, int64_t nb,
                                   int64_t ns) {
    DevBuf npts, ntgt;
    const int64_t total = p->n_pts + nb + ns;
    VP_HIP(npts.reserve(sizeof(float2) * total));
    VP_HIP(hipMemcpy(npts.ptr, p->pts.ptr, sizeof(float2) * p->n_pts, hipMemcpyDeviceToDevice));
    if (nb) VP_HIP(hipMemcpy(npts.as<float2>() + p->n_pts, bxy.data(), sizeof(float2) * nb, hipMemcpyHostToDevice));
    if (ns)
        VP_HIP(hipMemcpy(npts.as<float2>() + p->n_pts + nb, sxy.data(), sizeof(float2) * ns, hipMemcpyHostToDevice));
    if (nb + ns) {
        VP_HIP(ntgt.reserve(sizeof(float) * (nb + ns)));
        if (nb) VP_HIP(hipMemcpy(ntgt.ptr, bg.data(), sizeof(float) * nb, hipMemcpyHostToDevice));
        if (ns) VP_HIP(hipMemcpy(ntgt.as<float>() + nb, sd.data(), sizeof(float) * ns, hipMemcpyHostToDevice));
    }
    std::swap(p->pts.ptr, npts.ptr);
    std::swap(p->pts.bytes, npts.bytes);
    std::swap(p->tgt.ptr, ntgt.ptr);
    std::swap(p->tgt.bytes, ntgt.bytes);
    p->n_bnd = nb;
    p->n_sen = ns;
    ++p->gen;
    return VPINN_OK;
}

}  // namespace vp

// host copies of the boundary and sensor sets (so either can be replaced alone)
struct vpinn_point_sets {
    std::vector<float> bxy, bg, sxy, sd;
};

namespace {
struct ProblemWithSets : vpinn_problem {
    vpinn_point_sets sets;
};

vpinn_status convert_set(int64_t n, const double *xy, const double *val, std::vector<float> &oxy,
                         std::vector<float> &oval, const char *what) {
    if (n < 0) return vp::fail(VPINN_E_INVALID, std::string(what) + ": negative count");
    if (n > 0 && (!xy || !val)) return vp::fail(VPINN_E_INVALID, std::string(what) + ": null array");
    oxy.resize(2 * n);
    oval.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(xy[2 * i]) || !std::isfinite(xy[2 * i + 1]) || !std::isfinite(val[i]))
            return vp::fail(VPINN_E_INVALID, std::string(what) + ": point " + std::to_string(i) + " is not finite");
        oxy[2 * i] = (float)xy[2 * i];
        oxy[2 * i + 1] = (float)xy[2 * i + 1];
        oval[i] = (float)val[i];
    }
    return VPINN_OK;
}
}  // namespace

extern "C" {

int64_t vpinn_n_params(int32_t width, int32_t n_hidden) {
    if (width < 1 || n_hidden < 1) return -1;
    return (int64_t)width * 2 + width + (int64_t)(n_hidden - 1) * ((int64_t)width * width + width) + width + 1;
}

int64_t vpinn_n_params_out(int32_t width, int32_t n_hidden, int32_t n_outputs) {
    if (n_outputs < 1 || n_outputs > 2) return -1;
    const int64_t n1 = vpinn_n_params(width, n_hidden);
    return n1 < 0 ? -1 : n1 + (int64_t)(n_outputs - 1) * (width + 1);
}

const char *vpinn_last_error(void) { return vp::g_err.c_str(); }

vpinn_status vpinn_set_shared_points(vpinn_problem *p, const vpinn_mesh *mesh, int32_t enable) {
    using namespace vp;
    if (!p) return fail(VPINN_E_INVALID, "problem is null");
    if (enable != 0 && enable != 1) return fail(VPINN_E_INVALID, "enable must be 0 or 1");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the problem's device");
    if (!enable) {
        p->n_uniq = 0;
        p->umap.release();
        p->usoff.release();
        p->uslot.release();
        p->upts.release();
        ++p->gen;
        return VPINN_OK;
    }
    if (!mesh || !mesh->xy || !mesh->quad) return fail(VPINN_E_INVALID, "mesh is null");
    if (mesh->n_elem != p->n_elem) return fail(VPINN_E_INVALID, "the mesh's element count differs from the problem's");
    for (int64_t k = 0; k < 4 * mesh->n_elem; ++k)
        if (mesh->quad[k] < 0 || mesh->quad[k] >= mesh->n_nodes)
            return fail(VPINN_E_MESH, "element " + std::to_string(k / 4) + ": vertex index out of range");
    std::vector<int32_t> umap;
    int64_t n_uniq = 0;
    vpinn_status st = shared_point_map(mesh, p->n, umap, n_uniq);
    if (st) return st;
    // the problem's own points: the first slot of each distinct point gives its
    // coordinates, and every other slot must lie on it
    std::vector<float2> pts((size_t)p->n_pts), upts((size_t)n_uniq);
    VP_HIP(hipMemcpy(pts.data(), p->pts.ptr, sizeof(float2) * p->n_pts, hipMemcpyDeviceToHost));
    std::vector<int32_t> first((size_t)n_uniq, -1), count((size_t)n_uniq + 1, 0);
    for (int64_t s = 0; s < p->n_pts; ++s) {
        const int32_t u = umap[(size_t)s];
        if (first[(size_t)u] < 0) {
            first[(size_t)u] = (int32_t)s;
            upts[(size_t)u] = pts[(size_t)s];
        } else {
            const float2 a = pts[(size_t)s], b = upts[(size_t)u];
            const float tol = 1e-6f * std::max(1.0f, std::max(std::fabs(b.x), std::fabs(b.y)));
            if (std::fabs(a.x - b.x) > tol || std::fabs(a.y - b.y) > tol)
                return fail(VPINN_E_MESH, "element " + std::to_string(s / p->nq) +
                                              ": a shared quadrature point does not match its partner (not the "
                                              "problem's mesh?)");
        }
        ++count[(size_t)u + 1];
    }
    for (int64_t u = 0; u < n_uniq; ++u) count[(size_t)u + 1] += count[(size_t)u];
    std::vector<int32_t> slots((size_t)p->n_pts), fill(count.begin(), count.end() - 1);
    for (int64_t s = 0; s < p->n_pts; ++s) slots[(size_t)fill[(size_t)umap[(size_t)s]]++] = (int32_t)s;
    DevBuf dm, doff, dsl, dpts;
    VP_HIP(dm.reserve(sizeof(int32_t) * p->n_pts));
    VP_HIP(doff.reserve(sizeof(int32_t) * (n_uniq + 1)));
    VP_HIP(dsl.reserve(sizeof(int32_t) * p->n_pts));
    VP_HIP(dpts.reserve(sizeof(float2) * n_uniq));
    VP_HIP(hipMemcpy(dm.ptr, umap.data(), sizeof(int32_t) * p->n_pts, hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(doff.ptr, count.data(), sizeof(int32_t) * (n_uniq + 1), hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(dsl.ptr, slots.data(), sizeof(int32_t) * p->n_pts, hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(dpts.ptr, upts.data(), sizeof(float2) * n_uniq, hipMemcpyHostToDevice));
    p->umap = std::move(dm);
    p->usoff = std::move(doff);
    p->uslot = std::move(dsl);
    p->upts = std::move(dpts);
    p->n_uniq = n_uniq;
    ++p->gen;
    return VPINN_OK;
}

static vpinn_status assemble_operator(const vpinn_mesh *mesh, int32_t quad_order, int32_t test_order, double diff,
                                      double conv_x, double conv_y, bool vardiff, bool matfree,
                                      const vpinn_forcing *forcing, void *stream, vpinn_problem **out) {
    using namespace vp;
    if (!out) return fail(VPINN_E_INVALID, "out is null");
    *out = nullptr;
    if (!std::isfinite(diff) || !(diff > 0.0) || !std::isfinite(conv_x) || !std::isfinite(conv_y))
        return fail(VPINN_E_INVALID, "the diffusion coefficient must be finite and > 0, the velocity finite");
    if (quad_order < 2 || quad_order > VPINN_MAX_QUAD_ORDER)
        return fail(VPINN_E_INVALID, "quad_order must be in 2.." + std::to_string(VPINN_MAX_QUAD_ORDER));
    if (test_order < 1 || test_order > VPINN_MAX_TEST_ORDER)
        return fail(VPINN_E_INVALID, "test_order must be in 1.." + std::to_string(VPINN_MAX_TEST_ORDER));
    if (matfree && quad_order > 16)
        return fail(VPINN_E_UNSUPPORTED, "the matrix-free contraction needs quad_order <= 16");
    if (!forcing) return fail(VPINN_E_INVALID, "forcing is null");
    if (forcing->kind == VPINN_FORCING_CALLBACK) {
        if (!forcing->fn) return fail(VPINN_E_INVALID, "callback forcing without a function");
    } else if (forcing->kind == VPINN_FORCING_SINSIN) {
        if (!std::isfinite(forcing->amp) || !std::isfinite(forcing->kx) || !std::isfinite(forcing->ky))
            return fail(VPINN_E_NONFINITE, "forcing coefficients are not finite");
    } else {
        return fail(VPINN_E_INVALID, "unknown forcing kind");
    }
    vpinn_status st = validate_mesh(mesh);
    if (st) return st;
    const int64_t nq = (int64_t)quad_order * quad_order, ntest = (int64_t)test_order * test_order;
    const int64_t n_elem = mesh->n_elem;
    if (n_elem > (int64_t(1) << 40) / (matfree ? nq : nq * ntest))
        return fail(VPINN_E_INVALID, "tensor size overflows");

    ProblemWithSets *p = new (std::nothrow) ProblemWithSets();
    if (!p) return fail(VPINN_E_NOMEM, "host allocation failed");
    auto bail = [&](vpinn_status s) {
        delete p;
        return s;
    };
    if (hipGetDevice(&p->device) != hipSuccess) return bail(fail(VPINN_E_DEVICE, "no HIP device"));
    p->n_elem = n_elem;
    p->n = quad_order;
    p->nt = test_order;
    p->nq = (int)nq;
    p->ntest = (int)ntest;
    p->n_pts = n_elem * nq;
    if (vardiff) {
        // nothing folded: G stays the diffusion weights and M is kept for the convection term
        p->vardiff = true;
        p->vd_bx = conv_x;
        p->vd_by = conv_y;
    } else {
        p->diff = diff;
        p->conv_x = conv_x;
        p->conv_y = conv_y;
    }
    p->matfree = matfree;
    p->shared_g = !vardiff && !matfree && congruent_elements(mesh);
    hipStream_t s = (hipStream_t)stream;
    const size_t gbytes = sizeof(float) * (size_t)((p->shared_g ? 1 : n_elem) * ntest * nq);
    bool ok = p->F.reserve(sizeof(float) * n_elem * ntest) == hipSuccess &&
              p->pts.reserve(sizeof(float2) * p->n_pts) == hipSuccess;
    if (matfree)
        ok = ok && p->geo.reserve(sizeof(float) * 8 * (size_t)n_elem) == hipSuccess &&
             p->tab.reserve(sizeof(float) * (size_t)(2 * quad_order + 2 * quad_order * test_order)) == hipSuccess;
    else
        ok = ok && p->Gx.reserve(gbytes) == hipSuccess && p->Gy.reserve(gbytes) == hipSuccess &&
             (!vardiff || p->M.reserve(sizeof(float) * (size_t)(n_elem * ntest * nq)) == hipSuccess);
    if (!ok) return bail(fail(VPINN_E_NOMEM, "device allocation of the assembled tensors failed"));
    DevBuf d_nodes, d_quad;
    if (d_nodes.reserve(sizeof(double) * 2 * mesh->n_nodes) != hipSuccess ||
        d_quad.reserve(sizeof(int32_t) * 4 * n_elem) != hipSuccess)
        return bail(fail(VPINN_E_NOMEM, "device allocation of the mesh failed"));
    if (hipMemcpy(d_nodes.ptr, mesh->xy, sizeof(double) * 2 * mesh->n_nodes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_quad.ptr, mesh->quad, sizeof(int32_t) * 4 * n_elem, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(VPINN_E_DEVICE, "mesh upload failed"));
    st = assemble_device(p, d_nodes.as<double>(), mesh->n_nodes, d_quad.as<int32_t>(), forcing, s);
    if (st) return bail(st);
    *out = p;
    return VPINN_OK;
}

vpinn_status vpinn_assemble(const vpinn_mesh *mesh, int32_t quad_order, int32_t test_order,
                            const vpinn_forcing *forcing, void *stream, vpinn_problem **out) {
    return assemble_operator(mesh, quad_order, test_order, 1.0, 0.0, 0.0, false, false, forcing, stream, out);
}

vpinn_status vpinn_assemble_matrix_free(const vpinn_mesh *mesh, int32_t quad_order, int32_t test_order, double eps,
                                        double bx, double by, int32_t variable_diffusion,
                                        const vpinn_forcing *forcing, void *stream, vpinn_problem **out) {
    if (variable_diffusion != 0 && variable_diffusion != 1) {
        if (out) *out = nullptr;
        return vp::fail(VPINN_E_INVALID, "variable_diffusion must be 0 or 1");
    }
    return assemble_operator(mesh, quad_order, test_order, variable_diffusion ? 1.0 : eps, bx, by,
                             variable_diffusion == 1, true, forcing, stream, out);
}

vpinn_status vpinn_assemble_vardiff(const vpinn_mesh *mesh, int32_t quad_order, int32_t test_order, double bx,
                                    double by, const vpinn_forcing *forcing, void *stream, vpinn_problem **out) {
    return assemble_operator(mesh, quad_order, test_order, 1.0, bx, by, true, false, forcing, stream, out);
}

vpinn_status vpinn_assemble_cd2d(const vpinn_mesh *mesh, int32_t quad_order, int32_t test_order, double eps,
                                 double bx, double by, const vpinn_forcing *forcing, void *stream,
                                 vpinn_problem **out) {
    return assemble_operator(mesh, quad_order, test_order, eps, bx, by, false, false, forcing, stream, out);
}

vpinn_status vpinn_set_boundary(vpinn_problem *pp, int64_t n, const double *xy, const double *g) {
    using namespace vp;
    if (!pp) return fail(VPINN_E_INVALID, "problem is null");
    auto *p = static_cast<ProblemWithSets *>(pp);
    std::vector<float> bxy, bg;
    vpinn_status st = convert_set(n, xy, g, bxy, bg, "boundary");
    if (st) return st;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the problem's device");
    st = rebuild_points(p, bxy, bg, p->sets.sxy, p->sets.sd, n, p->n_sen);
    if (st) return st;
    p->sets.bxy.swap(bxy);
    p->sets.bg.swap(bg);
    return VPINN_OK;
}

vpinn_status vpinn_set_sensors(vpinn_problem *pp, int64_t n, const double *xy, const double *d) {
    using namespace vp;
    if (!pp) return fail(VPINN_E_INVALID, "problem is null");
    auto *p = static_cast<ProblemWithSets *>(pp);
    std::vector<float> sxy, sd;
    vpinn_status st = convert_set(n, xy, d, sxy, sd, "sensors");
    if (st) return st;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the problem's device");
    st = rebuild_points(p, p->sets.bxy, p->sets.bg, sxy, sd, p->n_bnd, n);
    if (st) return st;
    p->sets.sxy.swap(sxy);
    p->sets.sd.swap(sd);
    return VPINN_OK;
}

vpinn_status vpinn_get_info(const vpinn_problem *p, vpinn_problem_info *info) {
    using namespace vp;
    if (!p || !info) return fail(VPINN_E_INVALID, "null argument");
    info->n_elem = p->n_elem;
    info->n_quad = p->nq;
    info->n_test = p->ntest;
    info->n_points = p->n_pts;
    info->n_boundary = p->n_bnd;
    info->n_sensors = p->n_sen;
    info->quad_order = p->n;
    info->test_order = p->nt;
    info->diffusion = p->vardiff ? 0.0 : p->diff;
    info->velocity_x = p->vardiff ? p->vd_bx : p->conv_x;
    info->velocity_y = p->vardiff ? p->vd_by : p->conv_y;
    info->shared_premultiplier = p->shared_g ? 1 : 0;
    info->variable_diffusion = p->vardiff ? 1 : 0;
    info->matrix_free = p->matfree ? 1 : 0;
    info->n_distinct_points = p->n_uniq;
    return VPINN_OK;
}

vpinn_status vpinn_read_tensor(const vpinn_problem *p, int32_t which, float *host_dst, int64_t count) {
    using namespace vp;
    if (!p || !host_dst) return fail(VPINN_E_INVALID, "null argument");
    const void *src = nullptr;
    int64_t want = 0;
    if (p->matfree && (which == VPINN_TENSOR_GX || which == VPINN_TENSOR_GY || which == VPINN_TENSOR_M))
        return fail(VPINN_E_INVALID, "a matrix-free problem stores no G or M");
    switch (which) {
    case VPINN_TENSOR_GX: src = p->Gx.ptr; want = p->n_elem * p->ntest * p->nq; break;
    case VPINN_TENSOR_GY: src = p->Gy.ptr; want = p->n_elem * p->ntest * p->nq; break;
    case VPINN_TENSOR_F: src = p->F.ptr; want = p->n_elem * p->ntest; break;
    case VPINN_TENSOR_X: src = p->pts.ptr; want = 2 * p->n_pts; break;
    case VPINN_TENSOR_M:
        if (!p->vardiff) return fail(VPINN_E_INVALID, "M is kept only for problems from vpinn_assemble_vardiff");
        src = p->M.ptr;
        want = p->n_elem * p->ntest * p->nq;
        break;
    default: return fail(VPINN_E_INVALID, "unknown tensor id");
    }
    if (count != want) return fail(VPINN_E_INVALID, "count must be " + std::to_string(want));
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the problem's device");
    if (p->shared_g && (which == VPINN_TENSOR_GX || which == VPINN_TENSOR_GY)) {
        // one stored premultiplier, replicated for every element on the host
        const int64_t per = (int64_t)p->ntest * p->nq;
        VP_HIP(hipMemcpy(host_dst, src, sizeof(float) * per, hipMemcpyDeviceToHost));
        for (int64_t e = 1; e < p->n_elem; ++e) std::copy(host_dst, host_dst + per, host_dst + e * per);
        return VPINN_OK;
    }
    VP_HIP(hipMemcpy(host_dst, src, sizeof(float) * count, hipMemcpyDeviceToHost));
    return VPINN_OK;
}

static vpinn_status check_cfg(const vpinn_loss_cfg *cfg) {
    using namespace vp;
    if (!cfg) return fail(VPINN_E_INVALID, "cfg is null");
    if (cfg->n_hidden < 1 || cfg->n_hidden > VPINN_MAX_HIDDEN)
        return fail(VPINN_E_UNSUPPORTED, "n_hidden must be in 1.." + std::to_string(VPINN_MAX_HIDDEN));
    if (cfg->width < 1 || cfg->width > VPINN_MAX_WIDTH)
        return fail(VPINN_E_UNSUPPORTED, "width must be in 1.." + std::to_string(VPINN_MAX_WIDTH));
    if (cfg->loss_norm != VPINN_NORM_TEST && cfg->loss_norm != VPINN_NORM_ELEM)
        return fail(VPINN_E_INVALID, "unknown loss_norm");
    if (cfg->path != VPINN_PATH_FUSED && cfg->path != VPINN_PATH_PLAIN) return fail(VPINN_E_INVALID, "unknown path");
    if (!std::isfinite(cfg->tau) || !std::isfinite(cfg->gamma) || cfg->tau < 0 || cfg->gamma < 0)
        return fail(VPINN_E_INVALID, "tau and gamma must be finite and >= 0");
    if (cfg->n_outputs < 0 || cfg->n_outputs > 2) return fail(VPINN_E_INVALID, "n_outputs must be 0, 1 or 2");
    return VPINN_OK;
}

// the network's outputs must match the operator: two (u, eps) for space-dependent
// diffusion, on the fused path, with a trainable scalar eps excluded
static vpinn_status check_outputs(const vpinn_problem *p, const vpinn_loss_cfg *cfg, bool scalar_eps) {
    using namespace vp;
    const bool two = cfg->n_outputs == 2;
    if (two != p->vardiff)
        return fail(VPINN_E_INVALID, p->vardiff ? "a space-dependent diffusion problem needs cfg->n_outputs = 2"
                                                : "cfg->n_outputs = 2 needs a problem from vpinn_assemble_vardiff");
    if (two && cfg->path != VPINN_PATH_FUSED)
        return fail(VPINN_E_UNSUPPORTED, "space-dependent diffusion runs on the fused path only");
    if (two && scalar_eps)
        return fail(VPINN_E_INVALID, "a space-dependent diffusion problem takes no scalar eps");
    if (p->matfree && cfg->path != VPINN_PATH_FUSED)
        return fail(VPINN_E_UNSUPPORTED, "a matrix-free problem runs on the fused path only");
    return VPINN_OK;
}

vpinn_status vpinn_loss_and_grad(vpinn_problem *p, const vpinn_loss_cfg *cfg, const float *d_params,
                                 const float *d_eps, float *d_loss, float *d_grad, float *d_grad_eps, void *stream) {
    using namespace vp;
    if (!p || !d_params) return fail(VPINN_E_INVALID, "problem or params is null");
    if (!d_loss && !d_grad && !d_grad_eps) return fail(VPINN_E_INVALID, "nothing to compute");
    if ((d_eps || d_grad_eps) && p->folded())
        return fail(VPINN_E_INVALID, "a problem assembled with fixed convection-diffusion coefficients takes no eps");
    vpinn_status st = check_cfg(cfg);
    if (st) return st;
    st = check_outputs(p, cfg, d_eps || d_grad_eps);
    if (st) return st;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the problem's device");
    hipStream_t s = (hipStream_t)stream;
    if (cfg->path == VPINN_PATH_PLAIN) return plain_loss_grad(p, cfg, d_params, d_eps, d_loss, d_grad, d_grad_eps,
                                                              nullptr, s);
    return fused_loss_grad(p, cfg, d_params, d_eps, d_loss, d_grad, d_grad_eps, s);
}

vpinn_status vpinn_residual(vpinn_problem *p, const vpinn_loss_cfg *cfg, const float *d_params, const float *d_eps,
                            float *d_R, void *stream) {
    using namespace vp;
    if (!p || !d_params || !d_R) return fail(VPINN_E_INVALID, "null argument");
    if (d_eps && p->folded())
        return fail(VPINN_E_INVALID, "a problem assembled with fixed convection-diffusion coefficients takes no eps");
    vpinn_status st = check_cfg(cfg);
    if (st) return st;
    if (p->vardiff || cfg->n_outputs == 2)
        return fail(VPINN_E_UNSUPPORTED, "vpinn_residual (plain path) has no space-dependent diffusion");
    if (p->matfree) return fail(VPINN_E_UNSUPPORTED, "vpinn_residual (plain path) needs the stored G");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the problem's device");
    return plain_loss_grad(p, cfg, d_params, d_eps, nullptr, nullptr, nullptr, d_R, (hipStream_t)stream);
}

vpinn_status vpinn_eval_network_heads(int32_t width, int32_t n_hidden, int32_t n_outputs, const float *d_params,
                                      int64_t n, const float *d_xy, float *d_u, float *d_ux, float *d_uy, float *d_e,
                                      void *stream) {
    using namespace vp;
    if (width < 1 || width > VPINN_MAX_WIDTH || n_hidden < 1 || n_hidden > VPINN_MAX_HIDDEN)
        return fail(VPINN_E_UNSUPPORTED, "width or n_hidden out of range");
    if (n_outputs < 1 || n_outputs > 2) return fail(VPINN_E_INVALID, "n_outputs must be 1 or 2");
    if (d_e && n_outputs != 2) return fail(VPINN_E_INVALID, "d_e needs a network with two outputs");
    if (!d_params || (n > 0 && !d_xy) || n < 0) return fail(VPINN_E_INVALID, "null argument or negative n");
    return eval_mfma(n_hidden, width, n_outputs, d_params, n, reinterpret_cast<const float2 *>(d_xy), d_u, d_ux, d_uy,
                     d_e, (hipStream_t)stream);
}

static vpinn_status check_eval_error(int32_t width, int32_t n_hidden, int32_t n_outputs, int32_t output,
                                     const float *d_params, int64_t n, const float *d_xy, const float *d_ref,
                                     double *d_out) {
    using namespace vp;
    if (width < 1 || width > VPINN_MAX_WIDTH || n_hidden < 1 || n_hidden > VPINN_MAX_HIDDEN)
        return fail(VPINN_E_UNSUPPORTED, "width or n_hidden out of range");
    if (n_outputs < 1 || n_outputs > 2 || output < 0 || output >= n_outputs)
        return fail(VPINN_E_INVALID, "n_outputs must be 1 or 2 and output in 0 .. n_outputs - 1");
    if (!d_params || !d_xy || !d_ref || !d_out || n < 1) return fail(VPINN_E_INVALID, "null argument or n < 1");
    return VPINN_OK;
}

vpinn_status vpinn_eval_error_noalloc(int32_t width, int32_t n_hidden, int32_t n_outputs, int32_t output,
                                      const float *d_params, int64_t n, const float *d_xy, const float *d_ref,
                                      double *d_out, void *stream) {
    using namespace vp;
    vpinn_status st = check_eval_error(width, n_hidden, n_outputs, output, d_params, n, d_xy, d_ref, d_out);
    if (st) return st;
    if (n > VPINN_NOALLOC_MAX_POINTS)
        return fail(VPINN_E_INVALID, "n = " + std::to_string(n) + " exceeds the fixed workspace of " +
                                         std::to_string((int64_t)VPINN_NOALLOC_MAX_POINTS) +
                                         " points (VPINN_NOALLOC_MAX_POINTS): use vpinn_eval_error");
    float *pv = nullptr;
    double *part = nullptr;
    st = noalloc_workspace(&pv, &part);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    st = eval_mfma(n_hidden, width, n_outputs, d_params, n, reinterpret_cast<const float2 *>(d_xy),
                   output == 0 ? pv : nullptr, nullptr, nullptr, output == 1 ? pv : nullptr, s);
    if (st) return st;
    return error_stats(n, pv, d_ref, part, d_out, s);
}

vpinn_status vpinn_eval_error(int32_t width, int32_t n_hidden, int32_t n_outputs, int32_t output,
                              const float *d_params, int64_t n, const float *d_xy, const float *d_ref, double *d_out,
                              void *stream) {
    using namespace vp;
    vpinn_status cst = check_eval_error(width, n_hidden, n_outputs, output, d_params, n, d_xy, d_ref, d_out);
    if (cst) return cst;
    static thread_local DevBuf pbuf, part;
    static thread_local int ws_dev = -1;
    int dev = 0;
    VP_HIP(hipGetDevice(&dev));
    if (ws_dev != dev) {
        pbuf.release();
        part.release();
        ws_dev = dev;
    }
    VP_HIP(pbuf.reserve(sizeof(float) * (size_t)n));
    VP_HIP(part.reserve(sizeof(double) * 4 * 512));
    hipStream_t s = (hipStream_t)stream;
    const float2 *xy = reinterpret_cast<const float2 *>(d_xy);
    float *pv = pbuf.as<float>();
    vpinn_status st = eval_mfma(n_hidden, width, n_outputs, d_params, n, xy, output == 0 ? pv : nullptr, nullptr,
                                nullptr, output == 1 ? pv : nullptr, s);
    if (st) return st;
    return error_stats(n, pv, d_ref, part.as<double>(), d_out, s);
}

vpinn_status vpinn_eval_network(int32_t width, int32_t n_hidden, const float *d_params, int64_t n, const float *d_xy,
                                float *d_u, float *d_ux, float *d_uy, void *stream) {
    return vpinn_eval_network_heads(width, n_hidden, 1, d_params, n, d_xy, d_u, d_ux, d_uy, nullptr, stream);
}

vpinn_status vpinn_adam_step(int64_t n, float *d_params, const float *d_grad, float *d_m, float *d_v, int64_t step,
                             float lr, float beta1, float beta2, float eps, void *stream) {
    using namespace vp;
    if (n < 0 || step < 1) return fail(VPINN_E_INVALID, "n must be >= 0 and step >= 1");
    if (n > 0 && (!d_params || !d_grad || !d_m || !d_v)) return fail(VPINN_E_INVALID, "null argument");
    return adam_step(n, d_params, d_grad, d_m, d_v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

vpinn_status vpinn_batch_create(int32_t n, vpinn_problem *const *problems, const vpinn_loss_cfg *cfg,
                                vpinn_batch **out) {
    using namespace vp;
    if (!out) return fail(VPINN_E_INVALID, "out is null");
    *out = nullptr;
    if (n < 1 || !problems) return fail(VPINN_E_INVALID, "need n >= 1 problems");
    for (int i = 0; i < n; ++i) {
        if (!problems[i]) return fail(VPINN_E_INVALID, "problem " + std::to_string(i) + " is null");
        if (problems[i]->device != problems[0]->device)
            return fail(VPINN_E_INVALID, "all problems of a batch must live on one device");
    }
    vpinn_status st = check_cfg(cfg);
    if (st) return st;
    for (int i = 0; i < n; ++i) {
        st = check_outputs(problems[i], cfg, false);
        if (st) return fail(st, "problem " + std::to_string(i) + ": " + vpinn_last_error());
    }
    DeviceGuard dg(problems[0]->device);
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the problems' device");
    return batch_create(n, problems, cfg, out);
}

vpinn_status vpinn_batch_loss_and_grad(vpinn_batch *b, const float *d_params, const float *d_eps, float *d_losses,
                                       float *d_grads, float *d_grad_eps, void *stream) {
    using namespace vp;
    if (!b || !d_params) return fail(VPINN_E_INVALID, "batch or params is null");
    if (!d_losses && !d_grads && !d_grad_eps) return fail(VPINN_E_INVALID, "nothing to compute");
    DeviceGuard dg(batch_device(b));
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the batch's device");
    return batch_loss_and_grad(b, d_params, d_eps, d_losses, d_grads, d_grad_eps, (hipStream_t)stream);
}

static vpinn_status check_step_args(vpinn_batch *b, float *d_params, float *d_m, float *d_v, int64_t *d_step,
                                    float *d_eps, float *d_eps_m, float *d_eps_v) {
    using namespace vp;
    if (!b || !d_params || !d_m || !d_v || !d_step) return fail(VPINN_E_INVALID, "null argument");
    const int given = (d_eps != nullptr) + (d_eps_m != nullptr) + (d_eps_v != nullptr);
    if (given != 0 && given != 3) return fail(VPINN_E_INVALID, "d_eps, d_eps_m and d_eps_v go together");
    return VPINN_OK;
}

vpinn_status vpinn_batch_step(vpinn_batch *b, float *d_params, float *d_m, float *d_v, int64_t *d_step, float lr,
                              float beta1, float beta2, float eps, float *d_losses, float *d_eps, float *d_eps_m,
                              float *d_eps_v, void *stream) {
    using namespace vp;
    vpinn_status st = check_step_args(b, d_params, d_m, d_v, d_step, d_eps, d_eps_m, d_eps_v);
    if (st) return st;
    DeviceGuard dg(batch_device(b));
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the batch's device");
    return batch_step(b, d_params, d_m, d_v, d_step, lr, beta1, beta2, eps, d_losses, d_eps, d_eps_m, d_eps_v,
                      (hipStream_t)stream);
}

vpinn_status vpinn_batch_capture(vpinn_batch *b, float *d_params, float *d_m, float *d_v, int64_t *d_step, float lr,
                                 float beta1, float beta2, float eps, float *d_losses, float *d_eps, float *d_eps_m,
                                 float *d_eps_v, void *stream) {
    using namespace vp;
    vpinn_status st = check_step_args(b, d_params, d_m, d_v, d_step, d_eps, d_eps_m, d_eps_v);
    if (st) return st;
    DeviceGuard dg(batch_device(b));
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the batch's device");
    return batch_capture(b, d_params, d_m, d_v, d_step, lr, beta1, beta2, eps, d_losses, d_eps, d_eps_m, d_eps_v,
                         (hipStream_t)stream);
}

vpinn_status vpinn_batch_replay(vpinn_batch *b, void *stream) {
    using namespace vp;
    if (!b) return fail(VPINN_E_INVALID, "batch is null");
    DeviceGuard dg(batch_device(b));
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the batch's device");
    return batch_replay(b, (hipStream_t)stream);
}

vpinn_status vpinn_batch_get_tuning(const vpinn_batch *b, vpinn_tuning *out) {
    using namespace vp;
    if (!b || !out) return fail(VPINN_E_INVALID, "batch or out is null");
    return batch_get_tuning(b, out);
}

vpinn_status vpinn_batch_set_tuning(vpinn_batch *b, const vpinn_tuning *t) {
    using namespace vp;
    if (!b || !t) return fail(VPINN_E_INVALID, "batch or tuning is null");
    DeviceGuard dg(batch_device(b));
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the batch's device");
    return batch_set_tuning(b, t);
}

vpinn_status vpinn_batch_autotune(vpinn_batch *b, const float *d_params, int32_t reps, vpinn_tuning *best,
                                  void *stream) {
    using namespace vp;
    if (!b || !d_params) return fail(VPINN_E_INVALID, "batch or params is null");
    if (reps < 1 || reps > 100) return fail(VPINN_E_INVALID, "reps must be in 1..100");
    DeviceGuard dg(batch_device(b));
    if (!dg.ok) return fail(VPINN_E_DEVICE, "cannot select the batch's device");
    return batch_autotune(b, d_params, reps, best, (hipStream_t)stream);
}

vpinn_status vpinn_set_profile_events(vpinn_problem *p, void *const *events) {
    using namespace vp;
    if (!p) return fail(VPINN_E_INVALID, "problem is null");
    for (int i = 0; i < VPINN_PROFILE_EVENTS; ++i) p->prof[i] = events ? (hipEvent_t)events[i] : nullptr;
    return VPINN_OK;
}

vpinn_status vpinn_batch_set_profile_events(vpinn_batch *b, void *const *events) {
    using namespace vp;
    if (!b) return fail(VPINN_E_INVALID, "batch is null");
    batch_set_profile_events(b, events);
    return VPINN_OK;
}

void vpinn_batch_free(vpinn_batch *b) {
    if (!b) return;
    vp::DeviceGuard dg(vp::batch_device(b));
    vp::batch_destroy(b);
}

void vpinn_problem_free(vpinn_problem *p) {
    if (!p) return;
    vp::DeviceGuard dg(p->device);
    delete static_cast<ProblemWithSets *>(p);
}

}  // extern "C"
