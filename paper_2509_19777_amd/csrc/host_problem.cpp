// Host-side problem construction of libhplmm: Q1 assembly of a voxel solid
// (Sec. 2, Eqs. 1-4), grain/interface/contact-grid classification (Sec.
// 3.1-3.2) and mortar-node placement (Sec. 3.3, Eq. 7).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <stdexcept>

#include "common.h"

namespace hplmm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_text() { return g_last_error.c_str(); }

void fail(hplmm_status code, const std::string &msg) { throw Error{code, msg}; }

void NodeMap::build(int32_t nx_, int32_t ny_, int32_t nz_, const uint8_t *solid) {
    nx = nx_; ny = ny_; nz = nz_;
    NX = nx + 1; NY = ny + 1; NZ = nz + 1;
    std::vector<uint8_t> touched((size_t)(NX * NY * NZ), 0);
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                if (!solid[i + nx * (j + (int64_t)ny * k)]) continue;
                for (int c = 0; c < 8; ++c)
                    touched[(size_t)lat(i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1))] = 1;
            }
    lat2free.assign(touched.size(), -1);
    free2lat.clear();
    for (int64_t L = NX * NY; L < (int64_t)touched.size(); ++L)  // skip plane z = 0
        if (touched[(size_t)L]) {
            lat2free[(size_t)L] = (int32_t)free2lat.size();
            free2lat.push_back(L);
        }
}

// K_ab,ij = int lam dNa/dx_i dNb/dx_j + mu dNa/dx_j dNb/dx_i + mu d_ij grad Na . grad Nb
// over the unit cube (isotropic C of Eq. 3), with E = 1; two Gauss points per
// direction integrate the bilinear-in-each-direction integrand exactly.
void q1_element_stiffness(double nu, double K[24][24]) {
    const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double mu = 1.0 / (2.0 * (1.0 + nu));
    const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
    for (int r = 0; r < 24; ++r)
        for (int s = 0; s < 24; ++s) K[r][s] = 0.0;
    for (int qz = 0; qz < 2; ++qz)
        for (int qy = 0; qy < 2; ++qy)
            for (int qx = 0; qx < 2; ++qx) {
                const double p[3] = {g[qx], g[qy], g[qz]};
                double grad[8][3];
                for (int a = 0; a < 8; ++a) {
                    double f[3], s[3];
                    for (int d = 0; d < 3; ++d) {
                        const int on = (a >> d) & 1;
                        f[d] = on ? p[d] : 1.0 - p[d];
                        s[d] = on ? 1.0 : -1.0;
                    }
                    grad[a][0] = s[0] * f[1] * f[2];
                    grad[a][1] = f[0] * s[1] * f[2];
                    grad[a][2] = f[0] * f[1] * s[2];
                }
                const double w = 0.125;
                for (int a = 0; a < 8; ++a)
                    for (int b = 0; b < 8; ++b) {
                        const double dd = grad[a][0] * grad[b][0] + grad[a][1] * grad[b][1] +
                                          grad[a][2] * grad[b][2];
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) {
                                double v = lam * (grad[a][i] * grad[b][j]) +
                                           mu * (grad[a][j] * grad[b][i]);
                                if (i == j) v += mu * dd;
                                K[3 * a + i][3 * b + j] += w * v;
                            }
                    }
            }
}

static void check_dims(int32_t nx, int32_t ny, int32_t nz) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || (int64_t)nx * ny * nz > (int64_t)1 << 31)
        fail(HPLMM_E_ARG, "voxel dimensions must be positive and below 2^31 voxels");
}

}  // namespace hplmm

using namespace hplmm;

extern "C" const char *hplmm_last_error(void) { return last_error_text(); }

extern "C" hplmm_status hplmm_assemble_voxels(int32_t nx, int32_t ny, int32_t nz,
                                              const uint8_t *solid, const double *E, double nu,
                                              const double *traction, hplmm_system *out) {
    return guarded([&]() -> hplmm_status {
        if (!out) fail(HPLMM_E_ARG, "out is NULL");
        std::memset(out, 0, sizeof(*out));
        if (!solid || !E || !traction) fail(HPLMM_E_ARG, "NULL input array");
        check_dims(nx, ny, nz);
        if (!(nu > -1.0 && nu < 0.5)) fail(HPLMM_E_ARG, "Poisson ratio must lie in (-1, 0.5)");
        NodeMap nm;
        nm.build(nx, ny, nz, solid);
        const int64_t n = nm.n();
        if (n == 0) fail(HPLMM_E_ARG, "solid has no free nodes");
        double K[24][24];
        q1_element_stiffness(nu, K);
        // 27-point stencil accumulator per free node, slot = (dx+1) + 3(dy+1) + 9(dz+1)
        std::vector<double> stencil((size_t)n * 27 * 9, 0.0);
        std::vector<uint8_t> present((size_t)n * 27, 0);
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t vox = i + nx * (j + (int64_t)ny * k);
                    if (!solid[vox]) continue;
                    const double Ee = E[vox];
                    if (!std::isfinite(Ee) || Ee < 0.0) fail(HPLMM_E_ARG, "E must be finite and >= 0");
                    int32_t fid[8];
                    for (int a = 0; a < 8; ++a)
                        fid[a] = nm.lat2free[(size_t)nm.lat(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1))];
                    for (int a = 0; a < 8; ++a) {
                        if (fid[a] < 0) continue;
                        for (int b = 0; b < 8; ++b) {
                            if (fid[b] < 0) continue;
                            const int dx = (b & 1) - (a & 1), dy = ((b >> 1) & 1) - ((a >> 1) & 1),
                                      dz = ((b >> 2) & 1) - ((a >> 2) & 1);
                            const int slot = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
                            double *blk = &stencil[((size_t)fid[a] * 27 + slot) * 9];
                            present[(size_t)fid[a] * 27 + slot] = 1;
                            for (int r = 0; r < 3; ++r)
                                for (int c = 0; c < 3; ++c) blk[3 * r + c] += Ee * K[3 * a + r][3 * b + c];
                        }
                    }
                }
        int64_t nnzb = 0;
        for (size_t s = 0; s < present.size(); ++s) nnzb += present[s];
        out->n_nodes = n;
        out->nnzb = nnzb;
        out->row_ptr = (int64_t *)std::malloc(sizeof(int64_t) * (size_t)(n + 1));
        out->col_idx = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)nnzb);
        out->val = (double *)std::malloc(sizeof(double) * 9 * (size_t)nnzb);
        out->rhs = (double *)std::calloc((size_t)(3 * n), sizeof(double));
        out->node_xyz = (int32_t *)std::malloc(sizeof(int32_t) * 3 * (size_t)n);
        out->dof_fixed = nullptr;   // the clamped plane is eliminated, not flagged
        if (!out->row_ptr || !out->col_idx || !out->val || !out->rhs || !out->node_xyz) {
            hplmm_system_free(out);
            fail(HPLMM_E_OOM, "host allocation failed");
        }
        int64_t p = 0;
        for (int64_t v = 0; v < n; ++v) {
            out->row_ptr[v] = p;
            const int64_t L = nm.free2lat[(size_t)v];
            const int64_t i = L % nm.NX, j = (L / nm.NX) % nm.NY, k = L / (nm.NX * nm.NY);
            out->node_xyz[3 * v + 0] = (int32_t)i;
            out->node_xyz[3 * v + 1] = (int32_t)j;
            out->node_xyz[3 * v + 2] = (int32_t)k;
            for (int slot = 0; slot < 27; ++slot) {
                if (!present[(size_t)v * 27 + slot]) continue;
                const int dx = slot % 3 - 1, dy = (slot / 3) % 3 - 1, dz = slot / 9 - 1;
                const int32_t w = nm.lat2free[(size_t)nm.lat(i + dx, j + dy, k + dz)];
                out->col_idx[p] = w;
                std::memcpy(&out->val[9 * p], &stencil[((size_t)v * 27 + slot) * 9], 9 * sizeof(double));
                ++p;
            }
        }
        out->row_ptr[n] = p;
        // consistent traction load on the top face of the top solid layer
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                if (!solid[i + nx * (j + (int64_t)ny * (nz - 1))]) continue;
                for (int c = 0; c < 4; ++c) {
                    const int32_t f = nm.lat2free[(size_t)nm.lat(i + (c & 1), j + (c >> 1), nz)];
                    for (int d = 0; d < 3; ++d) out->rhs[3 * (int64_t)f + d] += 0.25 * traction[d];
                }
            }
        return HPLMM_OK;
    });
}

extern "C" void hplmm_system_free(hplmm_system *sys) {
    if (!sys) return;
    std::free(sys->row_ptr);
    std::free(sys->col_idx);
    std::free(sys->val);
    std::free(sys->rhs);
    std::free(sys->node_xyz);
    std::memset(sys, 0, sizeof(*sys));
}

namespace {

struct Labels {
    uint8_t n = 0;
    int32_t g[8];
    bool operator==(const Labels &o) const {
        if (n != o.n) return false;
        for (int i = 0; i < n; ++i)
            if (g[i] != o.g[i]) return false;
        return true;
    }
    void add(int32_t x) {
        for (int i = 0; i < n; ++i)
            if (g[i] == x) return;
        int p = n++;
        while (p > 0 && g[p - 1] > x) {
            g[p] = g[p - 1];
            --p;
        }
        g[p] = x;
    }
};

int32_t uf_find(std::vector<int32_t> &par, int32_t a) {
    while (par[(size_t)a] != a) {
        par[(size_t)a] = par[(size_t)par[(size_t)a]];
        a = par[(size_t)a];
    }
    return a;
}

}  // namespace

extern "C" hplmm_status hplmm_partition_from_voxels(int32_t nx, int32_t ny, int32_t nz,
                                                    const uint8_t *solid, const int32_t *voxel_label,
                                                    int32_t n_labels, int32_t w_zeta,
                                                    hplmm_partition *out) {
    return guarded([&]() -> hplmm_status {
        if (!out) fail(HPLMM_E_ARG, "out is NULL");
        std::memset(out, 0, sizeof(*out));
        if (!solid || !voxel_label) fail(HPLMM_E_ARG, "NULL input array");
        check_dims(nx, ny, nz);
        if (n_labels <= 0 || w_zeta < 0) fail(HPLMM_E_ARG, "n_labels must be > 0 and w_zeta >= 0");
        NodeMap nm;
        nm.build(nx, ny, nz, solid);
        const int64_t n = nm.n();
        std::vector<Labels> S((size_t)n);
        auto corners = [&](int64_t i, int64_t j, int64_t k, int32_t f[8]) {
            for (int a = 0; a < 8; ++a)
                f[a] = nm.lat2free[(size_t)nm.lat(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1))];
        };
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t vox = i + nx * (j + (int64_t)ny * k);
                    if (!solid[vox]) continue;
                    const int32_t g = voxel_label[vox];
                    if (g < 0 || g >= n_labels) fail(HPLMM_E_ARG, "voxel label out of range on a solid voxel");
                    int32_t f[8];
                    corners(i, j, k, f);
                    for (int a = 0; a < 8; ++a)
                        if (f[a] >= 0) S[(size_t)f[a]].add(g);
                }
        std::vector<int32_t> node_grain((size_t)n, -1);
        for (int64_t v = 0; v < n; ++v)
            if (S[(size_t)v].n == 1) node_grain[(size_t)v] = S[(size_t)v].g[0];
        std::vector<int32_t> par((size_t)n);
        std::iota(par.begin(), par.end(), 0);
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    if (!solid[i + nx * (j + (int64_t)ny * k)]) continue;
                    int32_t f[8];
                    corners(i, j, k, f);
                    for (int a = 0; a < 8; ++a) {
                        if (f[a] < 0 || node_grain[(size_t)f[a]] >= 0) continue;
                        for (int b = a + 1; b < 8; ++b) {
                            if (f[b] < 0 || node_grain[(size_t)f[b]] >= 0) continue;
                            if (!(S[(size_t)f[a]] == S[(size_t)f[b]])) continue;
                            int32_t ra = uf_find(par, f[a]), rb = uf_find(par, f[b]);
                            if (ra != rb) par[(size_t)std::max(ra, rb)] = std::min(ra, rb);
                        }
                    }
                }
        // interfaces numbered by their smallest node (= the union-find root,
        // since roots are always the smallest member)
        std::vector<int32_t> iface_of((size_t)n, -1);
        int32_t n_if = 0;
        std::vector<int64_t> count;
        for (int64_t v = 0; v < n; ++v) {
            if (node_grain[(size_t)v] >= 0) continue;
            const int32_t r = uf_find(par, (int32_t)v);
            if (r == v) {
                iface_of[(size_t)v] = n_if++;
                count.push_back(0);
            } else {
                iface_of[(size_t)v] = iface_of[(size_t)r];
            }
            count[(size_t)iface_of[(size_t)v]]++;
        }
        out->n_nodes = n;
        out->n_grains = n_labels;
        out->n_ifaces = n_if;
        out->node_grain = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
        out->iface_ptr = (int64_t *)std::malloc(sizeof(int64_t) * (size_t)(n_if + 1));
        int64_t tot = 0;
        for (auto c : count) tot += c;
        out->iface_nodes = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(tot, 1));
        if (!out->node_grain || !out->iface_ptr || !out->iface_nodes) {
            hplmm_partition_free(out);
            fail(HPLMM_E_OOM, "host allocation failed");
        }
        std::memcpy(out->node_grain, node_grain.data(), sizeof(int32_t) * (size_t)n);
        out->iface_ptr[0] = 0;
        for (int32_t c = 0; c < n_if; ++c) out->iface_ptr[c + 1] = out->iface_ptr[c] + count[(size_t)c];
        {
            std::vector<int64_t> fill(out->iface_ptr, out->iface_ptr + n_if);
            for (int64_t v = 0; v < n; ++v)
                if (iface_of[(size_t)v] >= 0) out->iface_nodes[fill[(size_t)iface_of[(size_t)v]]++] = (int32_t)v;
        }
        // contact grids: Chebyshev dilation by w_zeta of each interface
        std::vector<int32_t> stamp((size_t)n, -1);
        std::vector<int64_t> cptr(1, 0);
        std::vector<int32_t> cnodes;
        std::vector<int32_t> buf;
        for (int32_t c = 0; c < n_if; ++c) {
            buf.clear();
            for (int64_t p = out->iface_ptr[c]; p < out->iface_ptr[c + 1]; ++p) {
                const int64_t L = nm.free2lat[(size_t)out->iface_nodes[p]];
                const int64_t i = L % nm.NX, j = (L / nm.NX) % nm.NY, k = L / (nm.NX * nm.NY);
                for (int64_t dz = -w_zeta; dz <= w_zeta; ++dz)
                    for (int64_t dy = -w_zeta; dy <= w_zeta; ++dy)
                        for (int64_t dx = -w_zeta; dx <= w_zeta; ++dx) {
                            const int64_t ii = i + dx, jj = j + dy, kk = k + dz;
                            if (ii < 0 || jj < 0 || kk < 0 || ii >= nm.NX || jj >= nm.NY || kk >= nm.NZ) continue;
                            const int32_t u = nm.lat2free[(size_t)nm.lat(ii, jj, kk)];
                            if (u < 0 || stamp[(size_t)u] == c) continue;
                            stamp[(size_t)u] = c;
                            buf.push_back(u);
                        }
            }
            std::sort(buf.begin(), buf.end());
            cnodes.insert(cnodes.end(), buf.begin(), buf.end());
            cptr.push_back((int64_t)cnodes.size());
        }
        out->n_contacts = n_if;
        out->contact_ptr = (int64_t *)std::malloc(sizeof(int64_t) * cptr.size());
        out->contact_nodes = (int32_t *)std::malloc(sizeof(int32_t) * std::max<size_t>(cnodes.size(), 1));
        if (!out->contact_ptr || !out->contact_nodes) {
            hplmm_partition_free(out);
            fail(HPLMM_E_OOM, "host allocation failed");
        }
        std::memcpy(out->contact_ptr, cptr.data(), sizeof(int64_t) * cptr.size());
        if (!cnodes.empty()) std::memcpy(out->contact_nodes, cnodes.data(), sizeof(int32_t) * cnodes.size());
        return HPLMM_OK;
    });
}

extern "C" void hplmm_partition_free(hplmm_partition *p) {
    if (!p) return;
    std::free(p->node_grain);
    std::free(p->iface_ptr);
    std::free(p->iface_nodes);
    std::free(p->contact_ptr);
    std::free(p->contact_nodes);
    std::memset(p, 0, sizeof(*p));
}

namespace hplmm {

// Summed inverse distance from node y to the nodes in `others`, summed in list
// order (Eq. 7).
static double potential(const int32_t *xyz, int32_t y, const std::vector<int32_t> &others) {
    double s = 0.0;
    for (int32_t j : others) {
        const double dx = (double)(xyz[3 * y] - xyz[3 * j]);
        const double dy = (double)(xyz[3 * y + 1] - xyz[3 * j + 1]);
        const double dz = (double)(xyz[3 * y + 2] - xyz[3 * j + 2]);
        const double d2 = dx * dx + dy * dy + dz * dz;
        s += 1.0 / std::sqrt(d2);
    }
    return s;
}

static int32_t argmin_potential(const int32_t *xyz, int32_t N, const std::vector<int32_t> &others) {
    constexpr double kTie = 1e-12;
    std::vector<double> val((size_t)N);
    std::vector<uint8_t> taken((size_t)N, 0);
    for (int32_t j : others) taken[(size_t)j] = 1;
    double best = INFINITY;
    for (int32_t y = 0; y < N; ++y) {
        if (taken[(size_t)y]) continue;
        val[(size_t)y] = potential(xyz, y, others);
        best = std::min(best, val[(size_t)y]);
    }
    for (int32_t y = 0; y < N; ++y)
        if (!taken[(size_t)y] && val[(size_t)y] <= best * (1.0 + kTie)) return y;
    return -1;
}

// Mortar nodes of one interface (Sec. 3.3): the farthest pair, greedy
// additions minimising the summed inverse distance (Eq. 7), then sweeps in
// mortar order that move a node to the minimiser of its potential when that
// lowers it by more than a relative 1e-12.
std::vector<int32_t> place_mortars(const int32_t *xyz, int32_t N, int32_t n) {
    std::vector<int32_t> placed;
    const int32_t nu = std::min(n, N);
    if (nu >= N) {
        for (int32_t i = 0; i < N; ++i) placed.push_back(i);
        return placed;
    }
    if (nu == 1) return {0};
    int64_t best = -1;
    int32_t pa = 0, pb = 1;
    for (int32_t a = 0; a < N; ++a)
        for (int32_t b = a + 1; b < N; ++b) {
            const int64_t dx = xyz[3 * a] - xyz[3 * b], dy = xyz[3 * a + 1] - xyz[3 * b + 1],
                          dz = xyz[3 * a + 2] - xyz[3 * b + 2];
            const int64_t d2 = dx * dx + dy * dy + dz * dz;
            if (d2 > best) {
                best = d2;
                pa = a;
                pb = b;
            }
        }
    placed = {pa, pb};
    while ((int32_t)placed.size() < nu) placed.push_back(argmin_potential(xyz, N, placed));
    for (int sweep = 0; sweep < 100; ++sweep) {
        bool moved = false;
        for (int32_t m = 0; m < nu; ++m) {
            std::vector<int32_t> others;
            for (int32_t q = 0; q < nu; ++q)
                if (q != m) others.push_back(placed[(size_t)q]);
            const double cur = potential(xyz, placed[(size_t)m], others);
            const int32_t y = argmin_potential(xyz, N, others);
            if (y != placed[(size_t)m] && potential(xyz, y, others) < cur * (1.0 - 1e-12)) {
                placed[(size_t)m] = y;
                moved = true;
            }
        }
        if (!moved) break;
    }
    return placed;
}

}  // namespace hplmm

extern "C" hplmm_status hplmm_place_mortars(const int32_t *xyz, int32_t N, int32_t n, int32_t *idx_out) {
    return guarded([&]() -> hplmm_status {
        if (!xyz || !idx_out || N <= 0 || n <= 0) fail(HPLMM_E_ARG, "invalid mortar placement arguments");
        auto p = place_mortars(xyz, N, n);
        for (size_t i = 0; i < p.size(); ++i) idx_out[i] = p[i];
        return HPLMM_OK;
    });
}
