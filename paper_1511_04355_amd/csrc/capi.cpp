// C ABI of the afsbem library: argument validation, error capture, handles.
#include <cmath>
#include <cstring>
#include <string>

#include "internal.hpp"
#include "solver.hpp"
#include "mlp.hpp"
#include "batched.hpp"
#include "tune.hpp"

struct afsbem_mesh {
    std::vector<double> xyz;
    std::vector<int32_t> tri;      // [n_tri][3], or [n_tri][6] when order == 2
    int64_t n_vert = 0, n_tri = 0;
    int order = 1;                 // 1: flat triangles, 2: six-node (curved quadratic) triangles
};

struct afsbem_problem {
    afsbem::Problem p;
    std::vector<void *> allocs;
};

namespace afsbem {

static thread_local std::string g_last_error = "";

void set_error(const std::string &msg) { g_last_error = msg; }

template <class F>
static int guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return AFSBEM_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return AFSBEM_EINVAL;
    }
}

template <class T>
static T *upload(afsbem_problem *h, const std::vector<T> &v) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess)
        throw Error{AFSBEM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
    h->allocs.push_back(p);
    if (!v.empty())
        AFS_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return static_cast<T *>(p);
}

static void free_problem(afsbem_problem *h) {
    if (!h)
        return;
    delete h->p.ws;
    h->p.ws = nullptr;
    delete h->p.ws2;
    h->p.ws2 = nullptr;
    delete h->p.learn;
    h->p.learn = nullptr;
    delete h->p.barena;
    h->p.barena = nullptr;
    delete h->p.hmat;
    h->p.hmat = nullptr;
    if (h->p.st_asm)
        (void)hipStreamDestroy(h->p.st_asm);
    if (h->p.st_sol)
        (void)hipStreamDestroy(h->p.st_sol);
    h->p.st_asm = h->p.st_sol = nullptr;
    for (void *p : h->allocs)
        (void)hipFree(p);
    h->allocs.clear();
}

}  // namespace afsbem

using namespace afsbem;

extern "C" {

const char *afsbem_last_error(void) { return g_last_error.c_str(); }

int afsbem_version(int *major, int *minor) {
    if (major)
        *major = 0;
    if (minor)
        *minor = 1;
    return AFSBEM_OK;
}

int afsbem_mesh_create(const double *xyz, int64_t n_vert, const int32_t *tri, int64_t n_tri, afsbem_mesh **out) {
    return guarded([&] {
        AFS_REQUIRE(out && xyz && tri, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(n_vert >= 3 && n_tri >= 1, AFSBEM_EINVAL, "mesh needs at least 3 vertices and 1 triangle");
        AFS_REQUIRE(n_tri <= (int64_t)1 << 28, AFSBEM_EINVAL, "too many triangles");
        for (int64_t k = 0; k < 3 * n_tri; ++k)
            AFS_REQUIRE(tri[k] >= 0 && tri[k] < n_vert, AFSBEM_EINVAL,
                        "triangle " + std::to_string(k / 3) + " has a vertex index out of range");
        for (int64_t k = 0; k < 3 * n_vert; ++k)
            AFS_REQUIRE(std::isfinite(xyz[k]), AFSBEM_EINVAL, "non-finite vertex coordinate");
        auto *m = new afsbem_mesh();
        m->xyz.assign(xyz, xyz + 3 * n_vert);
        m->tri.assign(tri, tri + 3 * n_tri);
        m->n_vert = n_vert;
        m->n_tri = n_tri;
        *out = m;
        return AFSBEM_OK;
    });
}

int afsbem_mesh_create_quadratic(const double *xyz, int64_t n_vert, const int32_t *tri6, int64_t n_tri,
                                 afsbem_mesh **out) {
    return guarded([&] {
        AFS_REQUIRE(out && xyz && tri6, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(n_vert >= 6 && n_tri >= 1, AFSBEM_EINVAL, "mesh needs at least 6 nodes and 1 element");
        AFS_REQUIRE(n_tri <= (int64_t)1 << 24, AFSBEM_EINVAL, "too many elements");
        for (int64_t k = 0; k < 6 * n_tri; ++k)
            AFS_REQUIRE(tri6[k] >= 0 && tri6[k] < n_vert, AFSBEM_EINVAL,
                        "element " + std::to_string(k / 6) + " has a node index out of range");
        for (int64_t k = 0; k < 3 * n_vert; ++k)
            AFS_REQUIRE(std::isfinite(xyz[k]), AFSBEM_EINVAL, "non-finite node coordinate");
        auto *m = new afsbem_mesh();
        m->xyz.assign(xyz, xyz + 3 * n_vert);
        m->tri.assign(tri6, tri6 + 6 * n_tri);
        m->n_vert = n_vert;
        m->n_tri = n_tri;
        m->order = 2;
        *out = m;
        return AFSBEM_OK;
    });
}

int afsbem_mesh_destroy(afsbem_mesh *mesh) {
    delete mesh;
    return AFSBEM_OK;
}

int afsbem_problem_create(const afsbem_mesh *mesh, const afsbem_material *mat, const int8_t *bc_kind,
                          const afsbem_quad_policy *policy, afsbem_problem **out) {
    afsbem_problem *h = nullptr;
    int rc = guarded([&] {
        AFS_REQUIRE(mesh && mat && bc_kind && out, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(mat->mu > 0 && mat->rho > 0 && mat->nu > -1.0 && mat->nu < 0.5, AFSBEM_EINVAL,
                    "material needs mu > 0, rho > 0, -1 < nu < 0.5");
        afsbem_quad_policy pol{2.0, 8, 16, 16};
        if (policy)
            pol = *policy;
        AFS_REQUIRE(pol.far_ratio >= 0 && pol.max_subdiv >= 0 && pol.max_subdiv <= 12 && pol.self_n_theta >= 1 &&
                        pol.self_n_theta <= 64 && pol.self_n_rho >= 1 && pol.self_n_rho <= 64,
                    AFSBEM_EINVAL, "invalid quadrature policy");
        for (int64_t e = 0; e < mesh->n_tri; ++e)
            AFS_REQUIRE(bc_kind[e] == 0 || bc_kind[e] == 1, AFSBEM_EINVAL, "bc_kind must be 0 or 1");
        h = new afsbem_problem();
        Problem &P = h->p;
        P.mat = derive_material(*mat);
        P.pol = pol;
        AFS_HIP(hipGetDevice(&P.device));
        if (mesh->order == 2)
            build_plan_nystrom(mesh->xyz.data(), mesh->n_vert, mesh->tri.data(), mesh->n_tri, bc_kind, pol, P.mat,
                               P.host);
        else
            build_plan(mesh->xyz.data(), mesh->n_vert, mesh->tri.data(), mesh->n_tri, bc_kind, pol, P.mat, P.host);
        const HostPlan &H = P.host;
        DevicePlan &D = P.dev;
        D.n_tri = H.n_tri;
        D.nnz = (int64_t)H.near_col.size();
        D.n_leaves = (int64_t)(H.disc == 1 ? H.nys_leaves.size() / 6 : H.leaves.size() / 10);
        D.disc = H.disc;
        D.n_el = H.disc == 1 ? H.n_el : H.n_tri;
        if (H.disc == 1) {
            D.nys_geom = upload(h, H.nys_geom);
            D.nys_leaves = upload(h, H.nys_leaves);
            D.nys_self = upload(h, H.nys_self);
            std::vector<double> tab(H.nys_pt, H.nys_pt + 12);
            tab.insert(tab.end(), H.nys_lag, H.nys_lag + 36);
            D.nys_tab = upload(h, tab);
        }
        D.n_theta = H.n_theta;
        D.n_rho = H.n_rho;
        std::vector<double> cx(H.n_tri), cy(H.n_tri), cz(H.n_tri);
        for (int64_t e = 0; e < H.n_tri; ++e) {
            cx[e] = H.cen[3 * e];
            cy[e] = H.cen[3 * e + 1];
            cz[e] = H.cen[3 * e + 2];
        }
        D.colx = upload(h, cx);
        D.coly = upload(h, cy);
        D.colz = upload(h, cz);
        D.src = upload(h, H.src);
        D.kind = upload(h, H.kind);
        D.near_ptr = upload(h, H.near_ptr);
        D.near_col = upload(h, H.near_col);
        D.near_row = upload(h, H.near_row);
        D.near_order = upload(h, H.near_order);
        D.leaf_ptr = upload(h, H.leaf_ptr);
        D.leaves = upload(h, H.leaves);
        D.self_ang = upload(h, H.self_ang);
        D.self_cpv = upload(h, H.self_cpv);
        D.gl_rho = upload(h, H.gl_rho);
        D.nrm = upload(h, H.nrm);
        D.coef = upload(h, H.coef);
        // on-the-fly far field: collocation points as [n][4], FP32 copies
        std::vector<double> c4(4 * H.n_tri, 0.0);
        std::vector<float> c4f(4 * H.n_tri, 0.f), srcf(H.src.size()), coeff(H.coef.size());
        for (int64_t e = 0; e < H.n_tri; ++e)
            for (int d = 0; d < 3; ++d) {
                c4[4 * e + d] = H.cen[3 * e + d];
                c4f[4 * e + d] = (float)H.cen[3 * e + d];
            }
        for (size_t k = 0; k < H.src.size(); ++k)
            srcf[k] = (float)H.src[k];
        for (size_t k = 0; k < H.coef.size(); ++k)
            coeff[k] = (float)H.coef[k];
        D.col64 = upload(h, c4);
        D.col32 = upload(h, c4f);
        D.src32 = upload(h, srcf);
        D.coef32 = upload(h, coeff);
        D.n_clusters = (int64_t)H.clus_ptr.size() - 1;
        D.clus_ptr = upload(h, H.clus_ptr);
        D.clus_elem = upload(h, H.clus_elem);
        *out = h;
        return AFSBEM_OK;
    });
    if (rc != AFSBEM_OK && h) {
        free_problem(h);
        delete h;
    }
    return rc;
}

int afsbem_problem_destroy(afsbem_problem *p) {
    if (p) {
        free_problem(p);
        delete p;
    }
    return AFSBEM_OK;
}

int afsbem_problem_info(const afsbem_problem *p, int64_t *n_tri, int64_t *n_near_pairs, int64_t *n_leaves,
                        int64_t *self_nodes_per_element) {
    return guarded([&] {
        AFS_REQUIRE(p, AFSBEM_EINVAL, "null problem");
        if (n_tri)
            *n_tri = p->p.dev.n_tri;
        if (n_near_pairs)
            *n_near_pairs = p->p.dev.nnz;
        if (n_leaves)
            *n_leaves = p->p.dev.n_leaves;
        if (self_nodes_per_element)
            *self_nodes_per_element = (p->p.dev.disc == 1 ? 6 : 3) * (int64_t)p->p.dev.n_theta * p->p.dev.n_rho;
        return AFSBEM_OK;
    });
}

int afsbem_problem_points(const afsbem_problem *p, double *out8) {
    return guarded([&] {
        AFS_REQUIRE(p && out8, AFSBEM_EINVAL, "null pointer argument");
        const HostPlan &H = p->p.host;
        for (int64_t i = 0; i < H.n_tri; ++i) {
            double *o = out8 + 8 * i;
            for (int k = 0; k < 3; ++k) {
                o[k] = H.cen[3 * i + k];
                o[3 + k] = H.nrm[3 * i + k];
            }
            o[6] = H.disc == 1 ? H.src[kSrcStride * i + 3] : H.area[i];
            o[7] = (double)H.kind[i];
        }
        return AFSBEM_OK;
    });
}

int afsbem_assemble_device(afsbem_problem *p, double s_re, double s_im, const void *d_bc_val, int format, void *d_A,
                           void *d_A_lo, void *d_b, void *d_precond, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(p && d_bc_val && d_A && d_b, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(format == AFSBEM_FMT_C128 || (format == AFSBEM_FMT_SPLIT && d_A_lo), AFSBEM_EINVAL,
                    "format must be C128, or SPLIT with both planes");
        AFS_REQUIRE(std::isfinite(s_re) && std::isfinite(s_im), AFSBEM_EINVAL, "non-finite s");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        void *scratch = nullptr;
        AFS_HIP(hipMallocAsync(&scratch, assembly_scratch_bytes(p->p), st));
        KernelParams kp = kernel_params(p->p.mat, s_re, s_im);
        launch_assembly(p->p, kp, static_cast<const double *>(d_bc_val), format, d_A, d_A_lo,
                        static_cast<double *>(d_b), static_cast<double *>(d_precond), scratch, st);
        AFS_HIP(hipFreeAsync(scratch, st));
        return AFSBEM_OK;
    });
}

int afsbem_matvec_device(afsbem_problem *p, int format, int precision, const void *d_A, const void *d_A_lo,
                         const void *d_x, void *d_y, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(p && d_A && d_x && d_y, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(format == AFSBEM_FMT_C128 || format == AFSBEM_FMT_SPLIT, AFSBEM_EINVAL, "bad format");
        AFS_REQUIRE(precision == 0 || (precision == 1 && format == AFSBEM_FMT_SPLIT), AFSBEM_EINVAL,
                    "FP32 products need the SPLIT format");
        AFS_REQUIRE(format == AFSBEM_FMT_C128 || precision == 1 || d_A_lo, AFSBEM_EINVAL, "FP64 SPLIT needs lo plane");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const int64_t N = 3 * p->p.dev.n_tri;
        void *partial = nullptr;
        AFS_HIP(hipMallocAsync(&partial, (size_t)gemv_chunks(N) * N * 16, st));
        launch_gemv(N, format, precision, d_A, d_A_lo, static_cast<const double *>(d_x), static_cast<double *>(d_y),
                    static_cast<double *>(partial), st);
        AFS_HIP(hipFreeAsync(partial, st));
        return AFSBEM_OK;
    });
}

int afsbem_matvec_device_noalloc(afsbem_problem *p, int format, int precision, const void *d_A, const void *d_A_lo,
                                 const void *d_x, void *d_y, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(p && d_A && d_x && d_y, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(format == AFSBEM_FMT_C128 || format == AFSBEM_FMT_SPLIT, AFSBEM_EINVAL, "bad format");
        AFS_REQUIRE(precision == 0 || (precision == 1 && format == AFSBEM_FMT_SPLIT), AFSBEM_EINVAL,
                    "FP32 products need the SPLIT format");
        AFS_REQUIRE(format == AFSBEM_FMT_C128 || precision == 1 || d_A_lo, AFSBEM_EINVAL, "FP64 SPLIT needs lo plane");
        const int64_t N = 3 * p->p.dev.n_tri;
        launch_gemv_noalloc(N, format, precision, d_A, d_A_lo, static_cast<const double *>(d_x),
                            static_cast<double *>(d_y), static_cast<hipStream_t>(hip_stream));
        return AFSBEM_OK;
    });
}

int afsbem_matvec_free_device(afsbem_problem *p, double s_re, double s_im, int precision, const void *d_bc_val,
                              const void *d_x, void *d_y, void *d_b, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(p, AFSBEM_EINVAL, "null problem");
        AFS_REQUIRE(precision == 0 || precision == 1, AFSBEM_EINVAL, "precision must be 0 or 1");
        AFS_REQUIRE((d_x == nullptr) == (d_y == nullptr), AFSBEM_EINVAL, "x and y go together");
        AFS_REQUIRE(!d_b || d_bc_val, AFSBEM_EINVAL, "b needs the boundary values");
        AFS_REQUIRE(std::isfinite(s_re) && std::isfinite(s_im), AFSBEM_EINVAL, "non-finite s");
        AFS_REQUIRE(p->p.dev.disc == 0, AFSBEM_EINVAL,
                    "matrix-free application is not available for six-node (Nystrom) problems");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const Problem &P = p->p;
        const int64_t nt = P.dev.n_tri, N = 3 * nt;
        char *mem = nullptr;
        const size_t blk = ((size_t)std::max<int64_t>(P.dev.nnz, 1) * 144 + 255) / 256 * 256;
        const size_t sblk = ((size_t)nt * 144 + 255) / 256 * 256;
        const size_t zb = d_bc_val ? 0 : ((size_t)N * 16 + 255) / 256 * 256;
        const size_t scr = assembly_scratch_bytes(P);
        AFS_HIP(hipMallocAsync((void **)&mem, blk + sblk + zb + scr, st));
        double *nearblk = reinterpret_cast<double *>(mem), *selfblk = reinterpret_cast<double *>(mem + blk);
        const double *bc = static_cast<const double *>(d_bc_val);
        if (!bc) {
            AFS_HIP(hipMemsetAsync(mem + blk + sblk, 0, (size_t)N * 16, st));
            bc = reinterpret_cast<const double *>(mem + blk + sblk);
        }
        void *scratch = mem + blk + sblk + zb;
        KernelParams kp = kernel_params(P.mat, s_re, s_im);
        launch_block_setup(P, kp, bc, nearblk, selfblk, nullptr, scratch, st);
        double *part = static_cast<double *>(scratch);  // far partial sums (b first, then y)
        if (d_b) {
            mf_apply(P, kp, 0, 1, nullptr, nullptr, bc, nullptr, part, st);
            launch_finalize_b(P, mf_chunks(nt), part, scratch, static_cast<double *>(d_b), st);
        }
        if (d_x)
            mf_apply(P, kp, precision, 0, nearblk, selfblk, static_cast<const double *>(d_x),
                     static_cast<double *>(d_y), part, st);
        AFS_HIP(hipFreeAsync(mem, st));
        return AFSBEM_OK;
    });
}

int afsbem_plan_info(const afsbem_mesh *mesh, const int8_t *bc_kind, const afsbem_quad_policy *policy,
                     int64_t *out4) {
    return guarded([&] {
        AFS_REQUIRE(mesh && bc_kind && out4, AFSBEM_EINVAL, "null pointer argument");
        for (int64_t e = 0; e < mesh->n_tri; ++e)
            AFS_REQUIRE(bc_kind[e] == 0 || bc_kind[e] == 1, AFSBEM_EINVAL, "bc_kind must be 0 or 1");
        const afsbem_quad_policy pol = policy ? *policy : afsbem_quad_policy{2.0, 8, 16, 16};
        HostPlan H;
        const MaterialDerived mat = derive_material(afsbem_material{1.0, 0.25, 1.0});
        if (mesh->order == 2) {
            build_plan_nystrom(mesh->xyz.data(), mesh->n_vert, mesh->tri.data(), mesh->n_tri, bc_kind, pol, mat, H);
            out4[2] = (int64_t)(H.nys_leaves.size() / 6);
        } else {
            build_plan(mesh->xyz.data(), mesh->n_vert, mesh->tri.data(), mesh->n_tri, bc_kind, pol, mat, H);
            out4[2] = (int64_t)(H.leaves.size() / 10);
        }
        out4[0] = H.n_tri;
        out4[1] = (int64_t)H.near_col.size();
        out4[3] = (int64_t)H.clus_ptr.size() - 1;
        return AFSBEM_OK;
    });
}

int afsbem_hmat_partition_info(const afsbem_mesh *mesh, const int8_t *bc_kind, const afsbem_quad_policy *policy,
                                double eta, int64_t *out8) {
    return guarded([&] {
        AFS_REQUIRE(mesh && bc_kind && out8, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(mesh->order == 1, AFSBEM_EINVAL, "the hierarchical operator is built for flat-element meshes");
        AFS_REQUIRE(eta > 0.0 && std::isfinite(eta), AFSBEM_EINVAL, "eta must be > 0");
        for (int64_t e = 0; e < mesh->n_tri; ++e)
            AFS_REQUIRE(bc_kind[e] == 0 || bc_kind[e] == 1, AFSBEM_EINVAL, "bc_kind must be 0 or 1");
        Problem P;  // host plan only: nothing is uploaded
        P.pol = policy ? *policy : afsbem_quad_policy{2.0, 8, 16, 16};
        P.mat = derive_material(afsbem_material{1.0, 0.25, 1.0});
        build_plan(mesh->xyz.data(), mesh->n_vert, mesh->tri.data(), mesh->n_tri, bc_kind, P.pol, P.mat, P.host);
        HmatPlan H;
        hmat_build(P, eta, kHmatKmax, H, false);
        const int64_t n = H.n, nd = (int64_t)H.dense.size() / 4, nl = (int64_t)H.lowrank.size() / 4;
        std::vector<int64_t> pos(n);
        for (int64_t q = 0; q < n; ++q)
            pos[H.perm[q]] = q;
        int64_t covered = 0, near_in_lowrank = 0, largest = 0;
        for (int64_t d = 0; d < nd; ++d)
            covered += (H.dense[4 * d + 1] - H.dense[4 * d]) * (H.dense[4 * d + 3] - H.dense[4 * d + 2]);
        for (int64_t l = 0; l < nl; ++l) {
            const int64_t a0 = H.lowrank[4 * l], a1 = H.lowrank[4 * l + 1];
            const int64_t b0 = H.lowrank[4 * l + 2], b1 = H.lowrank[4 * l + 3];
            covered += (a1 - a0) * (b1 - b0);
            largest = std::max(largest, std::max(a1 - a0, b1 - b0));
            for (int64_t q = a0; q < a1; ++q) {
                const int32_t m = H.perm[q];
                for (int64_t pp = P.host.near_ptr[m]; pp < P.host.near_ptr[m + 1]; ++pp) {
                    const int64_t pn = pos[P.host.near_col[pp]];
                    near_in_lowrank += (pn >= b0 && pn < b1);
                }
            }
        }
        int64_t leaf_rows = 0;
        for (size_t L = 0; L + 1 < H.leaves.size(); L += 2)
            leaf_rows += H.leaves[L + 1] - H.leaves[L];
        out8[0] = n;
        out8[1] = nd;
        out8[2] = nl;
        out8[3] = covered;
        out8[4] = near_in_lowrank;
        out8[5] = largest;
        out8[6] = leaf_rows;
        out8[7] = (int64_t)H.leaf_item.size();
        return AFSBEM_OK;
    });
}

int afsbem_hmat_matvec_device(afsbem_problem *p, double s_re, double s_im, double eps, double eta, const void *d_x,
                              void *d_y, int32_t *max_rank, int64_t *n_lowrank, int64_t *n_dense,
                              void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(p && d_x && d_y, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(std::isfinite(s_re) && std::isfinite(s_im), AFSBEM_EINVAL, "non-finite s");
        AFS_REQUIRE(eps > 0.0 && eps < 1.0 && eta > 0.0 && std::isfinite(eta), AFSBEM_EINVAL,
                    "eps must be in (0, 1) and eta > 0");
        AFS_REQUIRE(p->p.dev.disc == 0, AFSBEM_EINVAL, "the hierarchical operator is built for flat-element problems");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        Problem &P = p->p;
        const int64_t N = 3 * P.dev.n_tri;
        Workspace ws;
        ws.ensure(P, kFmtBlocks, 1, 0);
        AFS_HIP(hipMemsetAsync(ws.x, 0, (size_t)N * 16, st));  // boundary values: b is not formed here
        const KernelParams kp = kernel_params(P.mat, s_re, s_im);
        launch_block_setup(P, kp, ws.x, ws.nearblk, ws.selfblk, ws.precond, ws.asm_scratch, st);
        hmat_ensure(P, eta);
        hmat_setup(P, ws, kp, eps, st);
        AFS_HIP(hipStreamSynchronize(st));
        bool ok = hmat_finish(P, ws, st);
        for (int tries = 0; !ok && ws.hm_exhausted && tries < 3; ++tries) {
            hmat_setup(P, ws, kp, eps, st);  // a larger pool
            AFS_HIP(hipStreamSynchronize(st));
            ok = hmat_finish(P, ws, st);
        }
        hmat_apply(P, ws, static_cast<const double *>(d_x), static_cast<double *>(d_y), st);
        AFS_HIP(hipStreamSynchronize(st));
        if (max_rank)
            *max_rank = ws.hm_max_rank;
        if (n_lowrank)
            *n_lowrank = (int64_t)P.hmat->lowrank.size() / 4;
        if (n_dense)
            *n_dense = (int64_t)P.hmat->dense.size() / 4;
        if (!ok)
            set_error("a low-rank block did not reach eps within the term limit");
        return ok ? AFSBEM_OK : AFSBEM_ENOCONV;
    });
}

int afsbem_autotune_set(int enabled) {
    autotune_set_enabled(enabled != 0);
    return AFSBEM_OK;
}

int afsbem_autotune_report(char *buf, int64_t cap, int64_t *len) {
    return guarded([&] {
        const std::string r = autotune_report();
        if (len)
            *len = (int64_t)r.size();
        if (buf && cap > 0) {
            const size_t n = std::min<size_t>((size_t)cap - 1, r.size());
            std::memcpy(buf, r.data(), n);
            buf[n] = 0;
        }
        return (int)AFSBEM_OK;
    });
}

int afsbem_mlp_n_params(int32_t d_in, int32_t hidden, int32_t d_out, int64_t *n) {
    return guarded([&] {
        AFS_REQUIRE(d_in >= 1 && hidden >= 1 && d_out >= 1 && n, AFSBEM_EINVAL, "bad MLP shape");
        *n = MlpShape(d_in, hidden, d_out).n_params;
        return AFSBEM_OK;
    });
}

int afsbem_mlp_forward(int32_t d_in, int32_t hidden, int32_t d_out, int32_t n, const float *d_params, const float *d_X,
                       float *d_Y, int mode, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(d_in >= 1 && hidden >= 1 && d_out >= 1 && n >= 0, AFSBEM_EINVAL, "bad MLP shape");
        AFS_REQUIRE(d_params && d_X && d_Y, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(mode == 0 || mode == 1, AFSBEM_EINVAL, "mode must be 0 (FP32) or 1 (BF16 MFMA)");
        if (n == 0)
            return AFSBEM_OK;
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        MlpShape s(d_in, hidden, d_out);
        void *work = nullptr;
        AFS_HIP(hipMallocAsync(&work, mlp_work_floats(s, n) * 4, st));
        mlp_forward(s, mode, n, d_params, d_X, d_Y, static_cast<float *>(work), st);
        AFS_HIP(hipFreeAsync(work, st));
        return AFSBEM_OK;
    });
}

int afsbem_mlp_loss_grad(int32_t d_in, int32_t hidden, int32_t d_out, int32_t n, const float *d_params,
                         const float *d_X, const float *d_T, float *d_grad, float *d_loss, int mode, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(d_in >= 1 && hidden >= 1 && d_out >= 1 && n >= 1, AFSBEM_EINVAL, "bad MLP shape");
        AFS_REQUIRE(d_params && d_X && d_T && d_grad, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(mode == 0 || mode == 1, AFSBEM_EINVAL, "mode must be 0 (FP32) or 1 (BF16 MFMA)");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        MlpShape s(d_in, hidden, d_out);
        void *work = nullptr;
        AFS_HIP(hipMallocAsync(&work, mlp_work_floats(s, n) * 4, st));
        mlp_loss_grad(s, mode, n, d_params, d_X, d_T, d_grad, d_loss, static_cast<float *>(work), st);
        AFS_HIP(hipFreeAsync(work, st));
        return AFSBEM_OK;
    });
}

int afsbem_mlp_adam(int64_t n_params, float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t t,
                    float lr, float beta1, float beta2, float eps, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(n_params >= 1 && d_params && d_grad && d_m && d_v && t >= 1, AFSBEM_EINVAL,
                    "bad Adam arguments");
        mlp_adam(n_params, d_params, d_grad, d_m, d_v, t, lr, beta1, beta2, eps, static_cast<hipStream_t>(hip_stream));
        return AFSBEM_OK;
    });
}

int afsbem_mlp_train_step(int32_t d_in, int32_t hidden, int32_t d_out, int32_t n, float *d_params, const float *d_X,
                          const float *d_T, float *d_m, float *d_v, int32_t t, float lr, float beta1, float beta2,
                          float eps, float *d_loss, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(d_in >= 1 && hidden >= 1 && d_out >= 1 && n >= 1, AFSBEM_EINVAL, "bad MLP shape");
        AFS_REQUIRE(d_params && d_X && d_T && d_m && d_v && t >= 1, AFSBEM_EINVAL, "bad training arguments");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        MlpShape s(d_in, hidden, d_out);
        void *work = nullptr;
        AFS_HIP(hipMallocAsync(&work, mlp_work_floats(s, n) * 4, st));
        mlp_train_step(s, n, d_params, d_X, d_T, d_m, d_v, t, lr, beta1, beta2, eps, d_loss,
                       static_cast<float *>(work), st);
        AFS_HIP(hipFreeAsync(work, st));
        return AFSBEM_OK;
    });
}

int afsbem_problem_clusters(const afsbem_problem *p, int64_t *n_clusters, int64_t *ptr_out, int32_t *elem_out) {
    return guarded([&] {
        AFS_REQUIRE(p && n_clusters, AFSBEM_EINVAL, "null pointer argument");
        const HostPlan &H = p->p.host;
        *n_clusters = (int64_t)H.clus_ptr.size() - 1;
        if (ptr_out)
            std::memcpy(ptr_out, H.clus_ptr.data(), H.clus_ptr.size() * sizeof(int64_t));
        if (elem_out)
            std::memcpy(elem_out, H.clus_elem.data(), H.clus_elem.size() * sizeof(int32_t));
        return AFSBEM_OK;
    });
}

int afsbem_precond_apply_device(afsbem_problem *p, int format, const void *d_A, const void *d_A_lo, const void *d_v,
                                void *d_z, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(p && d_A && d_v && d_z, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(format == AFSBEM_FMT_C128 || format == AFSBEM_FMT_SPLIT, AFSBEM_EINVAL, "bad format");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        void *inv = nullptr;
        AFS_HIP(hipMallocAsync(&inv, (size_t)std::max<int64_t>(p->p.dev.n_clusters, 1) * kClusterDim * kClusterDim * 8,
                               st));
        cluster_inverse(p->p.dev, format, d_A, d_A_lo, static_cast<float *>(inv), st);
        cluster_apply(p->p.dev, static_cast<float *>(inv), static_cast<const double *>(d_v), static_cast<double *>(d_z),
                      st);
        AFS_HIP(hipFreeAsync(inv, st));
        return AFSBEM_OK;
    });
}

int afsbem_solve_opts_default(afsbem_solve_opts *o) {
    if (!o) {
        set_error("null opts");
        return AFSBEM_EINVAL;
    }
    std::memset(o, 0, sizeof *o);
    o->tol = 1e-6;
    o->restart = 50;
    o->max_iter = 1000;
    o->precision = AFSBEM_PREC_FP64;
    o->warm_start = AFSBEM_WARM_NONE;
    o->inner_tol = 0.0;
    o->batch = 0;
    o->fault_inject = 0;
    o->profile = 0;
    o->learn_steps = 0;
    o->precond = 0;
    o->matrix_free = 0;
    o->no_graph = 0;
    return AFSBEM_OK;
}

int afsbem_solve_device(afsbem_problem *p, int32_t n_s, const double *s, const void *d_bc_val, const void *d_x0,
                        void *d_a_out, void *d_u_out, void *d_t_out, const afsbem_solve_opts *opts,
                        afsbem_solve_stats *stats, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(p && s && d_bc_val, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(n_s >= 0, AFSBEM_EINVAL, "n_s must be >= 0");
        afsbem_solve_opts o;
        afsbem_solve_opts_default(&o);
        if (opts)
            o = *opts;
        AFS_REQUIRE(o.tol > 0 && o.restart >= 1 && o.restart <= 4000 && o.max_iter >= 1, AFSBEM_EINVAL,
                    "invalid solver options");
        AFS_REQUIRE(o.learn_aug >= 0 && o.learn_aug <= 2, AFSBEM_EINVAL, "learn_aug must be 0, 1 or 2");
        AFS_REQUIRE(o.no_recycle == 0 || o.no_recycle == 1, AFSBEM_EINVAL, "no_recycle must be 0 or 1");
        AFS_REQUIRE(o.precision == AFSBEM_PREC_FP64 || o.precision == AFSBEM_PREC_MIXED, AFSBEM_EINVAL,
                    "unknown precision");
        AFS_REQUIRE((o.warm_start != AFSBEM_WARM_USER && o.warm_start != AFSBEM_WARM_USER_AUG) || d_x0,
                    AFSBEM_EINVAL, "user warm start needs x0");
        AFS_REQUIRE((o.warm_start >= AFSBEM_WARM_NONE && o.warm_start <= AFSBEM_WARM_LEARNED) ||
                        o.warm_start == AFSBEM_WARM_EXTRAP || o.warm_start == AFSBEM_WARM_USER_AUG,
                    AFSBEM_EINVAL, "unknown warm start");
        AFS_REQUIRE(o.precond == 0 || o.precond == 1, AFSBEM_EINVAL, "precond must be 0 or 1");
        AFS_REQUIRE(o.matrix_free >= 0 && o.matrix_free <= 2, AFSBEM_EINVAL, "matrix_free must be 0, 1 or 2");
        AFS_REQUIRE(o.matrix_free != 2 || o.precision == AFSBEM_PREC_MIXED, AFSBEM_EINVAL,
                    "matrix_free = 2 (hierarchical inner operator) needs the mixed precision path");
        AFS_REQUIRE(o.hmat_eps >= 0.0 && o.hmat_eps < 1.0 && o.hmat_eta >= 0.0 && std::isfinite(o.hmat_eta),
                    AFSBEM_EINVAL, "hmat_eps must be in [0, 1) and hmat_eta >= 0");
        AFS_REQUIRE(o.warm_start != AFSBEM_WARM_LEARNED || d_a_out, AFSBEM_EINVAL,
                    "the learned warm start needs the solution output buffer");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const int64_t nt = p->p.dev.n_tri, N = 3 * nt;
        for (int32_t k = 0; k < n_s; ++k)
            AFS_REQUIRE(std::isfinite(s[2 * k]) && std::isfinite(s[2 * k + 1]), AFSBEM_EINVAL, "non-finite s");
        int rc = AFSBEM_OK;
        const double *bcd = static_cast<const double *>(d_bc_val);
        if (o.batch != 1 && n_s >= 2) {
            rc = solve_pipelined(p->p, o, n_s, s, bcd, static_cast<const double *>(d_x0), static_cast<double *>(d_a_out),
                                 static_cast<double *>(d_u_out), static_cast<double *>(d_t_out), stats, st);
        } else {
            void *xbuf = nullptr;  // EXTRAP guesses
            for (int32_t k = 0; k < n_s; ++k) {
                const double *bc = bcd + 2 * (size_t)k * N;
                if (o.warm_start == AFSBEM_WARM_EXTRAP && k >= 2 && !xbuf)
                    AFS_HIP(hipMallocAsync(&xbuf, (size_t)N * 16, st));
                const double *x0 = start_guess(o, k, N, s, static_cast<const double *>(d_x0),
                                               static_cast<const double *>(d_a_out), static_cast<double *>(xbuf), st);
                double *a = d_a_out ? static_cast<double *>(d_a_out) + 2 * (size_t)k * N : nullptr;
                double *u = d_u_out ? static_cast<double *>(d_u_out) + 2 * (size_t)k * N : nullptr;
                double *t = d_t_out ? static_cast<double *>(d_t_out) + 2 * (size_t)k * N : nullptr;
                afsbem_solve_opts ok = o;
                if (ok.warm_start == AFSBEM_WARM_EXTRAP)
                    ok.warm_start = AFSBEM_WARM_PREV;
                if (!x0 && ok.warm_start != AFSBEM_WARM_LEARNED)
                    ok.warm_start = AFSBEM_WARM_NONE;
                int r;
                try {
                    r = solve_one(p->p, ok, s[2 * k], s[2 * k + 1], bc, x0, a, u, t, stats ? &stats[k] : nullptr, st);
                } catch (...) {
                    if (xbuf)
                        (void)hipFreeAsync(xbuf, st);
                    throw;
                }
                if (r != AFSBEM_OK && rc == AFSBEM_OK)
                    rc = r;
            }
            if (xbuf)
                AFS_HIP(hipFreeAsync(xbuf, st));
        }
        if (rc == AFSBEM_ENOCONV)
            set_error("at least one frequency did not reach the tolerance");
        return rc;
    });
}

int afsbem_solve(afsbem_problem *p, int32_t n_s, const double *s, const double *bc_val, const double *x0,
                 double *a_out, double *u_out, double *t_out, const afsbem_solve_opts *opts,
                 afsbem_solve_stats *stats) {
    return guarded([&] {
        AFS_REQUIRE(p && s && bc_val, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(n_s >= 0, AFSBEM_EINVAL, "n_s must be >= 0");
        if (n_s == 0)
            return (int)AFSBEM_OK;
        const size_t bytes = (size_t)n_s * 3 * p->p.dev.n_tri * 16;
        const bool need_a = a_out || (opts && opts->warm_start == AFSBEM_WARM_LEARNED);
        std::vector<void *> bufs;
        struct Free {
            std::vector<void *> &b;
            ~Free() {
                for (void *q : b)
                    (void)hipFree(q);
            }
        } fr{bufs};
        auto dev = [&](bool want) -> void * {
            if (!want)
                return nullptr;
            void *q = nullptr;
            hipError_t e = hipMalloc(&q, bytes);
            if (e != hipSuccess)
                throw Error{AFSBEM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
            bufs.push_back(q);
            return q;
        };
        void *d_bc = dev(true), *d_x0 = dev(x0 != nullptr), *d_a = dev(need_a), *d_u = dev(u_out != nullptr),
             *d_t = dev(t_out != nullptr);
        AFS_HIP(hipMemcpy(d_bc, bc_val, bytes, hipMemcpyHostToDevice));
        if (x0)
            AFS_HIP(hipMemcpy(d_x0, x0, bytes, hipMemcpyHostToDevice));
        const int rc = afsbem_solve_device(p, n_s, s, d_bc, d_x0, d_a, d_u, d_t, opts, stats, nullptr);
        if (rc != AFSBEM_OK && rc != AFSBEM_ENOCONV)
            return rc;
        const std::string msg = afsbem_last_error();
        AFS_HIP(hipDeviceSynchronize());
        if (a_out)
            AFS_HIP(hipMemcpy(a_out, d_a, bytes, hipMemcpyDeviceToHost));
        if (u_out)
            AFS_HIP(hipMemcpy(u_out, d_u, bytes, hipMemcpyDeviceToHost));
        if (t_out)
            AFS_HIP(hipMemcpy(t_out, d_t, bytes, hipMemcpyDeviceToHost));
        if (rc == AFSBEM_ENOCONV)
            set_error(msg);
        return rc;
    });
}

int afsbem_solve_batched_device(int32_t n_prob, afsbem_problem *const *probs, const int32_t *n_s,
                                const double *s, const void *const *d_bc_val, void *const *d_a_out,
                                void *const *d_u_out, void *const *d_t_out, const afsbem_solve_opts *opts,
                                afsbem_solve_stats *stats, void *hip_stream) {
    return guarded([&] {
        AFS_REQUIRE(n_prob >= 0, AFSBEM_EINVAL, "n_prob must be >= 0");
        AFS_REQUIRE(n_prob == 0 || (probs && n_s && d_bc_val), AFSBEM_EINVAL, "null pointer argument");
        afsbem_solve_opts o;
        afsbem_solve_opts_default(&o);
        if (opts)
            o = *opts;
        AFS_REQUIRE(o.tol > 0 && o.restart >= 1 && o.restart <= 500 && o.max_iter >= 1, AFSBEM_EINVAL,
                    "invalid solver options");
        AFS_REQUIRE(o.precision == AFSBEM_PREC_FP64 || o.precision == AFSBEM_PREC_MIXED, AFSBEM_EINVAL,
                    "unknown precision");
        AFS_REQUIRE(o.warm_start == AFSBEM_WARM_NONE, AFSBEM_EINVAL, "the batched solve takes no warm start");
        AFS_REQUIRE(o.precond == 0 || o.precond == 1, AFSBEM_EINVAL, "precond must be 0 or 1");
        AFS_REQUIRE(o.matrix_free == 0, AFSBEM_EINVAL, "the batched solve stores its matrices");
        int dev = 0;
        AFS_HIP(hipGetDevice(&dev));
        std::vector<Problem *> pp(n_prob);
        std::vector<const double *> bc(n_prob);
        std::vector<double *> a(n_prob, nullptr), u(n_prob, nullptr), t(n_prob, nullptr);
        int64_t total = 0;
        for (int32_t q = 0; q < n_prob; ++q) {
            AFS_REQUIRE(probs[q] && n_s[q] >= 0, AFSBEM_EINVAL, "null problem or negative n_s");
            AFS_REQUIRE(probs[q]->p.device == dev, AFSBEM_EINVAL, "all problems must live on the current device");
            AFS_REQUIRE(n_s[q] == 0 || d_bc_val[q], AFSBEM_EINVAL, "null d_bc_val entry");
            pp[q] = &probs[q]->p;
            bc[q] = static_cast<const double *>(d_bc_val[q]);
            if (d_a_out)
                a[q] = static_cast<double *>(d_a_out[q]);
            if (d_u_out)
                u[q] = static_cast<double *>(d_u_out[q]);
            if (d_t_out)
                t[q] = static_cast<double *>(d_t_out[q]);
            total += n_s[q];
        }
        AFS_REQUIRE(total == 0 || s, AFSBEM_EINVAL, "null s");
        for (int64_t k = 0; k < total; ++k)
            AFS_REQUIRE(std::isfinite(s[2 * k]) && std::isfinite(s[2 * k + 1]), AFSBEM_EINVAL, "non-finite s");
        if (total == 0)
            return (int)AFSBEM_OK;
        const int rc = solve_batched(n_prob, pp.data(), n_s, s, bc.data(), a.data(), u.data(), t.data(), o, stats,
                                     static_cast<hipStream_t>(hip_stream));
        if (rc == AFSBEM_ENOCONV)
            set_error("at least one system did not reach the tolerance");
        return rc;
    });
}

}  // extern "C"
