// CPU harness driver: runs one case through the C ABI of the library
// sources compiled for the host (see include/hip/hip_runtime.h here) under
// AddressSanitizer + UndefinedBehaviorSanitizer.  TEST INFRASTRUCTURE.
//
// usage: driver <case_dir>
//   case_dir/config.txt   "key value" lines: n, storage, steps (comma list of
//                         step counts, run one after another), graph_steps,
//                         shape, and per droplet d: nodes_d, tris_d,
//                         f0dev_d (0/1), force_d (0/1)
//   case_dir/params.bin   n iblb_params records
//   case_dir/pos_d.bin    [dim][N] float64;  tris_d.bin [T][3] int32
//   case_dir/f0dev_d.bin  [Q][cells] float64; force_d.bin [dim][cells] float32
// writes case_dir/out_d_{rho,U,F,fdev,q,qdot,phi,diag}.bin and status.txt
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "iblb.h"

static std::string dir;

template <typename T>
static std::vector<T> load(const std::string& name, size_t count) {
    std::vector<T> v(count);
    FILE* f = fopen((dir + "/" + name).c_str(), "rb");
    if (!f) { fprintf(stderr, "missing %s\n", name.c_str()); exit(3); }
    size_t got = fread(v.data(), sizeof(T), count, f);
    fclose(f);
    if (got != count) { fprintf(stderr, "short %s\n", name.c_str()); exit(3); }
    return v;
}

template <typename T>
static void save(const std::string& name, const T* p, size_t count) {
    FILE* f = fopen((dir + "/" + name).c_str(), "wb");
    fwrite(p, sizeof(T), count, f);
    fclose(f);
}

// exact-size heap buffers so the sanitizer sees any access past their end
template <typename T>
static T* buf(size_t count) {
    void* p = nullptr;
    if (posix_memalign(&p, 256, count * sizeof(T) ? count * sizeof(T) : 1)) exit(4);
    memset(p, 0, count * sizeof(T));
    return static_cast<T*>(p);
}

// Network mode: config "mlp 1", "widths a,b,...", "batch B", "lr x";
// files x.bin [B][w0] f32, t.bin [B][wL] f32, params.bin [P] f32.  Writes
// y.bin, grads.bin, loss.txt and params_after.bin (after one Adam step).
static int run_mlp(std::map<std::string, std::string>& cfg) {
    std::vector<int> w;
    {
        std::stringstream ss(cfg["widths"]);
        std::string tok;
        while (std::getline(ss, tok, ',')) w.push_back(atoi(tok.c_str()));
    }
    const int L = (int)w.size() - 1, B = atoi(cfg["batch"].c_str());
    const float lr = (float)atof(cfg["lr"].c_str());
    size_t ws = iblb_mlp_workspace_bytes(L, w.data(), B);
    if (!ws) return 20;
    char* wsp = buf<char>(ws);
    iblb_mlp* m = nullptr;
    if (iblb_mlp_create(L, w.data(), B, wsp, ws, nullptr, &m)) return 21;
    const long long P = iblb_mlp_param_count(m);
    auto prm = load<float>("params.bin", P);
    auto x = load<float>("x.bin", (size_t)B * w[0]);
    auto t = load<float>("t.bin", (size_t)B * w[L]);
    float* xb = buf<float>(x.size());
    float* tb = buf<float>(t.size());
    float* yb = buf<float>((size_t)B * w[L]);
    float* gb = buf<float>(P);
    float* pb = buf<float>(P);
    memcpy(xb, x.data(), 4 * x.size());
    memcpy(tb, t.data(), 4 * t.size());
    memcpy(pb, prm.data(), 4 * P);
    double loss = 0;
    if (iblb_mlp_set_params(m, pb) || iblb_mlp_forward(m, xb, B, yb) ||
        iblb_mlp_gradients(m, xb, tb, B, gb, &loss) || iblb_mlp_adam_step(m, lr, 0.9f, 0.999f, 1e-8f) ||
        iblb_mlp_get_params(m, pb)) {
        fprintf(stderr, "mlp: %s\n", iblb_mlp_last_error(m));
        return 22;
    }
    save("y.bin", yb, (size_t)B * w[L]);
    save("grads.bin", gb, P);
    save("params_after.bin", pb, P);
    FILE* f = fopen((dir + "/loss.txt").c_str(), "w");
    fprintf(f, "%.17g\n", loss);
    fclose(f);
    iblb_mlp_destroy(m);
    free(xb); free(tb); free(yb); free(gb); free(pb); free(wsp);
    return 0;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    dir = argv[1];
    std::map<std::string, std::string> cfg;
    {
        std::ifstream in(dir + "/config.txt");
        std::string k, v;
        while (in >> k >> v) cfg[k] = v;
    }
    if (cfg.count("mlp")) return run_mlp(cfg);
    auto geti = [&](const std::string& k, int def) { return cfg.count(k) ? atoi(cfg[k].c_str()) : def; };
    const int n = geti("n", 1), storage = geti("storage", 0);
    std::vector<iblb_params> P = load<iblb_params>("params.bin", n);
    const int dim = P[0].dim, Q = dim == 2 ? 9 : 19;
    std::vector<int> nn(n), nt(n);
    for (int d = 0; d < n; ++d) {
        nn[d] = geti("nodes_" + std::to_string(d), 0);
        nt[d] = geti("tris_" + std::to_string(d), 0);
    }
    size_t ws = iblb_workspace_bytes(n, P.data(), nn.data(), nt.data(), storage);
    if (!ws) { fprintf(stderr, "workspace: %s\n", iblb_last_error(nullptr)); return 5; }
    char* w = buf<char>(ws);
    iblb_ctx* ctx = nullptr;
    int rc = iblb_create(n, P.data(), nn.data(), nt.data(), storage, w, ws, nullptr, &ctx);
    if (rc) { fprintf(stderr, "create: %s\n", iblb_last_error(nullptr)); return 6; }
    for (int d = 0; d < n; ++d) {
        const std::string s = std::to_string(d);
        const long cells = (long)P[d].nx * P[d].ny * (dim == 3 ? P[d].nz : 1);
        if (nn[d] > 0) {
            auto pos = load<double>("pos_" + s + ".bin", (size_t)dim * nn[d]);
            std::vector<int32_t> tri;
            if (dim == 3) tri = load<int32_t>("tris_" + s + ".bin", (size_t)3 * nt[d]);
            double* pb = buf<double>(pos.size());
            memcpy(pb, pos.data(), pos.size() * 8);
            int32_t* tb = nullptr;
            if (dim == 3) {
                tb = buf<int32_t>(tri.size());
                memcpy(tb, tri.data(), tri.size() * 4);
            }
            rc = iblb_set_interface(ctx, d, pb, tb);
            free(pb);
            free(tb);
            if (rc) { fprintf(stderr, "set_interface: %s\n", iblb_last_error(ctx)); return 7; }
        }
        if (geti("f0dev_" + s, 0)) {
            auto f = load<double>("f0dev_" + s + ".bin", (size_t)Q * cells);
            double* fb = buf<double>(f.size());
            memcpy(fb, f.data(), f.size() * 8);
            rc = iblb_write_populations(ctx, d, fb);
            free(fb);
            if (rc) return 8;
        }
        if (geti("force_" + s, 0)) {
            auto F = load<float>("force_" + s + ".bin", (size_t)dim * cells);
            float* fb = buf<float>(F.size());
            memcpy(fb, F.data(), F.size() * 4);
            rc = iblb_set_force_field(ctx, d, fb);
            free(fb);
            if (rc) return 9;
        }
    }
    if (cfg.count("graph_steps")) iblb_set_graph_steps(ctx, geti("graph_steps", 64));
    if (cfg.count("shape")) iblb_set_lb_variant(ctx, geti("shape", 0), nullptr);
    if (cfg.count("timing")) iblb_set_timing(ctx, geti("timing", 0));
    for (int d = 0; d < n; ++d)
        if (geti("inactive_" + std::to_string(d), 0)) iblb_set_active(ctx, d, 0);
    for (int d = 0; d < n; ++d) {
        const std::string key = "shear_" + std::to_string(d);
        if (cfg.count(key) && iblb_set_membrane_shear(ctx, d, atof(cfg[key].c_str()))) {
            fprintf(stderr, "membrane shear: %s\n", iblb_last_error(ctx));
            return 16;
        }
    }
    for (int d = 0; d < n; ++d) {
        const std::string key = "respace_" + std::to_string(d);
        if (cfg.count(key) && iblb_set_node_respacing(ctx, d, atof(cfg[key].c_str()))) {
            fprintf(stderr, "node re-spacing: %s\n", iblb_last_error(ctx));
            return 17;
        }
    }
    for (int d = 0; d < n; ++d) {
        const std::string key = "lambda_" + std::to_string(d);
        if (cfg.count(key) && iblb_set_viscosity_ratio(ctx, d, atof(cfg[key].c_str()))) {
            fprintf(stderr, "viscosity ratio: %s\n", iblb_last_error(ctx));
            return 13;
        }
    }
    // inside/outside classification at the initial positions
    auto save_masks = [&](const char* tag) -> int {
        for (int d = 0; d < n; ++d) {
            if (nn[d] == 0) continue;
            const long cells = (long)P[d].nx * P[d].ny * (dim == 3 ? P[d].nz : 1);
            uint8_t* m = buf<uint8_t>(cells);
            if (iblb_inside_mask(ctx, d, m)) {
                fprintf(stderr, "inside mask: %s\n", iblb_last_error(ctx));
                return 14;
            }
            save(std::string(tag) + std::to_string(d) + ".bin", m, cells);
            free(m);
        }
        return 0;
    };
    if (geti("mask", 0) && (rc = save_masks("inside0_"))) return rc;
    int step_rc = 0;
    {
        std::stringstream ss(cfg.count("steps") ? cfg["steps"] : "1");
        std::string tok;
        while (std::getline(ss, tok, ',')) {
            step_rc = iblb_step(ctx, atoi(tok.c_str()));
            if (step_rc) break;
        }
    }
    if (cfg.count("rest")) {  // tol,check_every,hold,max_steps
        double tol = 0;
        int check = 0, hold = 0;
        long long mx = 0;
        sscanf(cfg["rest"].c_str(), "%lf,%d,%d,%lld", &tol, &check, &hold, &mx);
        std::vector<long long> so(n);
        step_rc = iblb_run_to_rest(ctx, tol, 0.0, check, hold, mx, so.data());
        save("rest_steps.bin", so.data(), n);
    }
    if (geti("mask", 0) && step_rc == 0 && (rc = save_masks("inside1_"))) return rc;
    if (cfg.count("contact")) {  // z_cut,flat_tol
        double zc = 0, tol = 0;
        sscanf(cfg["contact"].c_str(), "%lf,%lf", &zc, &tol);
        for (int d = 0; d < n; ++d) {
            if (nn[d] == 0) continue;
            double r[3];
            if (iblb_contact_radius(ctx, d, zc, tol, r)) {
                fprintf(stderr, "contact radius: %s\n", iblb_last_error(ctx));
                return 15;
            }
            save("contact_" + std::to_string(d) + ".bin", r, 3);
        }
    }
    FILE* st = fopen((dir + "/status.txt").c_str(), "w");
    fprintf(st, "%d\n%s\n", step_rc, iblb_last_error(ctx));
    fclose(st);
    std::vector<iblb_diag> dg(n);
    rc = iblb_diagnostics(ctx, -1, dg.data());
    if (rc) { fprintf(stderr, "diag: %s\n", iblb_last_error(ctx)); return 10; }
    for (int d = 0; d < n; ++d) {
        const std::string s = std::to_string(d);
        const long cells = (long)P[d].nx * P[d].ny * (dim == 3 ? P[d].nz : 1);
        float* rho = buf<float>(cells);
        float* U = buf<float>((size_t)dim * cells);
        float* F = buf<float>((size_t)dim * cells);
        double* fd = buf<double>((size_t)Q * cells);
        if (iblb_read_fields(ctx, d, rho, U, F) || iblb_read_populations(ctx, d, fd)) return 11;
        save("out_" + s + "_rho.bin", rho, cells);
        save("out_" + s + "_U.bin", U, (size_t)dim * cells);
        save("out_" + s + "_F.bin", F, (size_t)dim * cells);
        save("out_" + s + "_fdev.bin", fd, (size_t)Q * cells);
        free(rho); free(U); free(F); free(fd);
        if (nn[d] > 0) {
            double* q = buf<double>((size_t)dim * nn[d]);
            float* v = buf<float>((size_t)dim * nn[d]);
            float* ph = buf<float>((size_t)dim * nn[d]);
            if (iblb_read_nodes(ctx, d, q, v, ph)) return 12;
            save("out_" + s + "_q.bin", q, (size_t)dim * nn[d]);
            save("out_" + s + "_qdot.bin", v, (size_t)dim * nn[d]);
            save("out_" + s + "_phi.bin", ph, (size_t)dim * nn[d]);
            free(q); free(v); free(ph);
        }
        save("out_" + s + "_diag.bin", &dg[d], 1);
    }
    iblb_destroy(ctx);
    free(w);
    return 0;
}
