// Drives the host setup (validation, overlap expansion, local graphs, coarse
// operator and inverse, local inverses) on a problem read from a directory of
// raw arrays, for a build with AddressSanitizer and UBSan. Prints OK or a reason.
#include <cstdio>
#include <cstdint>
#include <string>
#include <vector>

#include "setup.h"

template <typename T>
static bool load(const std::string& dir, const char* name, std::vector<T>& v) {
    FILE* f = std::fopen((dir + "/" + name).c_str(), "rb");
    if (!f) return false;
    std::fseek(f, 0, SEEK_END);
    const long bytes = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    v.resize((size_t)bytes / sizeof(T));
    const size_t got = std::fread(v.data(), sizeof(T), v.size(), f);
    std::fclose(f);
    return got == v.size();
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    const std::string dir = argv[1];
    std::vector<double> xy, val, b, u0, w;
    std::vector<int32_t> tri, rowptr, col, sub_nodes, part;
    std::vector<uint8_t> dir_flags;
    std::vector<int64_t> sub_ptr, meta;
    if (!load(dir, "xy", xy) || !load(dir, "val", val) || !load(dir, "b", b) || !load(dir, "u0", u0) ||
        !load(dir, "weights", w) || !load(dir, "tri", tri) || !load(dir, "rowptr", rowptr) ||
        !load(dir, "col", col) || !load(dir, "sub_nodes", sub_nodes) || !load(dir, "part", part) ||
        !load(dir, "dirichlet", dir_flags) || !load(dir, "sub_ptr", sub_ptr) || !load(dir, "meta", meta)) {
        std::printf("missing input\n");
        return 1;
    }
    ddmgnn_problem_desc d{};
    d.n_nodes = (int64_t)dir_flags.size();
    d.xy = xy.data();
    d.n_tri = (int64_t)tri.size() / 3;
    d.tri = tri.data();
    d.dirichlet = dir_flags.data();
    d.a_rowptr = rowptr.data();
    d.a_col = col.data();
    d.a_val = val.data();
    d.b = b.data();
    d.u0 = u0.data();
    d.n_sub = (int32_t)sub_ptr.size() - 1;
    d.sub_ptr = sub_ptr.data();
    d.sub_nodes = sub_nodes.data();
    d.weights = w.data();
    std::string e = ddmgnn::validate(d);
    if (!e.empty()) {
        std::printf("validate: %s\n", e.c_str());
        return 1;
    }
    std::vector<int64_t> sp;
    std::vector<int32_t> sn;
    ddmgnn::expand_overlap(d.n_nodes, d.n_tri, d.tri, part.data(), (int32_t)meta[0], (int32_t)meta[1], sp, sn);
    if (sp != sub_ptr || sn != sub_nodes) {
        std::printf("overlap differs\n");
        return 1;
    }
    ddmgnn::HostSetup hs;
    e = ddmgnn::build_setup(d, hs);
    if (!e.empty()) {
        std::printf("setup: %s\n", e.c_str());
        return 1;
    }
    std::vector<double> inv;
    std::vector<int64_t> off;
    e = ddmgnn::build_local_inverses(d, inv, off);
    if (!e.empty()) {
        std::printf("local inverses: %s\n", e.c_str());
        return 1;
    }
    // a malformed copy must be refused, not read out of bounds
    std::vector<int32_t> bad_col(col);
    bad_col[0] = (int32_t)d.n_nodes + 5;
    d.a_col = bad_col.data();
    if (ddmgnn::validate(d).empty()) {
        std::printf("bad column accepted\n");
        return 1;
    }
    std::printf("OK edges=%lld coarse=%zu inverses=%zu\n", (long long)hs.n_edges, hs.a0inv.size(), inv.size());
    return 0;
}
