// Host-code exerciser for the address and undefined-behaviour sanitizers:
// graph construction and validation of the C ABI (graph.cpp, no HIP calls)
// on random and invalid inputs, and the FP64 reference decoders (oracle/bp.c)
// on random codes.  Prints "OK" when every call returned as expected.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "ldpc.h"

extern "C" {
int oracle_decode_block(int n, int m, const int32_t* row_ptr, const int32_t* col_idx, const float* llr, int gamma,
                        int max_iters, int early_stop, double lmax, int nthreads, double* post, uint8_t* bits,
                        int32_t* iters, uint8_t* converged, double* min_abs, uint8_t* syn_trace, double near,
                        int32_t* fragile, double* L_trace);
int oracle_decode_window(int n, int m, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* layer_of_row,
                         const int32_t* pos_of_col, int nlayers, int npos, const float* llr, int gamma, int W, int K,
                         double lmax, int nthreads, double* post, uint8_t* bits);
int oracle_decode_pipeline(int n, int m, const int32_t* row_ptr, const int32_t* col_idx,
                           const int32_t* layer_of_row, const int32_t* pos_of_col, int nlayers, int npos, int ms,
                           const float* llr, int gamma, int I, double lmax, int nthreads, double* post,
                           uint8_t* bits);
}

static int failures = 0;
#define EXPECT(c)                                                              \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "line %d: %s\n", __LINE__, #c);               \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

static void fuzz_graphs(std::mt19937_64& rng) {
    std::uniform_int_distribution<int> small(-2, 40);
    for (int trial = 0; trial < 3000; ++trial) {
        const int J = small(rng) % 10, L = small(rng) % 20, p = small(rng);
        const int cells = (J > 0 && L > 0) ? J * L : 1;
        std::vector<int32_t> a(cells);
        for (auto& x : a) x = (int32_t)(rng() % (std::max(p, 1) + 3)) - 2;   // some out of range
        ldpc_graph* g = nullptr;
        const ldpc_status st = ldpc_graph_create_qc(a.data(), J, L, p, &g);
        if (st == LDPC_OK) {
            ldpc_graph_info info;
            EXPECT(ldpc_graph_get_info(g, &info) == LDPC_OK);
            EXPECT(info.n == L * p && info.m == J * p);
            ldpc_graph_destroy(g);
        } else {
            EXPECT(g == nullptr);
        }
        ldpc_graph* c = nullptr;
        const int positions = (int)(rng() % 12) - 1;
        const ldpc_status sc = ldpc_graph_create_ldpccc_from_qc(a.data(), J, L, p, positions, (int)(rng() & 1), &c);
        if (sc == LDPC_OK) {
            ldpc_graph_info info;
            EXPECT(ldpc_graph_get_info(c, &info) == LDPC_OK);
            ldpc_graph_destroy(c);
        }
        // syndrome-former form with random sizes
        const int T = (int)(rng() % 4), ms = (int)(rng() % 4) - 1, Jb = (int)(rng() % 3), Lb = (int)(rng() % 4);
        const int sfn = std::max(T, 1) * std::max(ms + 1, 1) * std::max(Jb, 1) * std::max(Lb, 1);
        std::vector<int32_t> sf(sfn);
        for (auto& x : sf) x = (int32_t)(rng() % (std::max(p, 1) + 2)) - 1;
        ldpc_graph* s = nullptr;
        if (ldpc_graph_create_ldpccc_sf(sf.data(), T, ms, Jb, Lb, p, positions, 1, &s) == LDPC_OK) {
            ldpc_graph_info info;
            EXPECT(ldpc_graph_get_info(s, &info) == LDPC_OK);
            ldpc_graph_destroy(s);
        }
    }
    for (int code = -6; code <= 1; ++code) EXPECT(ldpc_status_str((ldpc_status)code) != nullptr);
    ldpc_graph_destroy(nullptr);
}

// random banded chain: layer t's rows meet positions t-ms..t
struct Chain {
    int n = 0, m = 0, nlayers, npos, ms;
    std::vector<int32_t> row_ptr{0}, col_idx, layer_of_row, pos_of_col;
};

static Chain random_chain(std::mt19937_64& rng, int npos, int ms, int c, int rows_per_layer) {
    Chain h;
    h.npos = npos;
    h.ms = ms;
    h.nlayers = npos + ms;
    h.n = npos * c;
    for (int v = 0; v < h.n; ++v) h.pos_of_col.push_back(v / c);
    for (int t = 0; t < h.nlayers; ++t) {
        for (int r = 0; r < rows_per_layer; ++r) {
            std::vector<int32_t> cols;
            for (int d = ms; d >= 0; --d) {
                const int pos = t - d;
                if (pos < 0 || pos >= npos) continue;
                const int k = 1 + (int)(rng() % 2);
                for (int i = 0; i < k; ++i) {
                    const int32_t v = pos * c + (int32_t)(rng() % c);
                    if (std::find(cols.begin(), cols.end(), v) == cols.end()) cols.push_back(v);
                }
            }
            if (cols.empty()) continue;
            std::sort(cols.begin(), cols.end());
            for (int32_t v : cols) h.col_idx.push_back(v);
            h.row_ptr.push_back((int32_t)h.col_idx.size());
            h.layer_of_row.push_back(t);
            ++h.m;
        }
    }
    return h;
}

static void run_oracle(std::mt19937_64& rng) {
    std::normal_distribution<float> noise(1.5f, 2.0f);
    for (int trial = 0; trial < 20; ++trial) {
        const int npos = 2 + (int)(rng() % 6), ms = (int)(rng() % 3), c = 4 + (int)(rng() % 6);
        Chain h = random_chain(rng, npos, ms, c, 2 + (int)(rng() % 3));
        const int gamma = 1 + (int)(rng() % 5);
        std::vector<float> llr((size_t)gamma * h.n);
        for (auto& x : llr) x = noise(rng);
        std::vector<double> post(llr.size()), min_abs(gamma);
        std::vector<uint8_t> bits(llr.size()), conv(gamma), trace((size_t)gamma * 8);
        std::vector<int32_t> iters(gamma), fragile(gamma);
        std::vector<double> Ltr((size_t)gamma * 8 * h.n);
        EXPECT(oracle_decode_block(h.n, h.m, h.row_ptr.data(), h.col_idx.data(), llr.data(), gamma, 8, 1, 30.0, 2,
                                   post.data(), bits.data(), iters.data(), conv.data(), min_abs.data(),
                                   trace.data(), 0.5, fragile.data(), Ltr.data()) == 0);
        for (int g = 0; g < gamma; ++g) EXPECT(iters[g] >= 1 && iters[g] <= 8);
        for (int g = 0; g < gamma; ++g) EXPECT(fragile[g] >= 0 && fragile[g] <= iters[g]);
        const int W = ms + 1 + (int)(rng() % 4);
        EXPECT(oracle_decode_window(h.n, h.m, h.row_ptr.data(), h.col_idx.data(), h.layer_of_row.data(),
                                    h.pos_of_col.data(), h.nlayers, h.npos, llr.data(), gamma, W, 3, 30.0, 2,
                                    post.data(), bits.data()) == 0);
        EXPECT(oracle_decode_pipeline(h.n, h.m, h.row_ptr.data(), h.col_idx.data(), h.layer_of_row.data(),
                                      h.pos_of_col.data(), h.nlayers, h.npos, ms, llr.data(), gamma,
                                      1 + (int)(rng() % 4), 30.0, 2, post.data(), bits.data()) == 0);
        for (double x : post) EXPECT(x >= -30.0 && x <= 30.0);
    }
    // invalid arguments are refused
    int32_t rp[2] = {0, 0};
    EXPECT(oracle_decode_block(0, 1, rp, nullptr, nullptr, 1, 0, 0, 30.0, 1, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr, 1e-3, nullptr, nullptr) == -1);
}

int main() {
    std::mt19937_64 rng(12345);
    fuzz_graphs(rng);
    run_oracle(rng);
    if (failures) {
        std::printf("FAILED %d\n", failures);
        return 1;
    }
    std::printf("OK\n");
    return 0;
}
