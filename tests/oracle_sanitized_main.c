/*
 * Driver for the sanitized build of the oracle (AddressSanitizer + UndefinedBehaviorSanitizer,
 * compiled by tests/test_oracle_sanitized.py).  The oracle's own source is included, so the
 * sanitizers see exactly the code the other tests call through ctypes.
 *
 * Input (stdin, little-endian): repeated records { int64 n; int64 m; int32 src[m]; int32 dst[m] }
 * until end of file.  For each graph every oracle routine runs and the routines that must agree
 * are compared here; one line per graph goes to stdout:
 *   n m_undirected sum_t sum_lcc_bits_xor sum_edge_counts m_directed sum_directed_numerator
 * The test compares these lines with the normal build's results.  Exit status 1 on a mismatch
 * between routines; the sanitizers abort on any out-of-bounds access or undefined behaviour.
 */
#include <stdio.h>

#include "../oracle/oracle.c"

static int check_equal(const uint64_t* a, const uint64_t* b, int64_t n, const char* what) {
    for (int64_t i = 0; i < n; ++i)
        if (a[i] != b[i]) {
            fprintf(stderr, "%s differs at %lld: %llu vs %llu\n", what, (long long)i, (unsigned long long)a[i],
                    (unsigned long long)b[i]);
            return 1;
        }
    return 0;
}

int main(void) {
    int64_t hdr[2];
    int bad = 0;
    while (fread(hdr, sizeof(int64_t), 2, stdin) == 2) {
        const int64_t n = hdr[0], m_in = hdr[1];
        int32_t* src = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m_in + 1));
        int32_t* dst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m_in + 1));
        if (fread(src, sizeof(int32_t), (size_t)m_in, stdin) != (size_t)m_in ||
            fread(dst, sizeof(int32_t), (size_t)m_in, stdin) != (size_t)m_in) {
            fprintf(stderr, "truncated input\n");
            return 2;
        }
        int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m_in + 1));
        const int64_t nnz = oracle_csr(n, m_in, src, dst, off, adj);
        if (nnz < 0) return 3;
        const int64_t m = nnz / 2;
        uint64_t* tf = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
        uint64_t* te = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
        uint64_t* tv = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
        double* lcc = (double*)malloc(sizeof(double) * (size_t)n);
        uint8_t* mark = (uint8_t*)calloc((size_t)n, 1);
        oracle_tc_forward(n, off, adj, tf);
        for (int method = 0; method < 3; ++method) {
            oracle_tc_edge_centric(n, off, adj, method, te);
            bad |= check_equal(tf, te, n, "edge-centric vs forward");
        }
        if (n <= 300) {
            oracle_tc_brute(n, off, adj, te);
            bad |= check_equal(tf, te, n, "brute force vs forward");
        }
        for (int64_t v = 0; v < n; ++v) tv[v] = oracle_tc_vertex(off, adj, (int32_t)v, mark);
        bad |= check_equal(tf, tv, n, "vertex at a time vs forward");
        for (int64_t v = 0; v < n && v < 64; ++v) {
            int64_t dv = -1;
            tv[v] = oracle_tc_vertex_pairs(m_in, src, dst, (int32_t)v, mark, &dv);
            if (dv != off[v + 1] - off[v]) {
                fprintf(stderr, "vertex from raw pairs: degree %lld of %lld, want %lld\n", (long long)dv, (long long)v,
                        (long long)(off[v + 1] - off[v]));
                bad = 1;
            }
        }
        bad |= check_equal(tf, tv, n < 64 ? n : 64, "vertex from raw pairs vs forward");
        oracle_lcc(n, off, tf, lcc);
        uint64_t sum_t = 0, lx = 0;
        for (int64_t v = 0; v < n; ++v) {
            sum_t += tf[v];
            uint64_t bits;
            memcpy(&bits, &lcc[v], sizeof(bits));
            lx ^= bits + (uint64_t)v * 0x9E3779B97F4A7C15ull;
        }
        int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
        int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
        uint64_t* ec = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m + 1));
        const int64_t me = oracle_edge_counts(n, off, adj, eu, ev, ec);
        uint64_t sum_c = 0;
        for (int64_t e = 0; e < me; ++e) sum_c += ec[e];
        if (me != m || sum_c != sum_t) {
            fprintf(stderr, "edge counts: %lld edges (want %lld), sum %llu (want %llu)\n", (long long)me,
                    (long long)m, (unsigned long long)sum_c, (unsigned long long)sum_t);
            bad = 1;
        }
        int64_t* doff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int32_t* dadj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m_in + 1));
        const int64_t md = oracle_csr_directed(n, m_in, src, dst, doff, dadj);
        uint64_t* num = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
        double* dl = (double*)malloc(sizeof(double) * (size_t)n);
        oracle_tc_directed(n, doff, dadj, num);
        oracle_lcc_directed(n, doff, num, dl);
        uint64_t sum_num = 0;
        for (int64_t v = 0; v < n; ++v) sum_num += num[v];
        printf("%lld %lld %llu %llu %llu %lld %llu\n", (long long)n, (long long)m, (unsigned long long)sum_t,
               (unsigned long long)lx, (unsigned long long)sum_c, (long long)md, (unsigned long long)sum_num);
        free(src);
        free(dst);
        free(off);
        free(adj);
        free(tf);
        free(te);
        free(tv);
        free(lcc);
        free(mark);
        free(eu);
        free(ev);
        free(ec);
        free(doff);
        free(dadj);
        free(num);
        free(dl);
    }
    return bad;
}
