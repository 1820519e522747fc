// Host-sanitizer driver (AddressSanitizer + UndefinedBehaviorSanitizer) for
// the plain C++ of the repository: the input generators (workloads/gen.cpp)
// and the oracle (oracle/oracle.cpp), linked into one program and driven
// through their C entry points on small inputs of every kind, index width
// and value width, with several host threads.  Exits non-zero on a
// mismatch; the sanitizers abort on any memory or UB error.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
int wl_er(int64_t n, int64_t m, int d, uint64_t seed, int64_t* rowptr, void* col, int col_width,
          int nthreads);
int64_t wl_er_wide(int64_t n, int64_t m, int d, uint64_t seed, const uint8_t* mask,
                   int64_t* rowptr, void* col, int col_width, int nthreads);
int64_t wl_banded(int64_t n, int64_t w, int k, uint64_t seed, int64_t* rowptr, void* col,
                  int col_width, int nthreads);
int64_t wl_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed,
                int merge, int64_t* rowptr, void* col, int col_width, int nthreads);
int wl_values(int64_t nnz, uint64_t seed, int kind, void* out, int val_width, int nthreads);
int64_t oracle_ip(int64_t nA, int64_t mA, const void* Arp, int Arpw, const void* Acol, int Acolw,
                  int64_t nB, int64_t mB, const void* Brp, int Brpw, const void* Bcol, int Bcolw,
                  const int64_t* rows, int64_t nreq, int64_t* ip_out);
void* oracle_spgemm(int64_t nA, int64_t mA, const void* Arp, int Arpw, const void* Acol, int Acolw,
                    const void* Aval, int64_t nB, int64_t mB, const void* Brp, int Brpw,
                    const void* Bcol, int Bcolw, const void* Bval, int valw, const int64_t* rows,
                    int64_t nreq, int nthreads);
int64_t oracle_nnz(void* h);
int64_t oracle_nrows(void* h);
void oracle_fetch(void* h, int64_t* rowptr, int64_t* col, double* val, double* ref, double* abssum);
void oracle_free(void* h);
}

struct Csr {
  int64_t n = 0, m = 0;
  std::vector<int64_t> rp64;
  std::vector<int32_t> rp32;
  std::vector<unsigned char> col, val;
  int rpw = 8, cw = 4, vw = 8;
  const void* rp() const { return rpw == 8 ? (const void*)rp64.data() : (const void*)rp32.data(); }
};

static void finish(Csr& X, int64_t nnz, int rpw, int cw, int vw, uint64_t seed, int kind) {
  X.rpw = rpw;
  X.cw = cw;
  X.vw = vw;
  X.col.resize((size_t)nnz * cw);  // already filled by the generator at its own capacity
  X.val.resize((size_t)(nnz ? nnz : 1) * vw);
  if (wl_values(nnz, seed, kind, X.val.data(), vw, 3) != 0) std::exit(3);
  if (rpw == 4) X.rp32.assign(X.rp64.begin(), X.rp64.end());
}

static int fails = 0;

static void check(const char* name, const Csr& A, const Csr& B, int threads) {
  std::vector<int64_t> ip(A.n);
  const int64_t tot = oracle_ip(A.n, A.m, A.rp(), A.rpw, A.col.data(), A.cw, B.n, B.m, B.rp(),
                                B.rpw, B.col.data(), B.cw, nullptr, 0, ip.data());
  void* h = oracle_spgemm(A.n, A.m, A.rp(), A.rpw, A.col.data(), A.cw, A.val.data(), B.n, B.m,
                          B.rp(), B.rpw, B.col.data(), B.cw, B.val.data(), A.vw, nullptr, 0,
                          threads);
  if (!h) {
    std::printf("%s: oracle rejected\n", name);
    ++fails;
    return;
  }
  const int64_t nnz = oracle_nnz(h), nr = oracle_nrows(h);
  std::vector<int64_t> rp(nr + 1), col(nnz ? nnz : 1);
  std::vector<double> val(nnz ? nnz : 1), ref(nnz ? nnz : 1), ab(nnz ? nnz : 1);
  oracle_fetch(h, rp.data(), col.data(), val.data(), ref.data(), ab.data());
  oracle_free(h);
  // invariants: nnz <= ip per row, ascending columns within a row, inside [0, m)
  for (int64_t i = 0; i < nr; ++i) {
    if (rp[i + 1] - rp[i] > ip[i]) ++fails;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= B.m) ++fails;
      if (e > rp[i] && col[e] <= col[e - 1]) ++fails;
    }
  }
  // a subset of rows, in a different order of threads, gives the same rows
  std::vector<int64_t> rows;
  for (int64_t i = 0; i < A.n; i += 3) rows.push_back(i);
  void* h2 = oracle_spgemm(A.n, A.m, A.rp(), A.rpw, A.col.data(), A.cw, A.val.data(), B.n, B.m,
                           B.rp(), B.rpw, B.col.data(), B.cw, B.val.data(), A.vw, rows.data(),
                           (int64_t)rows.size(), 1);
  const int64_t nnz2 = oracle_nnz(h2);
  std::vector<int64_t> rp2(rows.size() + 1), col2(nnz2 ? nnz2 : 1);
  std::vector<double> v2(nnz2 ? nnz2 : 1), r2(nnz2 ? nnz2 : 1), a2(nnz2 ? nnz2 : 1);
  oracle_fetch(h2, rp2.data(), col2.data(), v2.data(), r2.data(), a2.data());
  oracle_free(h2);
  for (size_t k = 0; k < rows.size(); ++k) {
    const int64_t i = rows[k];
    if (rp2[k + 1] - rp2[k] != rp[i + 1] - rp[i]) {
      ++fails;
      continue;
    }
    for (int64_t q = 0; q < rp2[k + 1] - rp2[k]; ++q)
      if (col2[rp2[k] + q] != col[rp[i] + q] || v2[rp2[k] + q] != val[rp[i] + q]) ++fails;
  }
  std::printf("%s: ip %lld nnz %lld fails %d\n", name, (long long)tot, (long long)nnz, fails);
}

int main() {
  for (int rpw : {4, 8})
    for (int cw : {4, 8})
      for (int vw : {4, 8}) {
        Csr A, B;
        // Erdos-Renyi A (300 x 400), banded B (400 x 400)
        A.n = 300;
        A.m = 400;
        A.rp64.resize(A.n + 1);
        A.col.resize((size_t)A.n * 7 * cw);
        if (wl_er(A.n, A.m, 7, 11, A.rp64.data(), A.col.data(), cw, 3) != 0) return 3;
        finish(A, A.rp64[A.n], rpw, cw, vw, 12, 0);
        B.n = B.m = 400;
        B.rp64.resize(B.n + 1);
        B.col.resize((size_t)B.n * 9 * cw);
        const int64_t nb = wl_banded(B.n, 64, 8, 13, B.rp64.data(), B.col.data(), cw, 2);
        finish(B, nb, rpw, cw, vw, 14, 1);
        char name[64];
        std::snprintf(name, sizeof name, "er x banded rp%d col%d val%d", rpw * 8, cw * 8, vw * 8);
        check(name, A, B, 4);
        // R-MAT squared, scale 9, and a wide ER with empty rows
        Csr R;
        R.n = R.m = 512;
        R.rp64.resize(R.n + 1);
        R.col.resize((size_t)16 * 512 * cw);
        const int64_t nr = wl_rmat(9, 16, 0.57, 0.19, 0.19, 15, 1, R.rp64.data(), R.col.data(), cw, 3);
        finish(R, nr, rpw, cw, vw, 16, 0);
        std::snprintf(name, sizeof name, "rmat9^2 rp%d col%d val%d", rpw * 8, cw * 8, vw * 8);
        check(name, R, R, 3);
        Csr W;
        W.n = 512;
        W.m = 1 << 16;
        std::vector<uint8_t> mask(W.n);
        for (int64_t i = 0; i < W.n; ++i) mask[i] = (uint8_t)(i % 3 != 0);
        W.rp64.resize(W.n + 1);
        W.col.resize((size_t)W.n * 20 * cw);
        const int64_t nw = wl_er_wide(W.n, W.m, 20, 17, mask.data(), W.rp64.data(), W.col.data(), cw, 2);
        if (nw < 0) return 3;
        finish(W, nw, rpw, cw, vw, 18, 0);
        std::snprintf(name, sizeof name, "rmat9 x wide rp%d col%d val%d", rpw * 8, cw * 8, vw * 8);
        check(name, R, W, 2);
      }
  std::printf("total fails %d\n", fails);
  return fails ? 1 : 0;
}
