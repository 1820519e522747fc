// CPU ORACLE -- test infrastructure only.
//
// Only the tests, the smoke check and the benchmark's CPU-baseline leg may
// load this library.  The product path never calls it and shares no source
// with it.
//
// What it computes: the plain definition of the sparse product C = A*B by
// Gustavson's row-wise formula (Section 2.1, Eq. 1): row i of C is the sum,
// over the stored entries (i, j) of A, of A_ij times row j of B.  The
// reordering of the paper's method changes only the order in which products
// are summed (Sections 1 and 3.1), so the definition is the oracle.
//
// The accumulator is an ordered map keyed by column (Section 2.1 names a map
// as the alternative to the dense accumulator).  Following the dense
// accumulation algorithm (Section 2.1, Algorithm 1):
//   * each accumulator slot starts at +0.0 and products are added in stored
//     order: for each entry of A's row in stored order, for each entry of the
//     B row in stored order;
//   * a column present in the structure is kept even when its sum is zero;
//   * the product is rounded to the value type before it is added (this file
//     is compiled with -ffp-contract=off, so no fused multiply-add).
// The output row lists columns in ascending order.
//
// Besides that input-precision sum ("val") each entry carries
//   * "ref": the same sum accumulated in long double from long double
//     products (the high-precision value the error bound is measured from);
//   * "abssum": the sum of |product| (the scale of the summation error bound
//     |c - c_exact| <= gamma_k * sum |a_ik b_kj|).
//
// The intermediate-product count of a row is the number of products the
// formula forms, nnz of B_j summed over the entries (i, j) of A (Section 4.3,
// n_interProd).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <thread>
#include <vector>

namespace {

struct Acc {
  double val = 0.0;        // input-precision running sum (float sums are exact in double storage)
  long double ref = 0.0L;  // high-precision running sum
  long double abs = 0.0L;  // running sum of |product|
};

struct Mat {
  int64_t n, m;
  const void* rp; int rpw;
  const void* col; int colw;
  const void* val; int valw;
  int64_t rowptr(int64_t i) const {
    return rpw == 4 ? (int64_t)((const int32_t*)rp)[i] : ((const int64_t*)rp)[i];
  }
  int64_t colidx(int64_t k) const {
    return colw == 4 ? (int64_t)((const int32_t*)col)[k] : ((const int64_t*)col)[k];
  }
  double value(int64_t k) const {
    return valw == 4 ? (double)((const float*)val)[k] : ((const double*)val)[k];
  }
};

struct RowOut {
  std::vector<int64_t> col;
  std::vector<double> val, ref, abs;
};

struct Result {
  std::vector<int64_t> rows;      // requested rows, in output order
  std::vector<int64_t> rownnz;    // per requested row
  std::vector<RowOut> parts;      // per thread block, concatenated in order
  std::vector<int64_t> part_rows; // number of rows in each part
  int64_t nnz = 0;
};

int64_t row_ip(const Mat& A, const Mat& B, int64_t i) {
  int64_t s = 0;
  for (int64_t p = A.rowptr(i); p < A.rowptr(i + 1); ++p) {
    int64_t j = A.colidx(p);
    s += B.rowptr(j + 1) - B.rowptr(j);
  }
  return s;
}

void compute_row(const Mat& A, const Mat& B, int64_t i, bool f32, RowOut& out, int64_t& nnz) {
  std::map<int64_t, Acc> acc;
  for (int64_t p = A.rowptr(i); p < A.rowptr(i + 1); ++p) {
    const int64_t j = A.colidx(p);
    const double a = A.value(p);
    for (int64_t q = B.rowptr(j); q < B.rowptr(j + 1); ++q) {
      const int64_t k = B.colidx(q);
      const double b = B.value(q);
      Acc& s = acc[k];  // a new key starts at +0.0
      if (f32) {
        const float t = (float)a * (float)b;
        s.val = (double)((float)s.val + t);
      } else {
        const double t = a * b;
        s.val = s.val + t;
      }
      const long double tl = (long double)a * (long double)b;
      s.ref += tl;
      s.abs += fabsl(tl);
    }
  }
  for (const auto& kv : acc) {
    out.col.push_back(kv.first);
    out.val.push_back(kv.second.val);
    out.ref.push_back((double)kv.second.ref);
    out.abs.push_back((double)kv.second.abs);
  }
  nnz = (int64_t)acc.size();
}

}  // namespace

extern "C" {

// Intermediate-product count of each requested row (all rows when rows is
// null).  Returns the total.
int64_t oracle_ip(int64_t nA, int64_t mA, const void* Arp, int Arpw, const void* Acol, int Acolw,
                  int64_t nB, int64_t mB, const void* Brp, int Brpw, const void* Bcol, int Bcolw,
                  const int64_t* rows, int64_t nreq, int64_t* ip_out) {
  (void)mA; (void)mB; (void)nB;
  Mat A{nA, mA, Arp, Arpw, Acol, Acolw, nullptr, 8};
  Mat B{nB, mB, Brp, Brpw, Bcol, Bcolw, nullptr, 8};
  int64_t cnt = rows ? nreq : nA, tot = 0;
  for (int64_t r = 0; r < cnt; ++r) {
    int64_t v = row_ip(A, B, rows ? rows[r] : r);
    if (ip_out) ip_out[r] = v;
    tot += v;
  }
  return tot;
}

// C rows for the requested rows (all rows when rows is null), computed by
// nthreads host threads (<= 0: all hardware threads) over contiguous blocks
// of rows holding about equal intermediate-product counts.  Returns an
// opaque handle, or null on bad arguments (shape mismatch, widths).
void* oracle_spgemm(int64_t nA, int64_t mA, const void* Arp, int Arpw, const void* Acol, int Acolw,
                    const void* Aval, int64_t nB, int64_t mB, const void* Brp, int Brpw,
                    const void* Bcol, int Bcolw, const void* Bval, int valw, const int64_t* rows,
                    int64_t nreq, int nthreads) {
  if (mA != nB) return nullptr;
  if ((Arpw != 4 && Arpw != 8) || (Brpw != 4 && Brpw != 8) || (Acolw != 4 && Acolw != 8) ||
      (Bcolw != 4 && Bcolw != 8) || (valw != 4 && valw != 8))
    return nullptr;
  Mat A{nA, mA, Arp, Arpw, Acol, Acolw, Aval, valw};
  Mat B{nB, mB, Brp, Brpw, Bcol, Bcolw, Bval, valw};
  const bool f32 = (valw == 4);
  Result* res = new Result();
  int64_t cnt = rows ? nreq : nA;
  res->rows.resize(cnt);
  for (int64_t r = 0; r < cnt; ++r) res->rows[r] = rows ? rows[r] : r;
  res->rownnz.assign(cnt, 0);
  if (nthreads <= 0) {
    unsigned h = std::thread::hardware_concurrency();
    nthreads = h ? (int)h : 1;
  }
  // split rows into contiguous blocks with about equal work (ip + 1 per row)
  std::vector<int64_t> work(cnt + 1, 0);
  for (int64_t r = 0; r < cnt; ++r) work[r + 1] = work[r] + row_ip(A, B, res->rows[r]) + 1;
  int nparts = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads, cnt));
  std::vector<int64_t> cut(nparts + 1, cnt);
  cut[0] = 0;
  for (int t = 1; t < nparts; ++t) {
    int64_t target = work[cnt] * t / nparts;
    cut[t] = std::lower_bound(work.begin(), work.end(), target) - work.begin();
    cut[t] = std::min<int64_t>(std::max<int64_t>(cut[t], cut[t - 1]), cnt);
  }
  res->parts.resize(nparts);
  res->part_rows.resize(nparts);
  std::vector<std::thread> ts;
  for (int t = 0; t < nparts; ++t) {
    ts.emplace_back([&, t] {
      for (int64_t r = cut[t]; r < cut[t + 1]; ++r)
        compute_row(A, B, res->rows[r], f32, res->parts[t], res->rownnz[r]);
    });
    res->part_rows[t] = cut[t + 1] - cut[t];
  }
  for (auto& th : ts) th.join();
  for (int64_t r = 0; r < cnt; ++r) res->nnz += res->rownnz[r];
  return res;
}

int64_t oracle_nnz(void* h) { return h ? ((Result*)h)->nnz : -1; }
int64_t oracle_nrows(void* h) { return h ? (int64_t)((Result*)h)->rows.size() : -1; }

// Copies out: rowptr[nrows+1] (offsets over the requested rows), col, val,
// ref, abssum [nnz].  Any output pointer may be null.
void oracle_fetch(void* h, int64_t* rowptr, int64_t* col, double* val, double* ref, double* abssum) {
  Result* res = (Result*)h;
  if (!res) return;
  if (rowptr) {
    rowptr[0] = 0;
    for (size_t r = 0; r < res->rownnz.size(); ++r) rowptr[r + 1] = rowptr[r] + res->rownnz[r];
  }
  int64_t off = 0;
  for (const RowOut& p : res->parts) {
    size_t k = p.col.size();
    if (col) std::copy(p.col.begin(), p.col.end(), col + off);
    if (val) std::copy(p.val.begin(), p.val.end(), val + off);
    if (ref) std::copy(p.ref.begin(), p.ref.end(), ref + off);
    if (abssum) std::copy(p.abs.begin(), p.abs.end(), abssum + off);
    off += (int64_t)k;
  }
}

void oracle_free(void* h) { delete (Result*)h; }

}  // extern "C"
