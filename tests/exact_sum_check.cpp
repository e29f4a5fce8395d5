// CPU check of the exact-sum limbs of the member means
// (paper_1805_00569_amd/csrc/exact_sum.hpp): reads "f" or "d", a number of
// accumulators A, then the values as hexadecimal bit patterns, one per line,
// until the end of input.  Value i goes to accumulator i mod A (as a thread of
// the mean kernel takes every A-th member), each accumulator normalises its
// limbs after every ExactSum<T>::ADDS values and at the end, the accumulators'
// limbs are added, and the sum is rounded once.  Prints the FP64 result as a
// hexadecimal bit pattern.
#define __host__
#define __device__
#define __forceinline__ inline
#include "../paper_1805_00569_amd/csrc/exact_sum.hpp"

#include <cinttypes>
#include <cstdio>
#include <vector>

template <typename T, typename U>
static int run(int A) {
  constexpr int NL = krr::ExactSum<T>::NL;
  std::vector<std::vector<int64_t>> acc(A, std::vector<int64_t>(NL, 0));
  std::vector<int> since(A, 0);
  unsigned long long bits;
  long long i = 0;
  while (scanf("%llx", &bits) == 1) {
    const U ub = (U)bits;
    T x;
    memcpy(&x, &ub, sizeof(T));
    std::vector<int64_t>& a = acc[i % A];
    const krr::XsTerms t = krr::xs_terms(x);
    a[t.l0] += t.c0;
    if (sizeof(T) == 8) a[t.l1] += t.c1;
    int& s = since[i % A];
    if (++s == krr::ExactSum<T>::ADDS) {
      krr::xs_normalise<NL>([&](int k) { return a[k]; }, [&](int k, int64_t v) { a[k] = v; });
      s = 0;
    }
    ++i;
  }
  std::vector<int64_t> tot(NL, 0);
  for (auto& a : acc) {
    krr::xs_normalise<NL>([&](int k) { return a[k]; }, [&](int k, int64_t v) { a[k] = v; });
    for (int k = 0; k < NL; ++k) tot[k] += a[k];
  }
  const double r = krr::xs_round<T>(tot.data());
  uint64_t rb;
  memcpy(&rb, &r, 8);
  printf("%016" PRIx64 "\n", rb);
  return 0;
}

int main() {
  char kind[4];
  int A;
  if (scanf("%3s %d", kind, &A) != 2 || A < 1) return 2;
  return kind[0] == 'f' ? run<float, uint32_t>(A) : run<double, uint64_t>(A);
}
