// opcount.hpp -- TEST INFRASTRUCTURE ONLY.
//
// A scalar that behaves like double and counts the floating-point operations
// performed on it, so that instantiating the oracle with it yields the
// algorithmic operation count of the method (add/sub, mul, div, sqrt and
// compare, each counted once per scalar operation).  Counting is per thread;
// the counting entry point runs single-threaded.
#ifndef PPM_OPCOUNT_HPP
#define PPM_OPCOUNT_HPP

#include <cmath>
#include <cstdint>

struct OpCountTally {
  int64_t add = 0, mul = 0, div = 0, sqrt = 0, cmp = 0;
};
inline OpCountTally &opc_tally() {
  static thread_local OpCountTally t;
  return t;
}
inline void opc_reset() { opc_tally() = OpCountTally(); }
inline void opc_read(int64_t ops[6]) {
  const OpCountTally &t = opc_tally();
  ops[0] = t.add; ops[1] = t.mul; ops[2] = t.div; ops[3] = t.sqrt; ops[4] = t.cmp; ops[5] = 0;
}

struct OpCount {
  double v;
  OpCount() : v(0.0) {}
  OpCount(double x) : v(x) {}  // NOLINT: implicit, so literals mix with counted values
  friend OpCount operator+(OpCount a, OpCount b) { opc_tally().add++; return OpCount(a.v + b.v); }
  friend OpCount operator-(OpCount a, OpCount b) { opc_tally().add++; return OpCount(a.v - b.v); }
  friend OpCount operator*(OpCount a, OpCount b) { opc_tally().mul++; return OpCount(a.v * b.v); }
  friend OpCount operator/(OpCount a, OpCount b) { opc_tally().div++; return OpCount(a.v / b.v); }
  friend OpCount operator-(OpCount a) { return OpCount(-a.v); }
  friend bool operator<(OpCount a, OpCount b) { opc_tally().cmp++; return a.v < b.v; }
  friend bool operator>(OpCount a, OpCount b) { opc_tally().cmp++; return a.v > b.v; }
  friend bool operator<=(OpCount a, OpCount b) { opc_tally().cmp++; return a.v <= b.v; }
  friend bool operator>=(OpCount a, OpCount b) { opc_tally().cmp++; return a.v >= b.v; }
  friend bool operator==(OpCount a, OpCount b) { opc_tally().cmp++; return a.v == b.v; }
  friend OpCount sqrt(OpCount a) { opc_tally().sqrt++; return OpCount(std::sqrt(a.v)); }
  friend OpCount fabs(OpCount a) { return OpCount(std::fabs(a.v)); }
};

inline double opc_val(double x) { return x; }
inline double opc_val(OpCount x) { return x.v; }

#endif
