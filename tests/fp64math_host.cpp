// Host build of the pair kernels' FP64 exp and rsqrt refinement, for the
// accuracy test (tests/test_host_logic.py loads it with ctypes).
#include "../paper_1412_8502_amd/csrc/fp64math.hpp"

extern "C" double host_exp_nonpos(double x) { return pasta::exp_nonpos(x); }
extern "C" double host_rsqrt_refine(double x, double y0) { return pasta::rsqrt_refine(x, y0); }
