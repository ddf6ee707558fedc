// Host build of the fusion kernel's fixed-point helpers (gsdf_fixed.hpp),
// exposed through a C ABI for tests/test_fixed_point.py.  The header is
// written for host and device; built by g++ the qualifiers are empty.
#define __host__
#define __device__
#include "../../paper_2111_13652_amd/csrc/gsdf_fixed.hpp"

extern "C" unsigned long long fixed_term_host(float ws, float wh, float x) {
    return gsdf::fixed_term(ws, wh, x);
}

extern "C" float from_fixed_host(unsigned long long a, double inv) { return gsdf::from_fixed(a, inv); }
