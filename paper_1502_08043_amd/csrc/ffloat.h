// Float-float ("split FP32") arithmetic for the mixed-precision node sums.
//
// A value is carried as an unevaluated sum hi + lo of two floats.  Products use
// the exact FMA remainder of the hi parts (TwoProduct) plus the cross terms;
// the lo*lo term (relative size 2^-48) is dropped.  Sums use Knuth's
// branch-free TwoSum on the hi parts and gather every rounding error and lo
// part in a second float.  The library is built with -ffp-contract=off, so
// the compiler never fuses the products these identities rely on.
#pragma once

#include <hip/hip_runtime.h>

namespace pwc {

struct ff {
    float h, l;
};

__device__ __forceinline__ ff ff_mul(ff a, ff b) {
    const float p = a.h * b.h;
    float e = fmaf(a.h, b.h, -p);          // exact: a.h * b.h = p + e
    e = fmaf(a.h, b.l, fmaf(a.l, b.h, e));
    return ff{p, e};
}

// (sh, sl) += t, with sh updated by TwoSum and sl collecting the error terms.
__device__ __forceinline__ void ff_acc(float &sh, float &sl, ff t) {
    const float s = sh + t.h;
    const float bb = s - sh;
    const float err = (sh - (s - bb)) + (t.h - bb);
    sh = s;
    sl += err + t.l;
}

__device__ __forceinline__ double ff_to_double(float h, float l) {
    return static_cast<double>(h) + static_cast<double>(l);
}

}  // namespace pwc
