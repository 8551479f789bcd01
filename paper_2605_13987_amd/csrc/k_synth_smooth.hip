// Register-FFT synthesis of H for the 2,3,5-smooth N_z that are not powers of
// two (the sizes synthesis_n1 lists): float path, two columns.  The kernel
// is the one of synth_pipe.hpp; this file only instantiates it, apart from
// k_bulk.hip so that the two compile in parallel.
#include "synth_pipe.hpp"

namespace wt {

namespace {

template <int NZ, typename TO>
hipError_t smooth_size(const Plan& p, char* b, void* h, hipStream_t s) {
    constexpr int N1 = synthesis_n1(NZ);
    static_assert(N1 > 0 && !synthesis_pow2(NZ), "smooth synthesis size");
    return synthesis_pipe<float, N1, NZ / N1, 2, TO>(p, b, h, s);
}

template <typename TO>
hipError_t smooth(const Plan& p, char* b, void* h, hipStream_t s) {
    switch (p.N[2]) {
        case 72: return smooth_size<72, TO>(p, b, h, s);
        case 80: return smooth_size<80, TO>(p, b, h, s);
        case 90: return smooth_size<90, TO>(p, b, h, s);
        case 96: return smooth_size<96, TO>(p, b, h, s);
        case 100: return smooth_size<100, TO>(p, b, h, s);
        case 108: return smooth_size<108, TO>(p, b, h, s);
        case 120: return smooth_size<120, TO>(p, b, h, s);
        case 144: return smooth_size<144, TO>(p, b, h, s);
        case 150: return smooth_size<150, TO>(p, b, h, s);
        case 160: return smooth_size<160, TO>(p, b, h, s);
        case 162: return smooth_size<162, TO>(p, b, h, s);
        case 180: return smooth_size<180, TO>(p, b, h, s);
        case 192: return smooth_size<192, TO>(p, b, h, s);
        case 200: return smooth_size<200, TO>(p, b, h, s);
        case 216: return smooth_size<216, TO>(p, b, h, s);
        case 240: return smooth_size<240, TO>(p, b, h, s);
        case 250: return smooth_size<250, TO>(p, b, h, s);
        case 270: return smooth_size<270, TO>(p, b, h, s);
        case 288: return smooth_size<288, TO>(p, b, h, s);
        case 300: return smooth_size<300, TO>(p, b, h, s);
        case 320: return smooth_size<320, TO>(p, b, h, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_synthesis_smooth(const Plan& p, char* b, void* h, hipStream_t s) {
    if (p.precision != 1 || p.n_cols != 2) return hipErrorInvalidValue;
    return p.h_format == 1 ? smooth<_Float16>(p, b, h, s) : smooth<float>(p, b, h, s);
}

}  // namespace wt
