// Register-FFT synthesis of H for the 2,3,5-smooth N_z that are not powers of
// two: float path, two columns, one instantiation per schedule of
// kSmoothSchedules (the plan's synth_n1 and synth_tbc pick one).  The kernel
// is the one of synth_pipe.hpp; this file only instantiates it, apart from
// k_bulk.hip so that the two compile in parallel.
#include "synth_pipe.hpp"

namespace wt {

namespace {

template <int I, typename TO>
hipError_t smooth(const Plan& p, char* b, void* h, hipStream_t s) {
    if constexpr (I == kNumSmoothSchedules) {
        return hipErrorInvalidValue;
    } else {
        constexpr PipeSchedule c = kSmoothSchedules[I];
        static_assert(!synthesis_pow2(c.nz) && pipe_fits(pipe_shape_for(c.nz, c.n1, c.tbc), 4), "smooth schedule");
        if (p.N[2] == c.nz && p.synth_n1 == c.n1 && p.synth_tbc == c.tbc)
            return synthesis_pipe<float, c.n1, c.nz / c.n1, 2, TO, c.tbc>(p, b, h, s);
        return smooth<I + 1, TO>(p, b, h, s);
    }
}

}  // namespace

hipError_t launch_synthesis_smooth(const Plan& p, char* b, void* h, hipStream_t s) {
    if (p.precision != 1 || p.n_cols != 2) return hipErrorInvalidValue;
    return p.h_format == 1 ? smooth<0, _Float16>(p, b, h, s) : smooth<0, float>(p, b, h, s);
}

}  // namespace wt
