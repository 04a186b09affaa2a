// kernels_mpcd_ce.hip -- instantiations of the particle kernel (particles.hpp)
// with the Chapman-Enskog exchange (mode bit 8): stream (10), stream and
// collide (11), and with the MPCD-AT collision (15).  A translation unit of
// its own so that it compiles beside the Maxwell-Boltzmann set.
//
// Register budget: the exchange's acceptance test keeps the cell's tensor and
// one more Philox block live per particle, so these modes are built for three
// waves per SIMD (particle_waves in particles.hpp).
#include "particles.hpp"

namespace lbmpcd {

namespace {
struct CEModes {
    template <int DIM, typename PT, int NT, int PPT, int OVF = 0>
    static hipError_t run(const ParticleLaunch& L, hipStream_t s) {
        switch (L.mode) {
            case 10: return launch_p4<DIM, PT, NT, PPT, 10, OVF>(L, s);
            case 11: return launch_p4<DIM, PT, NT, PPT, 11, OVF>(L, s);
            case 15: return launch_p4<DIM, PT, NT, PPT, 15, OVF>(L, s);
            default: return hipErrorInvalidValue;
        }
    }
};
}  // namespace

hipError_t launch_particles_ce(const ParticleLaunch& L, hipStream_t s) {
    if (L.tfine == nullptr) return hipErrorInvalidValue;
    return launch_modes<CEModes>(L, s);
}

}  // namespace lbmpcd
