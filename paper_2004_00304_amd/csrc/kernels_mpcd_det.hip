// kernels_mpcd_det.hip -- instantiations of the particle kernel (particles.hpp)
// in the deterministic mode (bit 16): the sums of the collision, the MPCD-AT
// thermostat and the sample windows are fixed-point integer atomics, so a run
// does not depend on the order in which atomics land.  Collide (17), stream
// (18), both (19), and the MPCD-AT variants (21, 23); the Maxwell-Boltzmann
// exchange only.  A translation unit of its own so that it compiles beside
// the others.
#include "particles.hpp"

namespace lbmpcd {

namespace {
struct DetModes {
    template <int DIM, typename PT, int NT, int PPT, int OVF = 0>
    static hipError_t run(const ParticleLaunch& L, hipStream_t s) {
        switch (L.mode) {
            case 17: return launch_p4<DIM, PT, NT, PPT, 17, OVF>(L, s);
            case 18: return launch_p4<DIM, PT, NT, PPT, 18, OVF>(L, s);
            case 19: return launch_p4<DIM, PT, NT, PPT, 19, OVF>(L, s);
            case 21: return launch_p4<DIM, PT, NT, PPT, 21, OVF>(L, s);
            case 23: return launch_p4<DIM, PT, NT, PPT, 23, OVF>(L, s);
            default: return hipErrorInvalidValue;
        }
    }
};
}  // namespace

hipError_t launch_particles_det(const ParticleLaunch& L, hipStream_t s) { return launch_modes<DetModes>(L, s); }

}  // namespace lbmpcd
