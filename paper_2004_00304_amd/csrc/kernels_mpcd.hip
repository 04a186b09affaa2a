// kernels_mpcd.hip -- instantiations of the particle kernel (particles.hpp)
// for the Maxwell-Boltzmann exchange: collide (1), stream (2), both (3), and
// the MPCD-AT variants (5, 7); the dispatch of every mode.
#include "particles.hpp"

namespace lbmpcd {

size_t particle_lds_bytes(int, int, int) { return LDS_HDR + LDS_WIN + LDS_COLL; }

namespace {
struct PlainModes {
    template <int DIM, typename PT, int NT, int PPT, int OVF = 0>
    static hipError_t run(const ParticleLaunch& L, hipStream_t s) {
        switch (L.mode) {
            case 1: return launch_p4<DIM, PT, NT, PPT, 1, OVF>(L, s);
            case 2: return launch_p4<DIM, PT, NT, PPT, 2, OVF>(L, s);
            case 3: return launch_p4<DIM, PT, NT, PPT, 3, OVF>(L, s);
            case 5: return launch_p4<DIM, PT, NT, PPT, 5, OVF>(L, s);
            case 7: return launch_p4<DIM, PT, NT, PPT, 7, OVF>(L, s);
            default: return hipErrorInvalidValue;
        }
    }
};
}  // namespace

hipError_t launch_particles(const ParticleLaunch& L, hipStream_t s) {
    if (L.mode & 16) return launch_particles_det(L, s);
    if (L.mode & 8) return launch_particles_ce(L, s);
    return launch_modes<PlainModes>(L, s);
}

}  // namespace lbmpcd
