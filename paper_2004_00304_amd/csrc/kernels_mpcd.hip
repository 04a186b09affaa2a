// kernels_mpcd.hip -- instantiations of the particle kernel (particles.hpp)
// for the Maxwell-Boltzmann exchange: collide (1), stream (2), both (3), and
// the MPCD-AT variants (5, 7); the dispatch of every mode.
#include <cmath>

#include "particles.hpp"

namespace lbmpcd {

size_t particle_lds_bytes(int, int, int) { return LDS_HDR + LDS_WIN + LDS_COLL; }

namespace {
struct PlainModes {
    template <int DIM, typename PT, int NT, int PPT>
    static hipError_t run(const ParticleLaunch& L, hipStream_t s) {
        switch (L.mode) {
            case 1: return launch_p4<DIM, PT, NT, PPT, 1>(L, s);
            case 2: return launch_p4<DIM, PT, NT, PPT, 2>(L, s);
            case 3: return launch_p4<DIM, PT, NT, PPT, 3>(L, s);
            case 5: return launch_p4<DIM, PT, NT, PPT, 5>(L, s);
            case 7: return launch_p4<DIM, PT, NT, PPT, 7>(L, s);
            default: return hipErrorInvalidValue;
        }
    }
};
}  // namespace

// Binary32 particles with SRD, in tiles of 1025-2048 slots at 256 threads:
// six slots per thread instead of eight take the kernel from 114 to 96
// vector registers, five waves per SIMD instead of four.  A tile holding more
// than 1536 particles (the tile's expected occupancy plus two standard
// deviations of its Poisson count must stay below that, so it is rare) is
// skipped and listed by that launch and processed by a second, eight-slot
// launch over the list.
template <int DIM, int MODE>
static hipError_t launch_split(const ParticleLaunch& L, hipStream_t s) {
    hipError_t e = launch_p4<DIM, float, 256, 6, MODE, 1>(L, s);
    if (e == hipSuccess) e = launch_p4<DIM, float, 256, 8, MODE, 2>(L, s);
    return e;
}

template <int DIM>
static hipError_t launch_split_mode(const ParticleLaunch& L, hipStream_t s) {
    switch (L.mode) {
        case 1: return launch_split<DIM, 1>(L, s);
        case 2: return launch_split<DIM, 2>(L, s);
        case 3: return launch_split<DIM, 3>(L, s);
        case 5: return launch_split<DIM, 5>(L, s);
        case 7: return launch_split<DIM, 7>(L, s);
        default: return hipErrorInvalidValue;
    }
}

static bool split_applies(const ParticleLaunch& L) {
    if (L.part_fp != 32 || L.ovf == nullptr || (L.mode != 1 && L.mode != 2 && L.mode != 3 && L.mode != 5 && L.mode != 7)) return false;
    if ((L.wg_threads != 0 && L.wg_threads != 256) || L.cap_max <= 4 * 256 || L.cap_max > 8 * 256) return false;
    const double e = (double)L.exp_max;
    return e + 2.0 * std::sqrt(e) <= 6.0 * 256;
}

hipError_t launch_particles(const ParticleLaunch& L, hipStream_t s) {
    if (L.mode & 16) return launch_particles_det(L, s);
    if (L.mode & 8) return launch_particles_ce(L, s);
    if (L.tiles > 0 && split_applies(L))
        return L.dim == 2 ? launch_split_mode<2>(L, s) : launch_split_mode<3>(L, s);
    return launch_modes<PlainModes>(L, s);
}

}  // namespace lbmpcd
