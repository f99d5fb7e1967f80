// k_x32f.hip -- launcher of the forward FP32 x transform of the refinement path
// (FFT and dense matrix-core forms).
#include "xform_kernels.h"

namespace cans {

int launch_x_fwd_32(const Problem &pb, const Work &w, const double *in, float *out, const int *done, hipStream_t s)
{
    if (pb.ax.dense) {
        hipLaunchKernelGGL((k_dense_x<true, double, float, 0>), dense_grid(pb), dim3(256), dense_lds(pb.nx), s, in, out,
                           (long)pb.ny * pb.nz, pb.nx, mag_of(pb.nx), pb.ax.d_wf_hi, pb.ax.d_wf_lo, nullptr, done,
                           pb.d_dzf, pb.ny, w.partials);
        return check_launch();
    }
    const XGeom &g = pb.ax.gx32[1];
    const long nlines = (long)pb.ny * pb.nz;
    const dim3 grid((unsigned)xfwd_blocks(pb));
    const size_t sh = tile_lds(AX_X, g, sizeof(float));
    CANS_KIND_SWITCH(pb.ax.kind,
        hipLaunchKernelGGL((k_xform_x<KD, true, float, double, float, 0>), grid, dim3(kThreads), sh, s,
                           in, out, nlines, g, pb.ax.d_tw32, nullptr, done, pb.d_dzf, pb.ny, w.partials));
    return check_launch();
}


int launch_x_fwd_32_grp(const GroupLaunch &gl, hipStream_t s)
{
    const XJob *j = static_cast<const XJob *>(gl.jobs);
    CANS_KIND_SWITCH(gl.key,
        hipLaunchKernelGGL((k_xform_x_grp<KD, true, float, double, float, 0>), dim3(gl.blocks), dim3(kThreads),
                           gl.lds, s, j, gl.start, gl.np));
    return check_launch();
}

}  // namespace cans
