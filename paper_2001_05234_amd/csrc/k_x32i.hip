// k_x32i.hip -- launcher of the inverse FP32 x transform (and the refinement update)
// of the refinement path (FFT and dense matrix-core forms).
#include "xform_kernels.h"

namespace cans {

int launch_x_inv_32(const Problem &pb, const Work &w, const float *in, double *p, bool update, const int *done,
                    hipStream_t s)
{
    if (pb.ax.dense) {
        if (update)
            hipLaunchKernelGGL((k_dense_x<false, float, double, 1>), dense_grid(pb), dim3(256), dense_lds(pb.nx), s,
                               in, p, (long)pb.ny * pb.nz, pb.nx, mag_of(pb.nx), pb.ax.d_wi_hi, pb.ax.d_wi_lo,
                               w.info, done, nullptr, pb.ny, nullptr);
        else
            hipLaunchKernelGGL((k_dense_x<false, float, double, 0>), dense_grid(pb), dim3(256), dense_lds(pb.nx), s,
                               in, p, (long)pb.ny * pb.nz, pb.nx, mag_of(pb.nx), pb.ax.d_wi_hi, pb.ax.d_wi_lo,
                               w.info, done, nullptr, pb.ny, nullptr);
        return check_launch();
    }
    const XGeom &g = pb.ax.gx32[0];
    const long nlines = (long)pb.ny * pb.nz;
    const dim3 grid((unsigned)((nlines + g.L - 1) / g.L));
    const size_t sh = tile_lds(AX_X, g, sizeof(float));
    CANS_KIND_SWITCH(pb.ax.kind,
        if (update) hipLaunchKernelGGL((k_xform_x<KD, false, float, float, double, 1>), grid, dim3(kThreads), sh, s,
                                       in, p, nlines, g, pb.ax.d_tw32, w.info, done, nullptr, pb.ny, nullptr);
        else hipLaunchKernelGGL((k_xform_x<KD, false, float, float, double, 0>), grid, dim3(kThreads), sh, s,
                                in, p, nlines, g, pb.ax.d_tw32, w.info, done, nullptr, pb.ny, nullptr));
    return check_launch();
}


int launch_x_inv_32_grp(const GroupLaunch &gl, bool update, hipStream_t s)
{
    const XJob *j = static_cast<const XJob *>(gl.jobs);
    CANS_KIND_SWITCH(gl.key,
        if (update) hipLaunchKernelGGL((k_xform_x_grp<KD, false, float, float, double, 1>), dim3(gl.blocks),
                                       dim3(kThreads), gl.lds, s, j, gl.start, gl.np);
        else hipLaunchKernelGGL((k_xform_x_grp<KD, false, float, float, double, 0>), dim3(gl.blocks),
                                dim3(kThreads), gl.lds, s, j, gl.start, gl.np));
    return check_launch();
}

}  // namespace cans
