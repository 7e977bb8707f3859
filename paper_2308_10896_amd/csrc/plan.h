// The plan: host copy of a batch description, device-resident mesh-static
// data, and the byte layout of the caller's saved / scratch buffers.
#pragma once

#include <vector>

#include "dsm_internal.h"
#include "frames.h"

struct dsm_plan {
    // batch shape
    int device = -1;   // HIP device current at creation; the plan's device data live there
    int B = 0, L = 0, Cm = 0, R = 0, C = 1, nviews = 0;
    int camera_antialias = 1;
    long long V_total = 0, F_total = 0;
    int tile = 16;
    int bin_scale = 8;
    unsigned capacity = 0;
    int ntri = 0, ntiles = 0, nclip = 0;
    int max_verts = 0, max_faces = 0, max_light_texels = 0, max_cam_pix = 0;
    long long key_count = 0, map_floats = 0, image_floats = 0;
    int blur_tiles = 0, blur_rmax = 0, max_pose_verts = 0;
    int max_light_tiles = 0, max_cam_tiles = 0, max_lights_per_render = 0;
    int max_scene_verts = 0, max_scene_faces = 0;

    std::vector<dsm::ViewConst> views_h;
    std::vector<dsm::CamStatic> light_cams_h;
    std::vector<dsm::RenderConst> renders_h;
    std::vector<int> render_lights_h;
    std::vector<int> vert_off, face_off, pose_counts;
    std::vector<float> pose_centers;
    std::vector<dsm::BlurJob> blur_jobs_h;   // sorted by filter radius; [0, L): forward, [L, 2L): transpose
    bool has_cube = false;
    int max_cube_padded = 0, max_cube_texels = 0, max_cube_ring = 0;
    std::vector<dsm::CubeTap> cube_taps_h;
    struct BlurGroup {
        int R, first, n, tiles;
    };
    std::vector<BlurGroup> blur_groups;

    // plan-owned device data
    dsm::ViewConst *views_d = nullptr;
    dsm::CamStatic *light_cams_d = nullptr;
    dsm::RenderConst *renders_d = nullptr;
    int *render_lights_d = nullptr;
    int *faces_d = nullptr;
    int *adj_d = nullptr;
    int *tile_view_d = nullptr;
    dsm::BlurJob *blur_jobs_d = nullptr;
    dsm::CubeTap *cube_taps_d = nullptr;
    int *scene_vert_off_d = nullptr;    // [B+1]
    int *pose_counts_d = nullptr;       // [B]
    float *pose_centers_d = nullptr;    // [B,3]
    int *cam_renders_off_d = nullptr;   // [Cm+1] renders of each camera view
    int *cam_renders_d = nullptr;
    int *scene_views_off_d = nullptr;   // [B+1] views of each scene
    int *scene_views_d = nullptr;
    int *vc_off_d = nullptr;            // [V+1] triangle corners of each vertex
    int *vc_list_d = nullptr;           // (scene-local face << 2) | corner
    int *light_renders_off_d = nullptr; // [L+1] (render << 5 | slot) using each light
    int *light_renders_d = nullptr;
    int *scene_face_off_d = nullptr;    // [B+1]

    // layout of the caller's saved buffer (byte offsets): everything the
    // forward writes and the backward reads, the binning state included
    size_t sv_counters = 0, sv_zero_end = 0, sv_keys = 0, sv_clip = 0, sv_setup = 0, sv_sil = 0, sv_tv = 0, sv_F0 = 0,
           sv_M = 0, sv_img0 = 0, sv_pair_off = 0, sv_tile_start = 0, sv_bins = 0, sv_bin_pair = 0, sv_overflow = 0, sv_zc = 0, sv_aa_flag = 0,
           saved_bytes = 0;
    // layout of the caller's scratch buffer (byte offsets): temporaries of
    // one call, nothing carried from a forward to its backward
    size_t sc_pair_cnt = 0, sc_scan = 0, sc_tile_cnt = 0, sc_facing = 0, sc_big_bin = 0,
           sc_pair_slot = 0, sc_aa_list = 0, sc_aa_count = 0, sc_pair_flag = 0, sc_F1 = 0, sc_fwd_end = 0, sc_gimg0 = 0, sc_gM = 0, sc_gF1 = 0,
           sc_gclip = 0, sc_glight = 0, sc_zero_fwd_end = 0, sc_bigcount = 0, sc_zero_rec = 0, sc_zero_bwd_end = 0,
           sc_pair_sums = 0, sc_gtri = 0, sc_biglist = 0, sc_part_light = 0, sc_part_gm = 0, sc_part_render = 0, sc_jac = 0,
           scratch_bytes = 0;

    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};

namespace dsm {
// The forward pass with a scratch buffer that need only hold the forward's
// temporaries (plan->sc_fwd_end bytes): validates its arguments as
// dsm_forward does and enqueues the same kernels on `stream`.
dsm_status forward_in_scratch(dsm_plan *p, const float *verts, const float *lparams, const float *albedo, void *saved,
                              size_t saved_bytes, void *scratch, size_t scratch_bytes, float *images,
                              hipStream_t stream);
}  // namespace dsm
