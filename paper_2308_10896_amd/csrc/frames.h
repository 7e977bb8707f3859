// Light and viewer camera matrices, written once for any scalar type so the
// same code yields float64 values (forward) and their derivatives with
// respect to the light parameter (forward-mode duals, backward).
//
// The shadow map is parameterized by a projective camera map L of the light
// (Sec. 3).  Directional lights: orthographic camera far outside the scene
// facing the origin; spot (and point) lights: perspective camera at the light
// position (supplementary renderer details).  OpenGL conventions: right-handed
// view looking down -z, clip -> NDC in [-1,1]^3.
#pragma once

#include <math.h>

namespace dsm {

// Value plus three tangents (derivatives w.r.t. the 3 light parameters).
struct Dual3 {
    double v, d[3];
};

__host__ __device__ inline double val(double a) { return a; }
__host__ __device__ inline double val(const Dual3 &a) { return a.v; }

__host__ __device__ inline Dual3 operator+(const Dual3 &a, const Dual3 &b) {
    return Dual3{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}};
}
__host__ __device__ inline Dual3 operator-(const Dual3 &a, const Dual3 &b) {
    return Dual3{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}};
}
__host__ __device__ inline Dual3 operator-(const Dual3 &a) { return Dual3{-a.v, {-a.d[0], -a.d[1], -a.d[2]}}; }
__host__ __device__ inline Dual3 operator*(const Dual3 &a, const Dual3 &b) {
    return Dual3{a.v * b.v, {a.d[0] * b.v + a.v * b.d[0], a.d[1] * b.v + a.v * b.d[1], a.d[2] * b.v + a.v * b.d[2]}};
}
__host__ __device__ inline Dual3 operator*(double s, const Dual3 &b) {
    return Dual3{s * b.v, {s * b.d[0], s * b.d[1], s * b.d[2]}};
}
__host__ __device__ inline Dual3 operator/(const Dual3 &a, const Dual3 &b) {
    const double q = a.v / b.v;
    return Dual3{q, {(a.d[0] - q * b.d[0]) / b.v, (a.d[1] - q * b.d[1]) / b.v, (a.d[2] - q * b.d[2]) / b.v}};
}
__host__ __device__ inline Dual3 dsqrt(const Dual3 &a) {
    const double s = sqrt(a.v);
    const double h = 0.5 / s;
    return Dual3{s, {a.d[0] * h, a.d[1] * h, a.d[2] * h}};
}
__host__ __device__ inline double dsqrt(double a) { return sqrt(a); }

template <class T>
__host__ __device__ inline T mkT(double v);
template <>
__host__ __device__ inline double mkT<double>(double v) { return v; }
template <>
__host__ __device__ inline Dual3 mkT<Dual3>(double v) { return Dual3{v, {0, 0, 0}}; }

template <class T>
struct Vec3 {
    T x, y, z;
};

template <class T>
__host__ __device__ inline T dot3(const Vec3<T> &a, const Vec3<T> &b) {
    return (a.x * b.x + a.y * b.y) + a.z * b.z;
}
template <class T>
__host__ __device__ inline Vec3<T> cross3(const Vec3<T> &a, const Vec3<T> &b) {
    return Vec3<T>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T>
__host__ __device__ inline Vec3<T> sub3(const Vec3<T> &a, const Vec3<T> &b) {
    return Vec3<T>{a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class T>
__host__ __device__ inline Vec3<T> unit3(const Vec3<T> &a) {
    T n = dsqrt(dot3(a, a));
    return Vec3<T>{a.x / n, a.y / n, a.z / n};
}

// Static description of a camera (viewer or light), float64 on the host.
struct CamStatic {
    int kind;              // ViewKind
    double target[3], up[3];  // cube faces: target holds the face axis
    double focal;          // 1 / tan(fov/2), perspective
    double aspect;         // width / height
    double znear, zfar;
    double dir_distance;   // directional
    double ortho_half;     // directional
};

// view-projection P * lookAt(eye, target, up), row-major
template <class T>
__host__ __device__ inline void view_projection(const CamStatic &c, const Vec3<T> &eye, const Vec3<T> &target,
                                                T M[16]) {
    const Vec3<T> up{mkT<T>(c.up[0]), mkT<T>(c.up[1]), mkT<T>(c.up[2])};
    const Vec3<T> f = unit3(sub3(target, eye));
    const Vec3<T> s = unit3(cross3(f, up));
    const Vec3<T> u = cross3(s, f);
    const T zero = mkT<T>(0.0), one = mkT<T>(1.0);
    // V rows: [s, -s.eye], [u, -u.eye], [-f, f.eye], [0,0,0,1]
    const T V[16] = {s.x, s.y, s.z, -dot3(s, eye),
                     u.x, u.y, u.z, -dot3(u, eye),
                     -f.x, -f.y, -f.z, dot3(f, eye),
                     zero, zero, zero, one};
    double P[16] = {0};
    const double n = c.znear, fa = c.zfar;
    if (c.kind == 0) {            // orthographic (directional light)
        P[0] = 1.0 / c.ortho_half;
        P[5] = 1.0 / c.ortho_half;
        P[10] = -2.0 / (fa - n);
        P[11] = -(fa + n) / (fa - n);
        P[15] = 1.0;
    } else {
        P[0] = c.focal / c.aspect;
        P[5] = c.focal;
        P[10] = (fa + n) / (n - fa);
        P[11] = 2.0 * fa * n / (n - fa);
        P[14] = -1.0;
    }
    for (int r = 0; r < 4; ++r)
        for (int col = 0; col < 4; ++col) {
            T acc = zero;
            for (int k = 0; k < 4; ++k)
                if (P[r * 4 + k] != 0.0) acc = acc + P[r * 4 + k] * V[k * 4 + col];
            M[r * 4 + col] = acc;
        }
}

// Light frame from the differentiable parameter p (position, or travel
// direction for directional lights): M, pos (position or eye), dir (unit
// travel direction, or cone axis).
template <class T>
__host__ __device__ inline void light_frame(const CamStatic &c, const T p[3], T M[16], T pos[3], T dir[3]) {
    Vec3<T> P3{p[0], p[1], p[2]};
    if (c.kind == 0) {
        const Vec3<T> w = unit3(P3);
        const Vec3<T> eye{-c.dir_distance * w.x, -c.dir_distance * w.y, -c.dir_distance * w.z};
        const Vec3<T> org{mkT<T>(0.0), mkT<T>(0.0), mkT<T>(0.0)};
        view_projection(c, eye, org, M);
        pos[0] = eye.x; pos[1] = eye.y; pos[2] = eye.z;
        dir[0] = w.x; dir[1] = w.y; dir[2] = w.z;
    } else {
        // cube faces keep their viewing axis in `target`: the camera looks
        // from the position along that fixed axis
        const Vec3<T> tg = c.kind == 4
            ? Vec3<T>{P3.x + mkT<T>(c.target[0]), P3.y + mkT<T>(c.target[1]), P3.z + mkT<T>(c.target[2])}
            : Vec3<T>{mkT<T>(c.target[0]), mkT<T>(c.target[1]), mkT<T>(c.target[2])};
        view_projection(c, P3, tg, M);
        const Vec3<T> ax = unit3(sub3(tg, P3));
        pos[0] = P3.x; pos[1] = P3.y; pos[2] = P3.z;
        dir[0] = ax.x; dir[1] = ax.y; dir[2] = ax.z;
    }
}

// Reference depth of a light's maps (normalized by zfar): the depth of the
// point its camera looks at (directional: the origin at dir_distance; point
// and spot lights: the target).  The maps store moments of z - zc instead of
// z: the variance m2 - m1^2 and every difference d - mu are unchanged, but
// the stored values are small where the scene lies near the reference, so
// float32 keeps more of the digits that m2 - m1^2 cancels.  Cube faces keep
// zc = 0: their seam padding mixes the six faces' maps, which must share one
// reference, and no single depth fits every direction.
template <class T>
__host__ __device__ inline double light_reference_depth(const CamStatic &c, const T p[3]) {
    if (c.kind == 0) return c.dir_distance / c.zfar;
    if (c.kind == 4) return 0.0;
    const double dx = c.target[0] - (double)p[0], dy = c.target[1] - (double)p[1], dz = c.target[2] - (double)p[2];
    return sqrt(dx * dx + dy * dy + dz * dz) / c.zfar;
}

}  // namespace dsm
