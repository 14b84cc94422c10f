// CPU oracle for the dynamic coherence-based EM ray tracer (Wang & Manocha,
// "Dynamic Coherence-Based EM Ray Tracing Simulations in Vehicular
// Environments").
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
// reference that the GPU library is checked against.  Only the test-suite, the
// smoke check and the benchmark's CPU-baseline leg may load it; the library
// never calls it, and the two share no source, header or helper.
//
// Everything is FP64 and brute force: every ray segment is tested against every
// triangle, every path is validated against every triangle.  No BVH, no
// blocking, no reordering.  Inputs are the same FP32 arrays the library gets,
// widened exactly to FP64.
//
// The steps follow the paper's description of a frame (Sec. III, "Backward ray
// tracing" list and the "Reflected and transmitted rays" item), with the
// forward direction (shoot from the transmitter, capture at receiver spheres)
// and the readings listed in the design notes:
//   1. a sphere of rays leaves the transmitter                    (step 1)
//   2. each ray is bounced specularly, recording the sequence of
//      reflecting faces, up to K reflections                      (step 2; <= 10)
//   3. a ray segment passing within the capture radius of a
//      receiver yields a candidate (tx, rx, order, face sequence)
//   4. candidates are de-duplicated (the per-depth "visited path"
//      tables) and each is refined by the image method: image
//      sources through the face planes, reflection points, and a
//      validity check (points inside faces, segments unoccluded)  (steps 3, 4)
//   5. each valid path gets its length, directions, Fresnel-
//      weighted polarised amplitude and phase                     (step 6)
//   6. per receiver, amplitudes are summed; received power is the
//      squared norm of the sum (phase-coherent)                   (phase calc.)
// The direct path's magnitude is the close-in model of Eq. (3) with path-loss
// exponent 2 (free space): P = Pt (lambda / (4 pi d))^2.
//
// Parity is pinned (closed forms, invariants, brute-force enumeration) by the
// `-m "not gpu"` tests; see the test files for each pin.
//
// Uncertainty bookkeeping.  The GPU traces in FP32.  For every ray segment the
// oracle also reports whether an FP32 tracer could legitimately decide
// differently: a hit within eps of a face silhouette, a near miss of another
// face before the hit, two faces hit at (nearly) the same distance, a hit near
// t_min, a capture distance within eps of the radius.  eps grows with the
// scene radius, the path length and the bounce index.  Those decisions are
// excluded from bit-exact comparison.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

namespace {

using cplx = std::complex<double>;

struct V3 {
    double x = 0, y = 0, z = 0;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 unit(V3 a) { return (1.0 / norm(a)) * a; }

struct CV3 {
    cplx x, y, z;
};
inline cplx cdot(CV3 e, V3 a) { return e.x * a.x + e.y * a.y + e.z * a.z; }
inline CV3 cscale(cplx s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline CV3 cadd(CV3 a, CV3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }

const double kC0 = 299792458.0;             // speed of light [m/s]
const double kEps0 = 8.8541878128e-12;      // vacuum permittivity [F/m]
const double kPi = 3.14159265358979323846;

struct Tri {
    V3 a, b, c;
    int face;
    double h0, h1, h2;   // altitudes from a, b, c to the opposite edge
};

struct Face {
    V3 n;                 // unit normal
    V3 p;                 // a point on the plane
    int material;
    int object;
    std::vector<int> tris;
    std::vector<std::pair<V3, V3>> silhouette;  // boundary edges of the face
};

struct Material {
    double eps_r, sigma, const_gamma;
    // penetration loss of a transmission through a face of this material, dB
    // (Table II); +inf: the material is opaque
    double pen_db = std::numeric_limits<double>::infinity();
};

struct Scene {
    std::vector<Tri> tris;
    std::vector<Face> faces;
    std::vector<Material> mats;
    double radius = 0;    // bounding radius about the origin (vertices)
};

// Rigid object transform x' = R x + t evaluated in FP64 and rounded to FP32.
// Each product of two FP32 numbers is exact in FP64, so left-to-right summation
// defines the result uniquely.
inline float xform_row(const float* row, float x, float y, float z) {
    double r = (double)row[0] * (double)x;
    r = r + (double)row[1] * (double)y;
    r = r + (double)row[2] * (double)z;
    r = r + (double)row[3];
    return (float)r;
}

// Moller-Trumbore in FP64.  Returns false for a ray parallel to the plane.
// Outputs the parametric distance t and barycentrics (w, u, v) for (a, b, c).
inline bool ray_plane_bary(const Tri& tr, V3 o, V3 d, double& t, double& w, double& u, double& v) {
    V3 e1 = tr.b - tr.a, e2 = tr.c - tr.a;
    V3 p = cross(d, e2);
    double det = dot(e1, p);
    if (det == 0.0) return false;
    double inv = 1.0 / det;
    V3 s = o - tr.a;
    u = dot(s, p) * inv;
    V3 q = cross(s, e1);
    v = dot(d, q) * inv;
    t = dot(e2, q) * inv;
    w = 1.0 - u - v;
    return true;
}

// Signed in-plane distance of the crossing point to the triangle's edge lines:
// positive inside, the distance to the nearest edge; negative outside.
inline double tri_margin(const Tri& tr, double w, double u, double v) {
    return std::min(w * tr.h0, std::min(u * tr.h1, v * tr.h2));
}

inline double point_segment_dist(V3 p, V3 a, V3 b) {
    V3 ab = b - a;
    double l2 = dot(ab, ab);
    double s = l2 > 0 ? dot(p - a, ab) / l2 : 0.0;
    s = std::max(0.0, std::min(1.0, s));
    return norm(p - (a + s * ab));
}

inline double silhouette_dist(const Face& f, V3 p) {
    double best = std::numeric_limits<double>::infinity();
    for (auto& e : f.silhouette) best = std::min(best, point_segment_dist(p, e.first, e.second));
    return best;
}

// Fresnel reflection coefficients for a plane interface, e^{+j w t} convention
// (the field phase factor of Eq. (1) is e^{-j beta0 S}), relative complex
// permittivity eps_c = eps_r - j sigma / (w eps0).  TE: E perpendicular to the
// plane of incidence; TM: E in it.  A non-NaN const_gamma g replaces both by a
// polarisation-independent mirror of magnitude g (Table II's scalar
// "reflection coefficient"): Gamma_TE = -g, Gamma_TM = +g.
inline void fresnel(const Material& m, double freq, double cos_t, cplx& g_te, cplx& g_tm) {
    if (!std::isnan(m.const_gamma)) {
        g_te = cplx(-m.const_gamma, 0.0);
        g_tm = cplx(m.const_gamma, 0.0);
        return;
    }
    cplx eps_c(m.eps_r, -m.sigma / (2.0 * kPi * freq * kEps0));
    double sin2 = 1.0 - cos_t * cos_t;
    cplx root = std::sqrt(eps_c - sin2);   // principal branch
    g_te = (cos_t - root) / (cos_t + root);
    g_tm = (eps_c * cos_t - root) / (eps_c * cos_t + root);
}

// Derivatives of the Fresnel coefficients above with respect to the complex
// relative permittivity eps_c (both are analytic in eps_c).  With
// r = sqrt(eps_c - sin^2) and c = cos(theta), dr/deps_c = 1 / (2 r):
//   d Gamma_TE / d eps_c = -c / (r (c + r)^2),
//   d Gamma_TM / d eps_c = 2 c (r - eps_c / (2 r)) / (eps_c c + r)^2.
// A constant-gamma material does not depend on (eps_r, sigma): zero.
inline void fresnel_deps(const Material& m, double freq, double cos_t, cplx& d_te, cplx& d_tm) {
    if (!std::isnan(m.const_gamma)) {
        d_te = d_tm = cplx(0.0, 0.0);
        return;
    }
    cplx eps_c(m.eps_r, -m.sigma / (2.0 * kPi * freq * kEps0));
    double sin2 = 1.0 - cos_t * cos_t;
    cplx r = std::sqrt(eps_c - sin2);
    cplx ctr = cos_t + r;
    d_te = -cos_t / (r * ctr * ctr);
    cplx den = eps_c * cos_t + r;
    d_tm = 2.0 * cos_t * (r - eps_c / (2.0 * r)) / (den * den);
}

// Flags per traced segment.
enum : int32_t {
    SEG_TIE = 1,    // another face is hit within the tie tolerance: the rest of the ray is uncertain
    SEG_EDGE = 2,   // an FP32 tracer could hit a different face (or none): the rest is uncertain
    SEG_TRI = 4,    // only the triangle id within the hit face is uncertain
};
// Flags per capture.
enum : int32_t {
    CAP_HIT = 1,        // captured in exact arithmetic (distance <= r)
    CAP_MARGINAL = 2,   // |distance - r| <= eps
    CAP_UNCERTAIN = 4,  // the segment (or an earlier one) carries SEG_TIE / SEG_EDGE
};

struct Capture {
    int64_t ray;
    int32_t tx, rx, order, flags;
    std::vector<int32_t> faces;
};

struct TraceArgs {
    const Scene* sc;
    const float* tx;
    int32_t ntx;
    const float* rx;
    int32_t nrx;
    double r;
    const float* dirs;
    const int64_t* ray_ids;
    int64_t nsel;
    int32_t K;          // interactions at most (segments 0..K)
    int32_t max_refl;   // reflections at most
    // branch b of a ray transmits at the interactions in sets[b] (bit j:
    // interaction j) and reflects at the others
    const uint32_t* sets;
    int32_t n_branch;
    int64_t n_dirs;     // rays in `dirs` (capture rows name ray b * n_dirs + id)
    double t_min;
    double eps_rel;
    double radius;   // bounding radius of geometry, transmitters and receivers
    int32_t* out_tri;
    int32_t* out_face;
    double* out_t;
    double* out_len;
    int32_t* out_flags;
};

// Trace one branch of one ray from one source; per segment write the closest
// hit and the uncertainty flags, and append captures.  The branch goes
// straight on through the faces of the interactions in its set (a penetrable
// face; it ends at an opaque one) and reflects at the others (it ends where
// it would reflect a (max_refl + 1)-th time).  Its segments up to its last
// transmission are those of the branch without that transmission, so it
// reports captures only after it.
void trace_one(const TraceArgs& A, int32_t txi, int32_t b, int64_t sel, std::vector<Capture>& caps) {
    const Scene& sc = *A.sc;
    const int64_t rid = A.ray_ids ? A.ray_ids[sel] : sel;
    const int K = A.K;
    const uint32_t tset = A.sets[b];
    int last_t = -1;
    for (int j = 0; j < 32; ++j)
        if ((tset >> j) & 1u) last_t = j;
    const int64_t slot = (((int64_t)txi * A.n_branch + b) * A.nsel + sel) * (K + 1);
    for (int k = 0; k <= K; ++k) {
        A.out_tri[slot + k] = -2;   // not traced
        A.out_face[slot + k] = -1;
        A.out_t[slot + k] = std::numeric_limits<double>::infinity();
        A.out_len[slot + k] = 0.0;
        A.out_flags[slot + k] = 0;
    }
    V3 o{A.tx[3 * txi], A.tx[3 * txi + 1], A.tx[3 * txi + 2]};
    V3 d{A.dirs[3 * rid], A.dirs[3 * rid + 1], A.dirs[3 * rid + 2]};
    const double dlen = norm(d);
    int excl = -1;
    double L = 0.0;
    bool uncertain = false;
    std::vector<int32_t> seq;
    for (int k = 0; k <= K; ++k) {
        // --- closest hit: lexicographic min of (t, triangle id) over all triangles
        //     of other faces than the one just left, with t > t_min
        int best = -1;
        double tb = std::numeric_limits<double>::infinity(), wb = 0, ub = 0, vb = 0;
        const int nt = (int)sc.tris.size();
        for (int i = 0; i < nt; ++i) {
            const Tri& tr = sc.tris[i];
            if (tr.face == excl) continue;
            double t, w, u, v;
            if (!ray_plane_bary(tr, o, d, t, w, u, v)) continue;
            if (!(t > A.t_min)) continue;
            if (w < 0 || u < 0 || v < 0) continue;
            if (t < tb) { tb = t; best = i; wb = w; ub = u; vb = v; }
        }
        const int bface = best >= 0 ? sc.tris[best].face : -1;
        // --- uncertainty of this decision for an FP32 tracer
        int32_t flags = 0;
        const double tie_tol = best >= 0 ? std::max(1e-6 * tb, 0.0) : 0.0;
        for (int i = 0; i < nt; ++i) {
            const Tri& tr = sc.tris[i];
            if (tr.face == excl) continue;
            double t, w, u, v;
            if (!ray_plane_bary(tr, o, d, t, w, u, v)) continue;
            const double eps = A.eps_rel * (k + 1) * (A.radius + L + std::fabs(t) * dlen);
            const double m = tri_margin(tr, w, u, v);
            if (m < -eps) continue;                      // robustly missed
            if (t * dlen < A.t_min * dlen - eps) continue;
            if (std::fabs((t - A.t_min) * dlen) <= eps) { flags |= SEG_EDGE; continue; }
            if (!(t > A.t_min)) continue;
            if (i == best) continue;
            if (best >= 0 && tr.face == bface) {
                if (std::fabs(t - tb) * dlen <= eps) flags |= SEG_TRI;
                continue;
            }
            if (m >= 0) {
                // a hit on another face: a tie if it is (nearly) as close as the best
                if (best >= 0 && (t - tb) * dlen <= std::max(tie_tol * dlen, eps)) flags |= SEG_TIE;
            } else {
                // a near miss: matters if it lies before (or at) the closest hit
                if (best < 0 || (t - tb) * dlen <= eps) flags |= SEG_EDGE;
            }
        }
        V3 hit = o + tb * d;
        if (best >= 0) {
            const Tri& tr = sc.tris[best];
            const double eps = A.eps_rel * (k + 1) * (A.radius + L + tb * dlen);
            if (silhouette_dist(sc.faces[bface], hit) <= eps) flags |= SEG_EDGE;
            else if (tri_margin(tr, wb, ub, vb) <= eps) flags |= SEG_TRI;
        }
        A.out_tri[slot + k] = best >= 0 ? best : -1;
        A.out_face[slot + k] = bface;
        A.out_t[slot + k] = tb;
        A.out_len[slot + k] = best >= 0 ? L + tb * dlen : std::numeric_limits<double>::infinity();
        A.out_flags[slot + k] = flags;
        if (flags & (SEG_TIE | SEG_EDGE)) uncertain = true;

        // --- capture: closest approach of the segment [o, o + tb d] to each sphere centre
        for (int c = 0; c < A.nrx && k > last_t; ++c) {
            V3 ctr{A.rx[3 * c], A.rx[3 * c + 1], A.rx[3 * c + 2]};
            double s = dot(ctr - o, d) / dot(d, d);
            s = std::max(0.0, std::min(s, tb));
            double dist = norm(o + s * d - ctr);
            const double eps = A.eps_rel * (k + 1) * (A.radius + L + s * dlen);
            if (dist > A.r + eps) continue;
            Capture cp;
            cp.ray = b * A.n_dirs + rid;
            cp.tx = txi;
            cp.rx = c;
            cp.order = k;
            cp.flags = (dist <= A.r ? CAP_HIT : 0) | (std::fabs(dist - A.r) <= eps ? CAP_MARGINAL : 0) |
                       (uncertain ? CAP_UNCERTAIN : 0);
            cp.faces = seq;
            caps.push_back(std::move(cp));
        }
        if (best < 0 || k == K) break;
        if ((tset >> k) & 1u) {
            // --- transmission: straight on through a penetrable face,
            //     recorded as -2 - face
            if (!std::isfinite(sc.mats[sc.faces[bface].material].pen_db)) break;
            seq.push_back(-2 - bface);
            L += tb * dlen;
            o = hit;
            excl = bface;
            continue;
        }
        int refl = 0;
        for (int j = 0; j < k; ++j) refl += ((tset >> j) & 1u) ? 0 : 1;
        if (refl == A.max_refl) break;
        // --- specular reflection off the hit face (the segment ends at the hit point)
        seq.push_back(bface);
        L += tb * dlen;
        const Tri& tr = sc.tris[best];
        V3 n = unit(cross(tr.b - tr.a, tr.c - tr.a));
        d = d - (2.0 * dot(d, n)) * n;
        o = hit;
        excl = bface;
    }
}

// Any-hit test for a validation segment p -> q: is some triangle (not on the
// faces fa, fb) crossed strictly inside (t_min, len - t_min)?  `marginal` is set
// when a triangle's decision lies within eps of flipping.
bool occluded(const Scene& sc, V3 p, V3 q, int fa, int fb, double t_min, double eps, bool& marginal) {
    V3 dv = q - p;
    double len = norm(dv);
    V3 d = (1.0 / len) * dv;
    bool hit = false;
    for (const Tri& tr : sc.tris) {
        if (tr.face == fa || tr.face == fb) continue;
        double t, w, u, v;
        if (!ray_plane_bary(tr, p, d, t, w, u, v)) continue;
        double m = tri_margin(tr, w, u, v);
        if (m < -eps) continue;
        if (t < t_min - eps || t > len - t_min + eps) continue;
        bool inside_t = t > t_min && t < len - t_min;
        if (std::fabs(m) <= eps || !inside_t) { marginal = true; }
        if (m >= 0 && inside_t) hit = true;
    }
    return hit;
}

struct PathOut {
    bool valid = false, marginal = false;
    double length = 0, tau = 0;
    V3 aod, aoa;
    std::vector<CV3> amp;   // one C^3 amplitude per frequency
    // with n_grad materials requested: d amp / d eps_c of each material's
    // faces, [freq][material] (zero for materials the path does not reflect on)
    std::vector<CV3> damp;
};

// Transmit field pattern, an extension of the paper's ideal omnidirectional
// antenna: g(u) = sum_j w_j B_j(phi), phi the azimuth of the departure
// direction u and B_j the periodic hat of half-width 2 pi / 16 centred on
// azimuth 2 pi j / 16 (the hats sum to one, so w = 1 is the isotropic
// antenna).  g scales the field, so the power scales with g^2.  No pattern
// (w == nullptr): g = 1.
constexpr int kPatternTaps = 16;

double hat(int j, double phi) {
    const double step = 2.0 * kPi / kPatternTaps;
    const double d = std::fabs(std::remainder(phi - j * step, 2.0 * kPi));   // periodic distance
    return std::max(0.0, 1.0 - d / step);
}

double pattern_gain(const double* w, V3 u) {
    if (!w) return 1.0;
    const double phi = std::atan2(u.y, u.x);
    double g = 0.0;
    for (int j = 0; j < kPatternTaps; ++j) g += w[j] * hat(j, phi);
    return g;
}

// Image-method refinement of one candidate (tx, rx, faces[0..order)) and its
// field.  Paper Sec. III, steps 3, 4 and 6.
PathOut refine_one(const Scene& sc, V3 T, V3 R, const int32_t* faces, int order, const double* freqs,
                   int nfreq, double tx_power, double atten_db_per_km, double t_min, double eps_rel,
                   int n_grad = 0, const double* pattern = nullptr) {
    PathOut out;
    out.amp.assign(nfreq, CV3{});
    out.damp.assign((size_t)nfreq * n_grad, CV3{});
    // interaction j: face fid[j - 1], a transmission when listed as -2 - face
    std::vector<int> fid(order);
    std::vector<bool> trans(order);
    for (int j = 0; j < order; ++j) {
        trans[j] = faces[j] <= -2;
        fid[j] = trans[j] ? -2 - faces[j] : faces[j];
        if (fid[j] < 0 || fid[j] >= (int)sc.faces.size()) return out;   // not a face: no path
        // no path goes through an opaque face
        if (trans[j] && !std::isfinite(sc.mats[sc.faces[fid[j]].material].pen_db)) return out;
    }
    // image chain I_0 = T, I_j = mirror of I_{j-1} in the plane of face j (a
    // transmission goes straight on: I_j = I_{j-1})
    std::vector<V3> img(order + 1);
    img[0] = T;
    for (int j = 1; j <= order; ++j) {
        const Face& f = sc.faces[fid[j - 1]];
        img[j] = trans[j - 1] ? img[j - 1] : img[j - 1] - (2.0 * dot(img[j - 1] - f.p, f.n)) * f.n;
    }
    const double length = norm(R - img[order]);
    const double eps = eps_rel * (std::max(sc.radius, std::max(norm(T), norm(R))) + length);
    // interaction points, walking back from the receiver
    std::vector<V3> pts(order + 2);
    pts[0] = T;
    pts[order + 1] = R;
    V3 Q = R;
    for (int j = order; j >= 1; --j) {
        const Face& f = sc.faces[fid[j - 1]];
        V3 D = img[j] - Q;
        double den = dot(D, f.n);
        if (den == 0.0) return out;
        double s = dot(f.p - Q, f.n) / den;
        double seglen = norm(D);
        if (std::fabs(s) * seglen <= eps || std::fabs(1.0 - s) * seglen <= eps) out.marginal = true;
        if (!(s > 0.0 && s < 1.0)) return out;
        V3 P = Q + s * D;
        // inside the face: inside one of its triangles (edges inclusive)
        bool inside = false;
        for (int ti : f.tris) {
            const Tri& tr = sc.tris[ti];
            double t, w, u, v;
            if (!ray_plane_bary(tr, P - f.n, f.n, t, w, u, v)) continue;
            if (w >= 0 && u >= 0 && v >= 0) { inside = true; break; }
        }
        if (silhouette_dist(f, P) <= eps) out.marginal = true;
        if (!inside) return out;
        pts[j] = P;
        Q = P;
    }
    // every sub-segment unoccluded (faces at its endpoints excluded)
    for (int j = 0; j <= order; ++j) {
        int fa = j >= 1 ? fid[j - 1] : -1;
        int fb = j + 1 <= order ? fid[j] : -1;
        bool marg = false;
        if (occluded(sc, pts[j], pts[j + 1], fa, fb, t_min, eps, marg)) {
            if (marg) out.marginal = true;
            return out;
        }
        if (marg) out.marginal = true;
    }
    out.valid = true;
    out.length = length;
    out.tau = length / kC0;
    out.aod = unit(pts[1] - pts[0]);
    out.aoa = unit(pts[order] - R);
    // transmit polarisation: theta-hat of the departure direction (vertical
    // polarisation of an ideal omnidirectional antenna); phi = 0 on the axis
    V3 u = out.aod;
    double rho = std::sqrt(u.x * u.x + u.y * u.y);
    V3 e0 = rho > 0 ? V3{u.z * u.x / rho, u.z * u.y / rho, -rho} : V3{u.z, 0.0, 0.0};
    for (int fi = 0; fi < nfreq; ++fi) {
        const double f = freqs[fi];
        CV3 E{cplx(e0.x, 0), cplx(e0.y, 0), cplx(e0.z, 0)};
        // forward-mode derivatives of E, one per material (its eps_c)
        std::vector<CV3> dE(n_grad, CV3{});
        for (int j = 1; j <= order; ++j) {
            const Face& fc = sc.faces[fid[j - 1]];
            if (trans[j - 1]) {
                // transmission: the field (and its derivatives) times the
                // amplitude factor of the material's penetration loss
                const double tf = std::pow(10.0, -sc.mats[fc.material].pen_db / 20.0);
                E = CV3{tf * E.x, tf * E.y, tf * E.z};
                for (int m = 0; m < n_grad; ++m) dE[m] = CV3{tf * dE[m].x, tf * dE[m].y, tf * dE[m].z};
                continue;
            }
            V3 ki = unit(pts[j] - pts[j - 1]);
            V3 kr = unit(pts[j + 1] - pts[j]);
            V3 n = fc.n;
            double cos_t = std::fabs(dot(ki, n));
            V3 sv = cross(ki, n);
            double sl = norm(sv);
            if (sl < 1e-12) {
                // normal incidence: any s perpendicular to k gives the same result
                V3 ax = std::fabs(ki.x) < 0.9 ? V3{1, 0, 0} : V3{0, 1, 0};
                sv = unit(cross(ki, ax));
            } else {
                sv = (1.0 / sl) * sv;
            }
            V3 p_in = cross(sv, ki);
            V3 p_out = cross(sv, kr);
            cplx gte, gtm;
            fresnel(sc.mats[fc.material], f, cos_t, gte, gtm);
            // E -> Gamma_TE (E.s) s + Gamma_TM (E.p_in) p_out; a derivative
            // passes through the same map, and the reflection on a face of
            // material m adds the map with the Gammas' derivatives applied to E
            for (int m = 0; m < n_grad; ++m)
                dE[m] = cadd(cscale(gte * cdot(dE[m], sv), sv), cscale(gtm * cdot(dE[m], p_in), p_out));
            if (fc.material < n_grad) {
                cplx dte, dtm;
                fresnel_deps(sc.mats[fc.material], f, cos_t, dte, dtm);
                dE[fc.material] = cadd(dE[fc.material],
                                       cadd(cscale(dte * cdot(E, sv), sv), cscale(dtm * cdot(E, p_in), p_out)));
            }
            E = cadd(cscale(gte * cdot(E, sv), sv), cscale(gtm * cdot(E, p_in), p_out));
        }
        const double lam = kC0 / f;
        const double k0 = 2.0 * kPi * f / kC0;
        double mag = std::sqrt(tx_power) * lam / (4.0 * kPi * length) *
                     std::pow(10.0, -atten_db_per_km * length / 1000.0 / 20.0) * pattern_gain(pattern, out.aod);
        cplx ph = std::polar(mag, -k0 * length);
        out.amp[fi] = CV3{ph * E.x, ph * E.y, ph * E.z};
        for (int m = 0; m < n_grad; ++m) out.damp[(size_t)fi * n_grad + m] = CV3{ph * dE[m].x, ph * dE[m].y, ph * dE[m].z};
    }
    return out;
}

template <class F>
void parallel_for(int64_t n, int nthreads, F fn) {
    if (nthreads <= 1 || n < 2) {
        for (int64_t i = 0; i < n; ++i) fn(i, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) {
        th.emplace_back([&, t] {
            for (;;) {
                int64_t i = next.fetch_add(1);
                if (i >= n) break;
                fn(i, t);
            }
        });
    }
    for (auto& x : th) x.join();
}

}  // namespace

extern "C" {

// Build the FP64 scene at one frame.  xf (nullable) holds [n_obj][3][4]
// object-to-world transforms applied to the object's vertex range.
void* oracle_scene_new(const float* V, int64_t nv, const int32_t* T, const int32_t* tri_face, int64_t nt,
                       const int32_t* face_material, const int32_t* face_object, int32_t nf,
                       const double* materials, int32_t nm, const int64_t* obj_range, int32_t nobj,
                       const float* xf) {
    std::vector<float> W(V, V + 3 * nv);
    if (xf) {
        for (int o = 0; o < nobj; ++o) {
            const float* M = xf + 12 * o;
            for (int64_t i = obj_range[2 * o]; i < obj_range[2 * o + 1]; ++i) {
                float x = V[3 * i], y = V[3 * i + 1], z = V[3 * i + 2];
                W[3 * i] = xform_row(M, x, y, z);
                W[3 * i + 1] = xform_row(M + 4, x, y, z);
                W[3 * i + 2] = xform_row(M + 8, x, y, z);
            }
        }
    }
    Scene* sc = new Scene();
    sc->mats.resize(nm);
    for (int i = 0; i < nm; ++i) sc->mats[i] = {materials[3 * i], materials[3 * i + 1], materials[3 * i + 2]};
    sc->faces.resize(nf);
    for (int f = 0; f < nf; ++f) {
        sc->faces[f].material = face_material[f];
        sc->faces[f].object = face_object[f];
    }
    auto vtx = [&](int32_t i) { return V3{W[3 * i], W[3 * i + 1], W[3 * i + 2]}; };
    auto vref = [&](int32_t i) { return V3{V[3 * i], V[3 * i + 1], V[3 * i + 2]}; };
    for (int64_t i = 0; i < 3 * nv; i += 3) {
        V3 p{W[i], W[i + 1], W[i + 2]};
        sc->radius = std::max(sc->radius, norm(p));
    }
    sc->tris.resize(nt);
    std::vector<double> best_area(nf, -1.0);
    for (int64_t i = 0; i < nt; ++i) {
        Tri& tr = sc->tris[i];
        tr.a = vtx(T[3 * i]);
        tr.b = vtx(T[3 * i + 1]);
        tr.c = vtx(T[3 * i + 2]);
        tr.face = tri_face[i];
        double twice_area = norm(cross(tr.b - tr.a, tr.c - tr.a));
        tr.h0 = twice_area / norm(tr.c - tr.b);
        tr.h1 = twice_area / norm(tr.a - tr.c);
        tr.h2 = twice_area / norm(tr.b - tr.a);
        Face& f = sc->faces[tr.face];
        f.tris.push_back((int)i);
        // The plane of a face is that of its largest triangle, chosen in the
        // upload pose (first of equal ones): a rotated face's FP32 vertices
        // are no longer exactly coplanar, and the choice must not depend on
        // the rounding of the current pose.
        const V3 ra = vref(T[3 * i]), rb = vref(T[3 * i + 1]), rc = vref(T[3 * i + 2]);
        const double ref_area = norm(cross(rb - ra, rc - ra));
        if (ref_area > best_area[tr.face]) {
            best_area[tr.face] = ref_area;
            f.n = unit(cross(tr.b - tr.a, tr.c - tr.a));
            f.p = tr.a;
        }
    }
    // silhouette: edges used by exactly one triangle of the face (by coordinates)
    for (int f = 0; f < nf; ++f) {
        std::map<std::tuple<double, double, double, double, double, double>, std::pair<int, std::pair<V3, V3>>> cnt;
        for (int ti : sc->faces[f].tris) {
            const Tri& tr = sc->tris[ti];
            V3 vs[3] = {tr.a, tr.b, tr.c};
            for (int e = 0; e < 3; ++e) {
                V3 p = vs[e], q = vs[(e + 1) % 3];
                auto kp = std::make_tuple(p.x, p.y, p.z), kq = std::make_tuple(q.x, q.y, q.z);
                if (kq < kp) std::swap(kp, kq);
                auto key = std::tuple_cat(kp, kq);
                auto it = cnt.find(key);
                if (it == cnt.end()) cnt[key] = {1, {p, q}};
                else it->second.first += 1;
            }
        }
        for (auto& kv : cnt)
            if (kv.second.first == 1) sc->faces[f].silhouette.push_back(kv.second.second);
    }
    return sc;
}

void oracle_scene_free(void* s) { delete static_cast<Scene*>(s); }

// Bounding radius (about the origin) of the scene's vertices.
void oracle_scene_radius(const void* s, double* out) { *out = static_cast<const Scene*>(s)->radius; }

// Fibonacci sphere of n directions: z_i = 1 - (2i+1)/n, rho = sqrt(1 - z^2),
// phi_i = i * pi * (3 - sqrt 5) (the golden angle), evaluated in FP64 and
// rounded to FP32 (not renormalised).
void oracle_fibonacci(int64_t n, float* out) {
    const double ga = kPi * (3.0 - std::sqrt(5.0));
    for (int64_t i = 0; i < n; ++i) {
        double z = 1.0 - (2.0 * (double)i + 1.0) / (double)n;
        double rho = std::sqrt(1.0 - z * z);
        double phi = (double)i * ga;
        out[3 * i] = (float)(rho * std::cos(phi));
        out[3 * i + 1] = (float)(rho * std::sin(phi));
        out[3 * i + 2] = (float)z;
    }
}

// Trace rays (all, or the subset ray_ids[0..nsel)) from every transmitter.
// Per (source, branch, ray, segment) outputs, shape [ntx][n_branch][nsel][K+1]:
//   tri (-1 miss, -2 not traced), face, t (parametric), len (path length at
//   the hit), flags (SEG_*).
// Captures are written to cap_rows [capacity][4 + K] = (ray, tx, rx, order,
// faces... padded with -1) and cap_flags [capacity] (CAP_*), ordered by
// (tx, ray, bounce, rx).  Returns the number of captures; if it exceeds
// `capacity`, only the first `capacity` are written.
int64_t oracle_trace(const void* scene, const float* tx, int32_t ntx, const float* rx, int32_t nrx, double r,
                     const float* dirs, int64_t n_dirs, const int64_t* ray_ids, int64_t nsel, int32_t K,
                     int32_t max_refl, const uint32_t* sets, int32_t n_branch, double t_min, double eps_rel,
                     int32_t nthreads, int32_t* out_tri, int32_t* out_face, double* out_t, double* out_len,
                     int32_t* out_flags, int32_t* cap_rows, int32_t* cap_flags, int64_t capacity) {
    const Scene* sc = static_cast<const Scene*>(scene);
    double radius = sc->radius;
    for (int i = 0; i < ntx; ++i) radius = std::max(radius, norm(V3{tx[3 * i], tx[3 * i + 1], tx[3 * i + 2]}));
    for (int i = 0; i < nrx; ++i) radius = std::max(radius, norm(V3{rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]}));
    TraceArgs A{sc, tx, ntx, rx, nrx, r, dirs, ray_ids, nsel, K, max_refl, sets, n_branch, n_dirs, t_min, eps_rel,
                radius, out_tri, out_face, out_t, out_len, out_flags};
    const int64_t n = (int64_t)ntx * n_branch * nsel;
    std::vector<std::vector<Capture>> per(n);
    parallel_for(n, nthreads, [&](int64_t i, int) {
        trace_one(A, (int32_t)(i / (n_branch * nsel)), (int32_t)((i / nsel) % n_branch), i % nsel, per[i]);
    });
    int64_t cnt = 0;
    const int w = 4 + K;
    for (auto& v : per) {
        for (auto& c : v) {
            if (cnt < capacity) {
                int32_t* row = cap_rows + cnt * w;
                row[0] = (int32_t)c.ray;
                row[1] = c.tx;
                row[2] = c.rx;
                row[3] = c.order;
                for (int j = 0; j < K; ++j) row[4 + j] = j < (int)c.faces.size() ? c.faces[j] : -1;
                cap_flags[cnt] = c.flags;
            }
            ++cnt;
        }
    }
    return cnt;
}

// Refine candidate paths keys [n][3 + K] = (tx, rx, order, faces... padded
// -1; a transmission through face f as -2 - f).  Outputs per path: valid, marginal (validity within eps of flipping),
// length, tau, aod[3], aoa[3], amp [n][nfreq][3][2] (re, im).  pattern:
// the 16 transmit pattern weights, or null for the isotropic antenna.
void oracle_refine(const void* scene, const float* tx, const float* rx, const int32_t* keys, int64_t n,
                   int32_t K, const double* freqs, int32_t nfreq, double tx_power, double atten_db_per_km,
                   double t_min, double eps_rel, int32_t nthreads, uint8_t* valid, uint8_t* marginal,
                   double* length, double* tau, double* aod, double* aoa, double* amp, const double* pattern) {
    const Scene& sc = *static_cast<const Scene*>(scene);
    parallel_for(n, nthreads, [&](int64_t i, int) {
        const int32_t* key = keys + i * (3 + K);
        int t = key[0], c = key[1], order = key[2];
        V3 T{tx[3 * t], tx[3 * t + 1], tx[3 * t + 2]};
        V3 R{rx[3 * c], rx[3 * c + 1], rx[3 * c + 2]};
        PathOut p = refine_one(sc, T, R, key + 3, order, freqs, nfreq, tx_power, atten_db_per_km, t_min, eps_rel,
                               0, pattern);
        valid[i] = p.valid;
        marginal[i] = p.marginal;
        length[i] = p.length;
        tau[i] = p.tau;
        double* ad = aod + 3 * i;
        double* aa = aoa + 3 * i;
        ad[0] = p.aod.x; ad[1] = p.aod.y; ad[2] = p.aod.z;
        aa[0] = p.aoa.x; aa[1] = p.aoa.y; aa[2] = p.aoa.z;
        for (int f = 0; f < nfreq; ++f) {
            double* a = amp + ((i * nfreq + f) * 3) * 2;
            const CV3& e = p.amp[f];
            a[0] = e.x.real(); a[1] = e.x.imag();
            a[2] = e.y.real(); a[3] = e.y.imag();
            a[4] = e.z.real(); a[5] = e.z.imag();
        }
    });
}

// Derivatives of every candidate's amplitude with respect to each material's
// complex permittivity: damp [n][nfreq][n_mat][3][2] (re, im); zero for an
// invalid candidate.  Same candidates and validity as oracle_refine.
void oracle_refine_grad(const void* scene, const float* tx, const float* rx, const int32_t* keys, int64_t n,
                        int32_t K, const double* freqs, int32_t nfreq, double tx_power, double atten_db_per_km,
                        double t_min, double eps_rel, int32_t nthreads, double* damp, const double* pattern) {
    const Scene& sc = *static_cast<const Scene*>(scene);
    const int nm = (int)sc.mats.size();
    parallel_for(n, nthreads, [&](int64_t i, int) {
        const int32_t* key = keys + i * (3 + K);
        int t = key[0], c = key[1], order = key[2];
        V3 T{tx[3 * t], tx[3 * t + 1], tx[3 * t + 2]};
        V3 R{rx[3 * c], rx[3 * c + 1], rx[3 * c + 2]};
        PathOut p = refine_one(sc, T, R, key + 3, order, freqs, nfreq, tx_power, atten_db_per_km, t_min, eps_rel, nm,
                               pattern);
        for (int f = 0; f < nfreq; ++f)
            for (int m = 0; m < nm; ++m) {
                double* a = damp + (((i * nfreq + f) * nm + m) * 3) * 2;
                const CV3 e = p.valid ? p.damp[(size_t)f * nm + m] : CV3{};
                a[0] = e.x.real(); a[1] = e.x.imag();
                a[2] = e.y.real(); a[3] = e.y.imag();
                a[4] = e.z.real(); a[5] = e.z.imag();
            }
    });
}

// Penetration loss per material in dB (+inf: opaque), n = the scene's materials.
void oracle_scene_set_penetration(void* scene, const double* loss_db, int32_t n) {
    Scene& sc = *static_cast<Scene*>(scene);
    for (int m = 0; m < n && m < (int)sc.mats.size(); ++m) sc.mats[m].pen_db = loss_db[m];
}

// Transmit pattern gain of a departure direction (for unit pins).
double oracle_pattern_gain(const double* w, double ux, double uy, double uz) {
    return pattern_gain(w, V3{ux, uy, uz});
}

// Fresnel coefficients (for unit pins): out = (re TE, im TE, re TM, im TM).
void oracle_fresnel(double eps_r, double sigma, double const_gamma, double freq, double cos_theta, double* out) {
    Material m{eps_r, sigma, const_gamma};
    cplx te, tm;
    fresnel(m, freq, cos_theta, te, tm);
    out[0] = te.real(); out[1] = te.imag();
    out[2] = tm.real(); out[3] = tm.imag();
}

}  // extern "C"
