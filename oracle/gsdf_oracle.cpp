// Gradient-SDF reference implementation ("the oracle") -- TEST INFRASTRUCTURE.
//
// A plain, slow, single-threaded FP64 implementation of the per-frame depth
// tracking and fusion method of Gradient-SDF (Sommer et al., CVPR 2022).  It
// exists only so that tests, the smoke check and the CPU-baseline leg of the
// benchmark can compare the GPU library against an obviously correct
// reading of the paper.  The product path never links, loads or calls it.
// It shares no code with the GPU library.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fno-fast-math -shared -fPIC
// (-ffp-contract=off keeps the binary32 "decision arithmetic" below free of
// fused multiply-adds, so every float operation is one IEEE rounding.)
//
// What follows the paper where:
//   * SDF running weighted average ............ Sec. 3.1, Eq. (1)-(2)
//   * gradient accumulation g <- g + w n ...... Sec. 3.2, Eq. (3)
//   * regular grid v_j = v_s m_j .............. Sec. 3.1
//   * 8^3 voxel blocks in a hash map ........... Sec. 3.1 (blocks), Sec. 5.1
//   * tracking energy, weighted least squares .. Sec. 4.1, Eq. (5)
//   * first-order Taylor distance, gradient,
//     nearest voxel by rounding ................ Sec. 4.1, Eq. (14)-(16)
//   * Gauss-Newton with a Cholesky solve ....... Sec. 5.1
//   * per-pixel ray-band integration, linear
//     weight, FALS normals, 75 deg filter ...... Sec. 5.3 (Setup)
//
// Readings where the paper is silent (each is listed in the design notes):
//   * sign: psi > 0 inside objects, < 0 in free space (Sec. 3.1); the
//     stored gradient points into the object, away from the camera.
//   * new distance estimate d(v) = n_w . (v - p), the point-to-plane
//     distance to the observed point p with the pixel's normal, clamped to
//     [-T, T]; linear weight w(d) = 1 (d <= eps), (T-d)/(T-eps) (eps<d<T),
//     0 (d >= T), eps = voxel size.
//   * voxels along the ray within truncation: the binary32 "decision
//     arithmetic" samples z_k = (D - T) + k (v_s/2), k = 0..2T/(v_s/2); the
//     voxel list is the sample voxels with consecutive repeats removed.
//   * normals: least-squares plane fit 1/z = a . [x/z, y/z, 1] on a 5x5
//     window (the FALS idea: the 3x3 matrix depends only on pixel geometry),
//     n = a/|a|; needs all 25 depths valid and |D_i - D_c| <= T.
//   * nearest voxel j* = floor(p / v_s + 1/2) per axis.
//   * tracking weight w_k: Huber IRLS weight min(1, delta/|r|).
//   * solve (H + mu I) dxi = -b with mu = damping * tr(H)/6; pose update
//     T <- exp(dxi^) T (left, world frame), dxi = (rho, phi).
//   * depth pyramid: 2x2 mean when all four are valid and max-min <= T.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <memory>
#include <unordered_map>
#include <vector>

namespace {

constexpr int kB = 8;               // voxels per block edge
constexpr int kBV = kB * kB * kB;   // voxels per block

struct Voxel {
    double psi = 0.0;               // running weighted mean, Eq. (1)
    double W = 0.0;                 // accumulated weight, Eq. (2)
    double g[3] = {0.0, 0.0, 0.0};  // accumulated weighted normals, Eq. (3)
};

struct Block {
    Voxel v[kBV];
};

struct I3 {
    int x, y, z;
};

int floordiv8(int m) {
    // floor(m / 8) for any sign
    return (int)std::floor((double)m / 8.0);
}

int64_t pack_key(int bx, int by, int bz) {
    const int64_t o = 1 << 20;
    return ((int64_t)(bx + o) << 42) | ((int64_t)(by + o) << 21) | (int64_t)(bz + o);
}

void unpack_key(int64_t k, int* bx, int* by, int* bz) {
    const int64_t o = 1 << 20, mask = (1 << 21) - 1;
    *bx = (int)(((k >> 42) & mask) - o);
    *by = (int)(((k >> 21) & mask) - o);
    *bz = (int)((k & mask) - o);
}

int local_index(int lx, int ly, int lz) { return lx + kB * ly + kB * kB * lz; }

}  // namespace

extern "C" {

struct OrcCam {
    double fx, fy, cx, cy;
    int32_t width, height;
    double zmin, zmax;
};

struct OrcMap {
    double vs;          // voxel size
    double T;           // truncation distance
    int bounded;
    int bmin[3], bmax[3];   // half-open block range when bounded
    std::unordered_map<int64_t, std::unique_ptr<Block>> blocks;
};

}  // extern "C"

namespace {

Block* find_block(const OrcMap* M, int bx, int by, int bz) {
    auto it = M->blocks.find(pack_key(bx, by, bz));
    return it == M->blocks.end() ? nullptr : it->second.get();
}

Voxel* find_voxel(const OrcMap* M, const I3& m) {
    int bx = floordiv8(m.x), by = floordiv8(m.y), bz = floordiv8(m.z);
    Block* b = find_block(M, bx, by, bz);
    if (!b) return nullptr;
    return &b->v[local_index(m.x - 8 * bx, m.y - 8 * by, m.z - 8 * bz)];
}

bool in_bounds(const OrcMap* M, int bx, int by, int bz) {
    if (!M->bounded) return true;
    return bx >= M->bmin[0] && bx < M->bmax[0] && by >= M->bmin[1] && by < M->bmax[1] &&
           bz >= M->bmin[2] && bz < M->bmax[2];
}

// ---------------------------------------------------------------------------
// Pixel validity (depth cut-off, Sec. 5.3) -- exact binary32 comparisons.
// ---------------------------------------------------------------------------
bool depth_valid(float D, const OrcCam& c) {
    return std::isfinite(D) && D > 0.0f && D >= (float)c.zmin && D <= (float)c.zmax;
}

// ---------------------------------------------------------------------------
// Decision arithmetic: which voxels a pixel's ray band touches (binary32).
// ---------------------------------------------------------------------------
struct Decision {
    float ifx, ify, cxf, cyf, invvs, Tf, Df;
    float R[9], t[3];
    int nsamples;
};

Decision make_decision(const OrcMap* M, const OrcCam& c, const double* T) {
    Decision d;
    d.ifx = (float)(1.0 / c.fx);
    d.ify = (float)(1.0 / c.fy);
    d.cxf = (float)c.cx;
    d.cyf = (float)c.cy;
    d.invvs = (float)(1.0 / M->vs);
    d.Tf = (float)M->T;
    d.Df = (float)(M->vs / 2.0);
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) d.R[3 * i + j] = (float)T[4 * i + j];
        d.t[i] = (float)T[4 * i + 3];
    }
    d.nsamples = (int)std::floor(2.0 * M->T / (M->vs / 2.0) + 0.5) + 1;
    return d;
}

// Voxels sampled along the depth band [D - T, D + T] of pixel (u, v), with
// consecutive repeats removed.
std::vector<I3> band_voxels(const Decision& d, int u, int v, float D) {
    std::vector<I3> out;
    float xr = ((float)u - d.cxf) * d.ifx;
    float yr = ((float)v - d.cyf) * d.ify;
    for (int k = 0; k < d.nsamples; ++k) {
        float z = (D - d.Tf) + (float)k * d.Df;
        if (!(z > 0.0f)) continue;
        float X = z * xr;
        float Y = z * yr;
        int m[3];
        for (int i = 0; i < 3; ++i) {
            float a = d.R[3 * i + 0] * X;
            float b = d.R[3 * i + 1] * Y;
            float e = d.R[3 * i + 2] * z;
            float q = ((a + b) + e) + d.t[i];
            float s = q * d.invvs;
            m[i] = (int)std::floor(s + 0.5f);
        }
        if (out.empty() || out.back().x != m[0] || out.back().y != m[1] || out.back().z != m[2])
            out.push_back({m[0], m[1], m[2]});
    }
    return out;
}

// ---------------------------------------------------------------------------
// Small dense linear algebra in FP64.
// ---------------------------------------------------------------------------
// Gaussian elimination with partial pivoting for an n x n system (n <= 6).
bool solve_dense(int n, const double* A_in, const double* b_in, double* x) {
    double A[36], b[6];
    std::memcpy(A, A_in, sizeof(double) * n * n);
    std::memcpy(b, b_in, sizeof(double) * n);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[p * n + k]);
            std::swap(b[c], b[p]);
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * x[k];
        x[r] = s / A[r * n + r];
    }
    return true;
}

// Cholesky factorisation A = L L^T and solve A x = b (Sec. 5.1: the GN
// system is solved by Cholesky decomposition).
bool cholesky_solve6(const double* A, const double* b, double* x) {
    double L[36] = {0};
    for (int j = 0; j < 6; ++j) {
        double s = A[j * 6 + j];
        for (int k = 0; k < j; ++k) s -= L[j * 6 + k] * L[j * 6 + k];
        if (!(s > 0.0)) return false;
        L[j * 6 + j] = std::sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double t = A[i * 6 + j];
            for (int k = 0; k < j; ++k) t -= L[i * 6 + k] * L[j * 6 + k];
            L[i * 6 + j] = t / L[j * 6 + j];
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * 6 + k] * y[k];
        y[i] = s / L[i * 6 + i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= L[k * 6 + i] * x[k];
        x[i] = s / L[i * 6 + i];
    }
    return true;
}

void hat(const double* w, double* K) {
    K[0] = 0;     K[1] = -w[2]; K[2] = w[1];
    K[3] = w[2];  K[4] = 0;     K[5] = -w[0];
    K[6] = -w[1]; K[7] = w[0];  K[8] = 0;
}

void matmul3(const double* A, const double* B, double* C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

// Exponential map of se(3), xi = (rho, phi): R = I + A K + B K^2,
// V = I + B K + C K^2, t = V rho, with K = [phi]x (textbook closed form).
void se3_exp(const double* xi, double* T) {
    const double* rho = xi;
    const double* phi = xi + 3;
    double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    double th = std::sqrt(th2);
    double A, B, C;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        A = std::sin(th) / th;
        B = (1.0 - std::cos(th)) / th2;
        C = (th - std::sin(th)) / (th2 * th);
    }
    double K[9], K2[9];
    hat(phi, K);
    matmul3(K, K, K2);
    double R[9], V[9];
    for (int i = 0; i < 9; ++i) {
        double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * K[i] + B * K2[i];
        V[i] = I + B * K[i] + C * K2[i];
    }
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T[4 * i + j] = R[3 * i + j];
        T[4 * i + 3] = V[3 * i + 0] * rho[0] + V[3 * i + 1] * rho[1] + V[3 * i + 2] * rho[2];
    }
}

// T <- A * T for 3x4 rigid transforms.
void compose_left(const double* A, double* T) {
    double out[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 4; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[4 * i + k] * T[4 * k + j];
            out[4 * i + j] = s + (j == 3 ? A[4 * i + 3] : 0.0);
        }
    }
    std::memcpy(T, out, sizeof(out));
}

// Left Jacobian of SE(3) as the series sum_{n>=0} ad(xi)^n / (n+1)!, with
// ad(xi) = [[phi^, rho^], [0, phi^]] -- the definition, summed until the
// terms vanish in double precision.
void se3_left_jacobian(const double* xi, double* Jl) {
    double ad[36] = {0};
    double P[9], Rh[9];
    hat(xi + 3, P);
    hat(xi, Rh);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            ad[6 * i + j] = P[3 * i + j];
            ad[6 * i + j + 3] = Rh[3 * i + j];
            ad[6 * (i + 3) + j + 3] = P[3 * i + j];
        }
    double term[36] = {0};
    for (int i = 0; i < 6; ++i) term[7 * i] = 1.0;
    std::memcpy(Jl, term, sizeof(term));
    for (int n = 1; n < 80; ++n) {
        double nt[36];
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double s = 0;
                for (int k = 0; k < 6; ++k) s += term[6 * i + k] * ad[6 * k + j];
                nt[6 * i + j] = s / (double)(n + 1);
            }
        double mx = 0;
        for (int i = 0; i < 36; ++i) {
            term[i] = nt[i];
            Jl[i] += nt[i];
            mx = std::max(mx, std::fabs(nt[i]));
        }
        if (mx < 1e-300) break;
    }
}

// ---------------------------------------------------------------------------
// Normals: least-squares plane fit on the 5x5 window (FALS idea).
// ---------------------------------------------------------------------------
struct Normal {
    bool valid;
    double n[3];     // camera frame, unit, n . x > 0
    double cosang;   // |n . x| / |x|
};

Normal fals_normal(const float* depth, const OrcCam& c, float Tf, int u, int v) {
    Normal r{false, {0, 0, 0}, 0};
    const int hw = 2;
    if (u < hw || v < hw || u >= c.width - hw || v >= c.height - hw) return r;
    float Dc = depth[(size_t)v * c.width + u];
    if (!depth_valid(Dc, c)) return r;
    double A[9] = {0}, b[3] = {0};
    for (int dv = -hw; dv <= hw; ++dv)
        for (int du = -hw; du <= hw; ++du) {
            float Di = depth[(size_t)(v + dv) * c.width + (u + du)];
            if (!depth_valid(Di, c)) return r;
            if (!(std::fabs(Di - Dc) <= Tf)) return r;   // binary32, exact here
            double ray[3] = {((double)(u + du) - c.cx) / c.fx, ((double)(v + dv) - c.cy) / c.fy, 1.0};
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) A[3 * i + j] += ray[i] * ray[j];
                b[i] += ray[i] / (double)Di;
            }
        }
    double a[3];
    if (!solve_dense(3, A, b, a)) return r;
    double na = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    if (!(na > 0)) return r;
    double ray[3] = {((double)u - c.cx) / c.fx, ((double)v - c.cy) / c.fy, 1.0};
    double dot = 0, nr = 0;
    for (int i = 0; i < 3; ++i) {
        r.n[i] = a[i] / na;
        dot += r.n[i] * ray[i];
        nr += ray[i] * ray[i];
    }
    if (dot < 0) {   // orient away from the camera
        for (int i = 0; i < 3; ++i) r.n[i] = -r.n[i];
        dot = -dot;
    }
    r.cosang = dot / std::sqrt(nr);
    r.valid = true;
    return r;
}

double w_linear(double d, double eps, double T) {
    if (d <= eps) return 1.0;
    if (d >= T) return 0.0;
    return (T - d) / (T - eps);
}

double huber_rho(double r, double delta) {
    double a = std::fabs(r);
    return a <= delta ? 0.5 * r * r : delta * a - 0.5 * delta * delta;
}

double huber_weight(double r, double delta) {
    double a = std::fabs(r);
    return a <= delta ? 1.0 : delta / a;
}

void transform(const double* T, const double* x, double* q) {
    for (int i = 0; i < 3; ++i)
        q[i] = T[4 * i] * x[0] + T[4 * i + 1] * x[1] + T[4 * i + 2] * x[2] + T[4 * i + 3];
}

I3 nearest_voxel(const double* q, double vs) {
    return {(int)std::floor(q[0] / vs + 0.5), (int)std::floor(q[1] / vs + 0.5),
            (int)std::floor(q[2] / vs + 0.5)};
}

// Taylor distance at q from the nearest voxel (Eq. (14)-(16)).  Returns false
// when the voxel is not allocated or carries no observation.
bool taylor(const OrcMap* M, const double* q, double* r, double* gh, I3* mstar, Voxel** vox) {
    I3 m = nearest_voxel(q, M->vs);
    Voxel* V = find_voxel(M, m);
    if (!V || !(V->W > 0.0)) return false;
    double ng = std::sqrt(V->g[0] * V->g[0] + V->g[1] * V->g[1] + V->g[2] * V->g[2]);
    if (!(ng > 0.0)) return false;
    double d = V->psi;
    for (int i = 0; i < 3; ++i) gh[i] = V->g[i] / ng;
    double vj[3] = {M->vs * m.x, M->vs * m.y, M->vs * m.z};
    for (int i = 0; i < 3; ++i) d += gh[i] * (q[i] - vj[i]);
    *r = d;
    if (mstar) *mstar = m;
    if (vox) *vox = V;
    return true;
}

// Tri-linear distance at q (Sec. 4.1 Eq. (12)-(13)), the direct SDF tracking
// the paper compares against: the 8 voxel centres around q,
// v_s (b + (i, j, k)) with b = floor(q / v_s) and i, j, k in {0, 1}, weighted
// by the tri-linear coefficients of f = q / v_s - b; its gradient is the
// derivative of that interpolant, i.e. differences of corner values along
// each axis weighted bilinearly in the other two (the same eight lookups).
// Returns false unless all eight voxels are allocated and observed.
bool trilinear(const OrcMap* M, const double* q, double* r, double* grad) {
    const double vs = M->vs;
    int b[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        const double s = q[a] / vs;
        b[a] = (int)std::floor(s);
        f[a] = s - b[a];
    }
    double c[2][2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                const Voxel* V = find_voxel(M, {b[0] + i, b[1] + j, b[2] + k});
                if (!V || !(V->W > 0.0)) return false;
                c[i][j][k] = V->psi;
            }
    const double wx[2] = {1.0 - f[0], f[0]}, wy[2] = {1.0 - f[1], f[1]}, wz[2] = {1.0 - f[2], f[2]};
    double d = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) d += c[i][j][k] * wx[i] * wy[j] * wz[k];
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) gx += (c[1][j][k] - c[0][j][k]) * wy[j] * wz[k];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k) gy += (c[i][1][k] - c[i][0][k]) * wx[i] * wz[k];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) gz += (c[i][j][1] - c[i][j][0]) * wx[i] * wy[j];
    *r = d;
    grad[0] = gx / vs;
    grad[1] = gy / vs;
    grad[2] = gz / vs;
    return true;
}

// Normal equations of the Huber-weighted tracking energy at pose T for one
// depth image (values in double).  out29 = 21 upper-triangular H entries
// (row-major), 6 of b, energy, count.  model 0: the Taylor distance of
// Eq. (14)-(16); model 1: the tri-linear distance of Eq. (12)-(13).
void normal_equations(const OrcMap* M, const double* depth, const OrcCam& c, const double* T,
                      double delta, double* out29, int model = 0) {
    double H[36] = {0}, b[6] = {0}, E = 0, n = 0;
    for (int v = 0; v < c.height; ++v)
        for (int u = 0; u < c.width; ++u) {
            double D = depth[(size_t)v * c.width + u];
            if (!(std::isfinite(D) && D > 0 && (float)D >= (float)c.zmin && (float)D <= (float)c.zmax))
                continue;
            double x[3] = {D * ((double)u - c.cx) / c.fx, D * ((double)v - c.cy) / c.fy, D};
            double q[3], r, gh[3];
            transform(T, x, q);
            if (model == 0 ? !taylor(M, q, &r, gh, nullptr, nullptr) : !trilinear(M, q, &r, gh)) continue;
            double J[6] = {gh[0], gh[1], gh[2],
                           q[1] * gh[2] - q[2] * gh[1],
                           q[2] * gh[0] - q[0] * gh[2],
                           q[0] * gh[1] - q[1] * gh[0]};
            double w = huber_weight(r, delta);
            for (int i = 0; i < 6; ++i) {
                for (int j = 0; j < 6; ++j) H[6 * i + j] += w * J[i] * J[j];
                b[i] += w * J[i] * r;
            }
            E += huber_rho(r, delta);
            n += 1;
        }
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) out29[k++] = H[6 * i + j];
    for (int i = 0; i < 6; ++i) out29[21 + i] = b[i];
    out29[27] = E;
    out29[28] = n;
}

// One damped Gauss-Newton step from the packed normal equations.  Returns
// false (and leaves T unchanged) when the Cholesky factorisation fails.
bool gn_step(const double* ne, double damping, double* T, double* dxi_out) {
    double H[36];
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            H[6 * i + j] = ne[k];
            H[6 * j + i] = ne[k];
            ++k;
        }
    double tr = 0;
    for (int i = 0; i < 6; ++i) tr += H[7 * i];
    double mu = damping * tr / 6.0;
    for (int i = 0; i < 6; ++i) H[7 * i] += mu;
    double rhs[6], dxi[6];
    for (int i = 0; i < 6; ++i) rhs[i] = -ne[21 + i];
    if (!cholesky_solve6(H, rhs, dxi)) return false;
    double E[12];
    se3_exp(dxi, E);
    compose_left(E, T);
    if (dxi_out) std::memcpy(dxi_out, dxi, sizeof(dxi));
    return true;
}

}  // namespace

// ===========================================================================
// C interface (called from Python through ctypes)
// ===========================================================================
extern "C" {

OrcMap* orc_map_new(double voxel_size, double truncation, int bounded, const int32_t* bmin,
                    const int32_t* bmax) {
    OrcMap* M = new OrcMap();
    M->vs = voxel_size;
    M->T = truncation;
    M->bounded = bounded;
    for (int i = 0; i < 3; ++i) {
        M->bmin[i] = bounded ? bmin[i] : 0;
        M->bmax[i] = bounded ? bmax[i] : 0;
    }
    return M;
}

void orc_map_free(OrcMap* M) { delete M; }

int64_t orc_num_blocks(const OrcMap* M) { return (int64_t)M->blocks.size(); }

OrcMap* orc_map_clone(const OrcMap* M) {
    OrcMap* C = orc_map_new(M->vs, M->T, M->bounded, M->bmin, M->bmax);
    for (auto& kv : M->blocks) C->blocks[kv.first] = std::make_unique<Block>(*kv.second);
    return C;
}

// Sorted (x, y, z) block keys.
void orc_export_keys(const OrcMap* M, int32_t* out) {
    std::vector<std::array<int, 3>> keys;
    keys.reserve(M->blocks.size());
    for (auto& kv : M->blocks) {
        int x, y, z;
        unpack_key(kv.first, &x, &y, &z);
        keys.push_back({x, y, z});
    }
    std::sort(keys.begin(), keys.end());
    for (size_t i = 0; i < keys.size(); ++i)
        for (int j = 0; j < 3; ++j) out[3 * i + j] = keys[i][j];
}

// Voxel values of the given blocks, voxel order lx + 8 ly + 64 lz.  Missing
// blocks read as zeros and set found[i] = 0.
void orc_export_voxels(const OrcMap* M, const int32_t* keys, int64_t n, double* psi, double* g,
                       double* W, int32_t* found) {
    for (int64_t i = 0; i < n; ++i) {
        Block* b = find_block(M, keys[3 * i], keys[3 * i + 1], keys[3 * i + 2]);
        if (found) found[i] = b ? 1 : 0;
        for (int j = 0; j < kBV; ++j) {
            const Voxel* V = b ? &b->v[j] : nullptr;
            psi[i * kBV + j] = V ? V->psi : 0.0;
            W[i * kBV + j] = V ? V->W : 0.0;
            for (int k = 0; k < 3; ++k) g[(i * kBV + j) * 3 + k] = V ? V->g[k] : 0.0;
        }
    }
}

// Set voxel values of the given blocks (creating blocks as needed).
void orc_import_voxels(OrcMap* M, const int32_t* keys, int64_t n, const double* psi,
                       const double* g, const double* W) {
    for (int64_t i = 0; i < n; ++i) {
        int64_t key = pack_key(keys[3 * i], keys[3 * i + 1], keys[3 * i + 2]);
        auto& slot = M->blocks[key];
        if (!slot) slot = std::make_unique<Block>();
        for (int j = 0; j < kBV; ++j) {
            Voxel& V = slot->v[j];
            V.psi = psi[i * kBV + j];
            V.W = W[i * kBV + j];
            for (int k = 0; k < 3; ++k) V.g[k] = g[(i * kBV + j) * 3 + k];
        }
    }
}

// Voxel list of one pixel's band (decision arithmetic); returns the count.
int orc_band_voxels(const OrcMap* M, const OrcCam* cam, const double* T, int u, int v, float D,
                    int32_t* out, int cap) {
    Decision d = make_decision(M, *cam, T);
    std::vector<I3> vox = band_voxels(d, u, v, D);
    int n = (int)vox.size();
    for (int i = 0; i < n && i < cap; ++i) {
        out[3 * i] = vox[i].x;
        out[3 * i + 1] = vox[i].y;
        out[3 * i + 2] = vox[i].z;
    }
    return n;
}

// Allocation (Sec. 5.3 / Sec. 3.1): every block holding a band voxel of a
// valid pixel.  Returns the number of blocks created.
int64_t orc_allocate(OrcMap* M, const float* depth, const OrcCam* cam, const double* T) {
    Decision d = make_decision(M, *cam, T);
    int64_t created = 0;
    for (int v = 0; v < cam->height; ++v)
        for (int u = 0; u < cam->width; ++u) {
            float D = depth[(size_t)v * cam->width + u];
            if (!depth_valid(D, *cam)) continue;
            for (const I3& m : band_voxels(d, u, v, D)) {
                int bx = floordiv8(m.x), by = floordiv8(m.y), bz = floordiv8(m.z);
                if (!in_bounds(M, bx, by, bz)) continue;
                auto& slot = M->blocks[pack_key(bx, by, bz)];
                if (!slot) {
                    slot = std::make_unique<Block>();
                    ++created;
                }
            }
        }
    return created;
}

// Normals of a depth image: n (H*W*3, camera frame), valid flag and the
// cosine between normal and viewing ray.
void orc_normals(const float* depth, const OrcCam* cam, double truncation, double* n_out,
                 int32_t* valid_out, double* cos_out) {
    float Tf = (float)truncation;
    for (int v = 0; v < cam->height; ++v)
        for (int u = 0; u < cam->width; ++u) {
            size_t i = (size_t)v * cam->width + u;
            Normal nr = fals_normal(depth, *cam, Tf, u, v);
            valid_out[i] = nr.valid ? 1 : 0;
            cos_out[i] = nr.cosang;
            for (int k = 0; k < 3; ++k) n_out[3 * i + k] = nr.n[k];
        }
}

// Fusion (Eq. (1)-(3)), observation by observation in pixel order.
// eps: linear-weight plateau; cos_min: cosine of the maximum viewing angle.
// gradients = 0 fuses the distance and weight only (Eq. (1)-(2)), leaving
// g untouched: the plain SDF map without stored gradients that the paper's
// runtime comparison integrates (Sec. 5.3).
// marginal_out (optional, H*W): 1 where the angle test is within margin of
// its threshold.  Returns the number of voxel updates with w > 0.
int64_t orc_integrate(OrcMap* M, const float* depth, const OrcCam* cam, const double* T,
                      double eps, double cos_min, double margin, int32_t gradients, int32_t* marginal_out) {
    Decision d = make_decision(M, *cam, T);
    float Tf = (float)M->T;
    const double* Rm = T;
    int64_t updates = 0;
    for (int v = 0; v < cam->height; ++v)
        for (int u = 0; u < cam->width; ++u) {
            size_t pix = (size_t)v * cam->width + u;
            if (marginal_out) marginal_out[pix] = 0;
            float Df = depth[pix];
            if (!depth_valid(Df, *cam)) continue;
            Normal nr = fals_normal(depth, *cam, Tf, u, v);
            if (!nr.valid) continue;
            if (marginal_out && std::fabs(nr.cosang - cos_min) < margin) marginal_out[pix] = 1;
            if (!(nr.cosang >= cos_min)) continue;
            double D = Df;
            double x[3] = {D * ((double)u - cam->cx) / cam->fx, D * ((double)v - cam->cy) / cam->fy, D};
            double p[3], nw[3];
            transform(T, x, p);
            for (int i = 0; i < 3; ++i)
                nw[i] = Rm[4 * i] * nr.n[0] + Rm[4 * i + 1] * nr.n[1] + Rm[4 * i + 2] * nr.n[2];
            for (const I3& m : band_voxels(d, u, v, Df)) {
                Voxel* V = find_voxel(M, m);
                if (!V) continue;
                double vj[3] = {M->vs * m.x, M->vs * m.y, M->vs * m.z};
                double dist = nw[0] * (vj[0] - p[0]) + nw[1] * (vj[1] - p[1]) + nw[2] * (vj[2] - p[2]);
                dist = std::min(M->T, std::max(-M->T, dist));
                double w = w_linear(dist, eps, M->T);
                if (!(w > 0.0)) continue;
                V->psi = (V->W * V->psi + w * dist) / (V->W + w);   // Eq. (1)
                V->W = V->W + w;                                      // Eq. (2)
                if (gradients)
                    for (int k = 0; k < 3; ++k) V->g[k] += w * nw[k]; // Eq. (3)
                ++updates;
            }
        }
    return updates;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Reduced-precision storage, emulated: psi/T and the mean gradient
// gbar = g / W are kept rounded to bfloat16 or IEEE binary16 and W to
// binary32, updated once per frame from float64 per-frame sums:
//   psi <- (W psi + S_wd) / (W + S_w),  gbar <- (W gbar + S_wn) / (W + S_w),
//   W <- W + S_w      (Eq. (1)-(3) applied to the frame's observations).
// For such maps the voxel's g field holds gbar.
// ---------------------------------------------------------------------------
double round_to_bits(double x, int bits) {
    // round to `bits` significant bits, ties to even (default rounding mode)
    if (x == 0.0 || !std::isfinite(x)) return x;
    int e;
    const double m = std::frexp(x, &e);  // x = m 2^e, 0.5 <= |m| < 1
    return std::ldexp(std::nearbyint(std::ldexp(m, bits)), e - bits);
}

double round_storage(double x, int storage) {
    if (storage == 1) return round_to_bits(x, 8);            // bfloat16: 8 significant bits
    if (storage == 2) {                                        // binary16
        if (std::fabs(x) < std::ldexp(1.0, -14))               // subnormal: quantum 2^-24
            return std::ldexp(std::nearbyint(std::ldexp(x, 24)), -24);
        return round_to_bits(x, 11);
    }
    return x;
}

}  // namespace

extern "C" {

int64_t orc_integrate_rounded(OrcMap* M, const float* depth, const OrcCam* cam, const double* T,
                              double eps, double cos_min, int storage) {
    Decision d = make_decision(M, *cam, T);
    float Tf = (float)M->T;
    struct Sum {
        double w = 0, wd = 0, wn[3] = {0, 0, 0};
    };
    std::unordered_map<int64_t, std::unordered_map<int, Sum>> frame;  // block -> voxel -> sums
    int64_t updates = 0;
    for (int v = 0; v < cam->height; ++v)
        for (int u = 0; u < cam->width; ++u) {
            float Df = depth[(size_t)v * cam->width + u];
            if (!depth_valid(Df, *cam)) continue;
            Normal nr = fals_normal(depth, *cam, Tf, u, v);
            if (!nr.valid || !(nr.cosang >= cos_min)) continue;
            double D = Df;
            double x[3] = {D * ((double)u - cam->cx) / cam->fx, D * ((double)v - cam->cy) / cam->fy, D};
            double p[3], nw[3];
            transform(T, x, p);
            for (int i = 0; i < 3; ++i) nw[i] = T[4 * i] * nr.n[0] + T[4 * i + 1] * nr.n[1] + T[4 * i + 2] * nr.n[2];
            for (const I3& m : band_voxels(d, u, v, Df)) {
                int bx = floordiv8(m.x), by = floordiv8(m.y), bz = floordiv8(m.z);
                if (!find_block(M, bx, by, bz)) continue;
                double vj[3] = {M->vs * m.x, M->vs * m.y, M->vs * m.z};
                double dist = nw[0] * (vj[0] - p[0]) + nw[1] * (vj[1] - p[1]) + nw[2] * (vj[2] - p[2]);
                dist = std::min(M->T, std::max(-M->T, dist));
                double w = w_linear(dist, eps, M->T);
                if (!(w > 0.0)) continue;
                Sum& S = frame[pack_key(bx, by, bz)][local_index(m.x - 8 * bx, m.y - 8 * by, m.z - 8 * bz)];
                S.w += w;
                S.wd += w * dist;
                for (int k = 0; k < 3; ++k) S.wn[k] += w * nw[k];
                ++updates;
            }
        }
    for (auto& bkv : frame) {
        Block* B = M->blocks[bkv.first].get();
        for (auto& vkv : bkv.second) {
            Voxel& V = B->v[vkv.first];
            const Sum& S = vkv.second;
            const double Wn = V.W + S.w;
            const double psi = (V.W * V.psi + S.wd) / Wn;
            V.psi = M->T * round_storage(psi / M->T, storage);
            for (int k = 0; k < 3; ++k) V.g[k] = round_storage((V.W * V.g[k] + S.wn[k]) / Wn, storage);
            V.W = (double)(float)Wn;
        }
    }
    return updates;
}

double orc_round_storage(double x, int storage) { return round_storage(x, storage); }

// Depth pyramid level (binary32): mean of each 2x2 block when all four are
// valid and their spread is within the truncation, else 0.
void orc_pyramid_down(const float* src, const OrcCam* cam, double truncation, float* dst) {
    int w2 = cam->width / 2, h2 = cam->height / 2;
    float Tf = (float)truncation;
    for (int v = 0; v < h2; ++v)
        for (int u = 0; u < w2; ++u) {
            float a = src[(size_t)(2 * v) * cam->width + 2 * u];
            float b = src[(size_t)(2 * v) * cam->width + 2 * u + 1];
            float c = src[(size_t)(2 * v + 1) * cam->width + 2 * u];
            float e = src[(size_t)(2 * v + 1) * cam->width + 2 * u + 1];
            bool ok = depth_valid(a, *cam) && depth_valid(b, *cam) && depth_valid(c, *cam) &&
                      depth_valid(e, *cam);
            float mx = std::max(std::max(a, b), std::max(c, e));
            float mn = std::min(std::min(a, b), std::min(c, e));
            ok = ok && (mx - mn <= Tf);
            dst[(size_t)v * w2 + u] = ok ? ((a + b) + (c + e)) * 0.25f : 0.0f;
        }
}

void orc_normal_equations(const OrcMap* M, const double* depth, const OrcCam* cam,
                          const double* T, double delta, double* out29) {
    normal_equations(M, depth, *cam, T, delta, out29);
}

// Fixed-iteration damped Gauss-Newton on one image (values in double).
// stats (optional, iters x 2): energy and count at each linearisation.
// Returns the number of failed (skipped) solves.
int orc_gn_level_model(const OrcMap* M, const double* depth, const OrcCam* cam, int iters,
                       double delta, double damping, double* T, double* stats, int model) {
    int failed = 0;
    for (int it = 0; it < iters; ++it) {
        double ne[29];
        normal_equations(M, depth, *cam, T, delta, ne, model);
        if (stats) {
            stats[2 * it] = ne[27];
            stats[2 * it + 1] = ne[28];
        }
        if (!gn_step(ne, damping, T, nullptr)) ++failed;
    }
    return failed;
}

int orc_gn_level(const OrcMap* M, const double* depth, const OrcCam* cam, int iters,
                 double delta, double damping, double* T, double* stats) {
    return orc_gn_level_model(M, depth, cam, iters, delta, damping, T, stats, 0);
}

// Coarse-to-fine tracking: pyramid (binary32), then iters[l] GN steps per
// level from the coarsest to the finest, with residual model `model`
// (0 Taylor, 1 tri-linear).
int orc_track_model(const OrcMap* M, const float* depth, const OrcCam* cam, int levels,
                    const int32_t* iters, double delta, double damping, double* T, double* stats, int model) {
    std::vector<std::vector<float>> pyr(levels);
    std::vector<OrcCam> cams(levels);
    pyr[0].assign(depth, depth + (size_t)cam->width * cam->height);
    cams[0] = *cam;
    for (int l = 1; l < levels; ++l) {
        const OrcCam& pc = cams[l - 1];
        OrcCam c = pc;
        c.width = pc.width / 2;
        c.height = pc.height / 2;
        c.fx = pc.fx / 2;
        c.fy = pc.fy / 2;
        c.cx = (pc.cx + 0.5) / 2 - 0.5;
        c.cy = (pc.cy + 0.5) / 2 - 0.5;
        pyr[l].resize((size_t)c.width * c.height);
        orc_pyramid_down(pyr[l - 1].data(), &pc, M->T, pyr[l].data());
        cams[l] = c;
    }
    int failed = 0, s = 0;
    for (int l = levels - 1; l >= 0; --l) {
        std::vector<double> dd(pyr[l].begin(), pyr[l].end());
        failed += orc_gn_level_model(M, dd.data(), &cams[l], iters[l], delta, damping, T,
                                     stats ? stats + 2 * s : nullptr, model);
        s += iters[l];
    }
    return failed;
}

int orc_track(const OrcMap* M, const float* depth, const OrcCam* cam, int levels,
              const int32_t* iters, double delta, double damping, double* T, double* stats) {
    return orc_track_model(M, depth, cam, levels, iters, delta, damping, T, stats, 0);
}

// Tri-linear distance and gradient at world point q (0 if undefined).
int orc_trilinear(const OrcMap* M, const double* q, double* r, double* grad) {
    return trilinear(M, q, r, grad) ? 1 : 0;
}

// ---- small numerical kernels exposed for pin tests ----
int orc_cholesky_solve6(const double* A, const double* b, double* x) {
    return cholesky_solve6(A, b, x) ? 1 : 0;
}
void orc_se3_exp(const double* xi, double* T) { se3_exp(xi, T); }
void orc_se3_left_jacobian(const double* xi, double* Jl) { se3_left_jacobian(xi, Jl); }
int orc_gn_step(const double* ne, double damping, double* T, double* dxi) {
    return gn_step(ne, damping, T, dxi) ? 1 : 0;
}
double orc_huber_rho(double r, double delta) { return huber_rho(r, delta); }
double orc_huber_weight(double r, double delta) { return huber_weight(r, delta); }
double orc_w_linear(double d, double eps, double T) { return w_linear(d, eps, T); }
void orc_nearest_voxel(const double* q, double vs, int32_t* m) {
    I3 r = nearest_voxel(q, vs);
    m[0] = r.x;
    m[1] = r.y;
    m[2] = r.z;
}
int orc_floordiv8(int m) { return floordiv8(m); }

// Taylor residual and its gradient direction at world point q (nan if none).
int orc_taylor(const OrcMap* M, const double* q, double* r, double* gh, int32_t* m) {
    I3 ms;
    if (!taylor(M, q, r, gh, &ms, nullptr)) return 0;
    m[0] = ms.x;
    m[1] = ms.y;
    m[2] = ms.z;
    return 1;
}

// ---------------------------------------------------------------------------
// Differentiable loss over keyframes.
//   L = sum_i sum_k rho_delta(r_ik),  T_i = exp(xi_i^) T0_i.
// Gradients: dL/dpsi_j = sum rho'(r); dL/dg_j = sum rho'(r) (I - gh gh^T)(q - v_j)/|g_j|;
// dL/dxi_i = Jl(xi_i)^T sum_k rho'(r_ik) [gh; q x gh].
// The voxel parameters are the map's psi and g (W only marks observed).
// assoc (K*H*W*3, optional): nearest-voxel association; freeze = 1 reads it,
// freeze = 0 writes it (pixels without a usable voxel get INT32_MIN).
// dpsi / dg (optional) are returned per block in key order of `keys`.
// ---------------------------------------------------------------------------
double orc_loss_grad(const OrcMap* M, int K, const double* depth, const OrcCam* cam,
                     const double* T0, const double* xi, double delta, int32_t* assoc,
                     int freeze, const int32_t* keys, int64_t nkeys, double* dpsi, double* dg,
                     double* dxi) {
    std::unordered_map<int64_t, int64_t> kidx;
    if (keys)
        for (int64_t i = 0; i < nkeys; ++i)
            kidx[pack_key(keys[3 * i], keys[3 * i + 1], keys[3 * i + 2])] = i;
    if (dpsi) std::fill(dpsi, dpsi + nkeys * kBV, 0.0);
    if (dg) std::fill(dg, dg + nkeys * kBV * 3, 0.0);
    double L = 0;
    const size_t npx = (size_t)cam->width * cam->height;
    for (int i = 0; i < K; ++i) {
        double E[12], T[12];
        se3_exp(xi + 6 * i, E);
        std::memcpy(T, T0 + 12 * i, sizeof(T));
        compose_left(E, T);
        double gl[6] = {0};
        for (int v = 0; v < cam->height; ++v)
            for (int u = 0; u < cam->width; ++u) {
                size_t pix = (size_t)v * cam->width + u;
                double D = depth[i * npx + pix];
                int32_t* as = assoc ? assoc + 3 * (i * npx + pix) : nullptr;
                if (!(std::isfinite(D) && D > 0 && (float)D >= (float)cam->zmin &&
                      (float)D <= (float)cam->zmax)) {
                    if (as && !freeze) as[0] = as[1] = as[2] = INT32_MIN;
                    continue;
                }
                double x[3] = {D * ((double)u - cam->cx) / cam->fx, D * ((double)v - cam->cy) / cam->fy, D};
                double q[3];
                transform(T, x, q);
                I3 m;
                if (as && freeze) {
                    if (as[0] == INT32_MIN) continue;
                    m = {as[0], as[1], as[2]};
                } else {
                    m = nearest_voxel(q, M->vs);
                }
                Voxel* V = find_voxel(M, m);
                double ng = V ? std::sqrt(V->g[0] * V->g[0] + V->g[1] * V->g[1] + V->g[2] * V->g[2]) : 0;
                if (!V || !(V->W > 0.0) || !(ng > 0.0)) {
                    if (as && !freeze) as[0] = as[1] = as[2] = INT32_MIN;
                    continue;
                }
                if (as && !freeze) {
                    as[0] = m.x;
                    as[1] = m.y;
                    as[2] = m.z;
                }
                double gh[3] = {V->g[0] / ng, V->g[1] / ng, V->g[2] / ng};
                double dq[3] = {q[0] - M->vs * m.x, q[1] - M->vs * m.y, q[2] - M->vs * m.z};
                double r = V->psi + gh[0] * dq[0] + gh[1] * dq[1] + gh[2] * dq[2];
                L += huber_rho(r, delta);
                double rp = huber_weight(r, delta) * r;   // rho'(r)
                double J[6] = {gh[0], gh[1], gh[2], q[1] * gh[2] - q[2] * gh[1],
                               q[2] * gh[0] - q[0] * gh[2], q[0] * gh[1] - q[1] * gh[0]};
                for (int k = 0; k < 6; ++k) gl[k] += rp * J[k];
                if (keys && (dpsi || dg)) {
                    int bx = floordiv8(m.x), by = floordiv8(m.y), bz = floordiv8(m.z);
                    auto it = kidx.find(pack_key(bx, by, bz));
                    if (it != kidx.end()) {
                        int64_t j = it->second * kBV + local_index(m.x - 8 * bx, m.y - 8 * by, m.z - 8 * bz);
                        if (dpsi) dpsi[j] += rp;
                        if (dg) {
                            double gd = gh[0] * dq[0] + gh[1] * dq[1] + gh[2] * dq[2];
                            for (int k = 0; k < 3; ++k) dg[3 * j + k] += rp * (dq[k] - gh[k] * gd) / ng;
                        }
                    }
                }
            }
        if (dxi) {
            double Jl[36];
            se3_left_jacobian(xi + 6 * i, Jl);
            for (int a = 0; a < 6; ++a) {
                double s = 0;
                for (int k = 0; k < 6; ++k) s += Jl[6 * k + a] * gl[k];
                dxi[6 * i + a] = s;
            }
        }
    }
    return L;
}

// ---------------------------------------------------------------------------
// Test helper: ray-cast the map's own Taylor surface, i.e. the first root
// along each ray of r(p) = psi_j* + gh_j* . (p - v_j*) with j* the nearest
// voxel of p.  Inside one nearest-voxel cell r is linear along the ray, so
// roots are exact.  Pixels without a root inside a cell get depth 0.
// ---------------------------------------------------------------------------
void orc_render_taylor(const OrcMap* M, const OrcCam* cam, const double* T, double smin,
                       double smax, double* depth_out) {
    const double vs = M->vs;
    for (int v = 0; v < cam->height; ++v)
        for (int u = 0; u < cam->width; ++u) {
            double ray[3] = {((double)u - cam->cx) / cam->fx, ((double)v - cam->cy) / cam->fy, 1.0};
            double o[3] = {T[3], T[7], T[11]}, d[3];
            for (int i = 0; i < 3; ++i) d[i] = T[4 * i] * ray[0] + T[4 * i + 1] * ray[1] + T[4 * i + 2] * ray[2];
            double s = smin, hit = 0.0;
            bool seen_neg = false;
            for (int step = 0; step < 100000 && s < smax; ++step) {
                double p[3] = {o[0] + s * d[0], o[1] + s * d[1], o[2] + s * d[2]};
                I3 m = nearest_voxel(p, vs);
                int mm[3] = {m.x, m.y, m.z};
                double sexit = smax;
                for (int k = 0; k < 3; ++k) {
                    if (d[k] > 0) sexit = std::min(sexit, ((mm[k] + 0.5) * vs - o[k]) / d[k]);
                    else if (d[k] < 0) sexit = std::min(sexit, ((mm[k] - 0.5) * vs - o[k]) / d[k]);
                }
                Voxel* V = find_voxel(M, m);
                double ng = V ? std::sqrt(V->g[0] * V->g[0] + V->g[1] * V->g[1] + V->g[2] * V->g[2]) : 0;
                if (V && V->W > 0 && ng > 0) {
                    double gh[3] = {V->g[0] / ng, V->g[1] / ng, V->g[2] / ng};
                    // r(s) = a + b s
                    double a = V->psi, b = 0;
                    for (int k = 0; k < 3; ++k) {
                        a += gh[k] * (o[k] - vs * mm[k]);
                        b += gh[k] * d[k];
                    }
                    double r_in = a + b * s;
                    if (r_in < 0) seen_neg = true;
                    if (seen_neg && b > 0) {
                        double sr = -a / b;
                        double margin = 1e-9 * vs;
                        if (sr > s + margin && sr < sexit - margin) {
                            double pr[3] = {o[0] + sr * d[0], o[1] + sr * d[1], o[2] + sr * d[2]};
                            I3 mc = nearest_voxel(pr, vs);
                            if (mc.x == m.x && mc.y == m.y && mc.z == m.z) hit = sr;
                            break;
                        }
                    }
                    if (r_in >= 0 && seen_neg) break;   // jumped over the surface
                }
                s = sexit + 1e-12;
            }
            depth_out[(size_t)v * cam->width + u] = hit;
        }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Photometric term over keyframes (joint refinement with colour).
//
// Surface point of voxel j (Sec. 4.2 Eq. (18)): p_j = v_j - psi_j gh_j, with
// gh_j held fixed (the paper treats it as a constant direction while psi
// changes).  Only voxels whose cell contains their surface point take part
// ("voxels that actually contain surface points", Sec. 4.2):
// max_k |psi_j gh_jk| <= v_s / 2, besides W > 0 and g != 0.
// Visibility nu_ij: x = R_i^T (p_j - t_i) has z >= zmin, projects to
// (u, v) = (fx x/z + cx, fy y/z + cy) with 0 <= u < width-1 and
// 0 <= v < height-1 (bilinear support), the depth D of the nearest pixel
// is valid with |z - D| <= T, and the surface faces the camera:
// gh_j . (p_j - t_i) > 0 (gh points into the solid).
// Residual per colour channel c against the voxel's stored colour rho_j:
//   r = I_i^c(u, v) - rho_j^c   (bilinear image sample),
// loss_i = lambda sum_{j visible} sum_c huber_delta(r).
// Gradients: d/drho = -lambda rho'(r); with e = sum_c lambda rho'(r_c) dI^c/d(u,v)
// and a = R_i (e . dpi/dx) (world frame): d/dpsi_j = -a . gh_j, and for a
// left increment of T_i, [-a ; a x p_j]; dxi_i = Jl(xi_i)^T of that sum.
// ---------------------------------------------------------------------------
namespace {

struct PhotoSample {
    double u, v, z, x[3];
};

bool photo_visible(const OrcCam& cam, const double* depth_i, const double* T, const double* p,
                   const double* gh, double trunc, PhotoSample* S) {
    double d[3] = {p[0] - T[3], p[1] - T[7], p[2] - T[11]};
    for (int r = 0; r < 3; ++r) S->x[r] = T[r] * d[0] + T[4 + r] * d[1] + T[8 + r] * d[2];  // R^T d
    S->z = S->x[2];
    if (!(S->z >= cam.zmin)) return false;
    S->u = cam.fx * S->x[0] / S->z + cam.cx;
    S->v = cam.fy * S->x[1] / S->z + cam.cy;
    if (!(S->u >= 0.0 && S->u < cam.width - 1 && S->v >= 0.0 && S->v < cam.height - 1)) return false;
    int iu = (int)std::floor(S->u + 0.5), iv = (int)std::floor(S->v + 0.5);
    double D = depth_i[(size_t)iv * cam.width + iu];
    if (!(std::isfinite(D) && D > 0 && (float)D >= (float)cam.zmin && (float)D <= (float)cam.zmax)) return false;
    if (!(std::fabs(S->z - D) <= trunc)) return false;
    return gh[0] * d[0] + gh[1] * d[1] + gh[2] * d[2] > 0.0;
}

// Bilinear sample of an H x W x 3 image and its derivatives in u and v.
void bilinear3(const double* img, const OrcCam& cam, double u, double v, double I[3], double dIu[3],
               double dIv[3]) {
    int u0 = (int)std::floor(u), v0 = (int)std::floor(v);
    double a = u - u0, b = v - v0;
    const double* p00 = img + 3 * ((size_t)v0 * cam.width + u0);
    const double* p10 = p00 + 3;
    const double* p01 = p00 + 3 * (size_t)cam.width;
    const double* p11 = p01 + 3;
    for (int c = 0; c < 3; ++c) {
        I[c] = (1 - a) * (1 - b) * p00[c] + a * (1 - b) * p10[c] + (1 - a) * b * p01[c] + a * b * p11[c];
        dIu[c] = (1 - b) * (p10[c] - p00[c]) + b * (p11[c] - p01[c]);
        dIv[c] = (1 - a) * (p01[c] - p00[c]) + a * (p11[c] - p10[c]);
    }
}

bool photo_surface(const Voxel& V, double vs, double gh[3]) {
    double ng = std::sqrt(V.g[0] * V.g[0] + V.g[1] * V.g[1] + V.g[2] * V.g[2]);
    if (!(V.W > 0.0) || !(ng > 0.0)) return false;
    for (int k = 0; k < 3; ++k) gh[k] = V.g[k] / ng;
    for (int k = 0; k < 3; ++k)
        if (std::fabs(V.psi * gh[k]) > 0.5 * vs) return false;
    return true;
}

}  // namespace

extern "C" {

// Photometric loss and gradients.  colors / dcolor: nkeys x 512 x 3 in the
// order of `keys` (voxel lx + 8 ly + 64 lz); dpsi: nkeys x 512; all gradient
// outputs optional (overwritten).  loss_kf: K values.  Returns the total.
double orc_photo_loss_grad(const OrcMap* M, int K, const double* depth, const double* rgb, const OrcCam* cam,
                           const double* T0, const double* xi, const int32_t* keys, int64_t nkeys,
                           const double* colors, double delta, double lambda, double* loss_kf,
                           double* dpsi, double* dcolor, double* dxi, int64_t* n_visible) {
    const size_t npx = (size_t)cam->width * cam->height;
    std::vector<double> T((size_t)12 * K), gl((size_t)6 * K, 0.0);
    for (int i = 0; i < K; ++i) {
        double E[12];
        se3_exp(xi + 6 * i, E);
        std::memcpy(&T[12 * i], T0 + 12 * i, 12 * sizeof(double));
        compose_left(E, &T[12 * i]);
        loss_kf[i] = 0.0;
    }
    if (dpsi) std::fill(dpsi, dpsi + nkeys * kBV, 0.0);
    if (dcolor) std::fill(dcolor, dcolor + nkeys * kBV * 3, 0.0);
    int64_t nvis = 0;
    for (int64_t b = 0; b < nkeys; ++b) {
        const Block* B = find_block(M, keys[3 * b], keys[3 * b + 1], keys[3 * b + 2]);
        if (!B) continue;
        for (int c = 0; c < kBV; ++c) {
            const Voxel& V = B->v[c];
            double gh[3];
            if (!photo_surface(V, M->vs, gh)) continue;
            int m[3] = {8 * keys[3 * b] + c % 8, 8 * keys[3 * b + 1] + (c / 8) % 8, 8 * keys[3 * b + 2] + c / 64};
            double p[3];
            for (int k = 0; k < 3; ++k) p[k] = M->vs * m[k] - V.psi * gh[k];
            const double* rho = colors + 3 * (b * kBV + c);
            for (int i = 0; i < K; ++i) {
                const double* Ti = &T[12 * i];
                PhotoSample S;
                if (!photo_visible(*cam, depth + i * npx, Ti, p, gh, M->T, &S)) continue;
                ++nvis;
                double I[3], dIu[3], dIv[3];
                bilinear3(rgb + 3 * i * npx, *cam, S.u, S.v, I, dIu, dIv);
                double eu = 0, ev = 0;
                for (int ch = 0; ch < 3; ++ch) {
                    double r = I[ch] - rho[ch];
                    loss_kf[i] += lambda * huber_rho(r, delta);
                    double rp = lambda * huber_weight(r, delta) * r;
                    if (dcolor) dcolor[3 * (b * kBV + c) + ch] -= rp;
                    eu += rp * dIu[ch];
                    ev += rp * dIv[ch];
                }
                // dL/dx (camera frame) through the projection, then world frame
                double gx[3] = {eu * cam->fx / S.z, ev * cam->fy / S.z,
                                -(eu * cam->fx * S.x[0] + ev * cam->fy * S.x[1]) / (S.z * S.z)};
                double a[3];
                for (int r = 0; r < 3; ++r) a[r] = Ti[4 * r] * gx[0] + Ti[4 * r + 1] * gx[1] + Ti[4 * r + 2] * gx[2];
                if (dpsi) dpsi[b * kBV + c] -= a[0] * gh[0] + a[1] * gh[1] + a[2] * gh[2];
                double* g6 = &gl[6 * i];
                g6[0] -= a[0];
                g6[1] -= a[1];
                g6[2] -= a[2];
                g6[3] += a[1] * p[2] - a[2] * p[1];
                g6[4] += a[2] * p[0] - a[0] * p[2];
                g6[5] += a[0] * p[1] - a[1] * p[0];
            }
        }
    }
    if (dxi) {
        for (int i = 0; i < K; ++i) {
            double Jl[36];
            se3_left_jacobian(xi + 6 * i, Jl);
            for (int q = 0; q < 6; ++q) {
                double s = 0;
                for (int k = 0; k < 6; ++k) s += Jl[6 * k + q] * gl[6 * i + k];
                dxi[6 * i + q] = s;
            }
        }
    }
    if (n_visible) *n_visible = nvis;
    double L = 0;
    for (int i = 0; i < K; ++i) L += loss_kf[i];
    return L;
}

// Mean colour of each surface voxel over the keyframes that see it
// (Sec. 4.2 Eq. (21)); count_out = N_j.  Voxels seen by none get 0.
void orc_mean_color(const OrcMap* M, int K, const double* depth, const double* rgb, const OrcCam* cam,
                    const double* T0, const double* xi, const int32_t* keys, int64_t nkeys, double* colors_out,
                    double* count_out) {
    const size_t npx = (size_t)cam->width * cam->height;
    std::vector<double> T((size_t)12 * K);
    for (int i = 0; i < K; ++i) {
        double E[12];
        se3_exp(xi + 6 * i, E);
        std::memcpy(&T[12 * i], T0 + 12 * i, 12 * sizeof(double));
        compose_left(E, &T[12 * i]);
    }
    std::fill(colors_out, colors_out + nkeys * kBV * 3, 0.0);
    std::fill(count_out, count_out + nkeys * kBV, 0.0);
    for (int64_t b = 0; b < nkeys; ++b) {
        const Block* B = find_block(M, keys[3 * b], keys[3 * b + 1], keys[3 * b + 2]);
        if (!B) continue;
        for (int c = 0; c < kBV; ++c) {
            const Voxel& V = B->v[c];
            double gh[3];
            if (!photo_surface(V, M->vs, gh)) continue;
            int m[3] = {8 * keys[3 * b] + c % 8, 8 * keys[3 * b + 1] + (c / 8) % 8, 8 * keys[3 * b + 2] + c / 64};
            double p[3];
            for (int k = 0; k < 3; ++k) p[k] = M->vs * m[k] - V.psi * gh[k];
            double sum[3] = {0, 0, 0}, n = 0;
            for (int i = 0; i < K; ++i) {
                PhotoSample S;
                if (!photo_visible(*cam, depth + i * npx, &T[12 * i], p, gh, M->T, &S)) continue;
                double I[3], dIu[3], dIv[3];
                bilinear3(rgb + 3 * i * npx, *cam, S.u, S.v, I, dIu, dIv);
                for (int ch = 0; ch < 3; ++ch) sum[ch] += I[ch];
                n += 1;
            }
            count_out[b * kBV + c] = n;
            if (n > 0)
                for (int ch = 0; ch < 3; ++ch) colors_out[3 * (b * kBV + c) + ch] = sum[ch] / n;
        }
    }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Implicit photometric bundle-adjustment energy (Sec. 4.2 Eq. (17)-(21)),
// without stored colour: each surface voxel's residuals are taken against
// the mean of its own samples over the keyframes that see it,
//   E = lambda sum_{i,j,c} nu_ij Phi(I_ij^c - (1/N_j) sum_k nu_kj I_kj^c),
// Phi the Huber penalty, surface points, visibility and samples as in
// orc_photo_loss_grad.  coupled = 1 differentiates through the mean
// (Eq. (17)); coupled = 0 holds the mean fixed (the decoupled Eq. (20)).
// With Phi' the Huber derivative, sample (i, j) contributes with weight
// Phi'(r_ij) - [coupled] (1/N_j) sum_k Phi'(r_kj) on dI_ij.  loss_kf gets
// each keyframe's share; gradients (optional, overwritten) as
// orc_photo_loss_grad (dpsi per keys order, dxi through Jl^T).
// ---------------------------------------------------------------------------
extern "C" double orc_photo_energy(const OrcMap* M, int K, const double* depth, const double* rgb,
                                   const OrcCam* cam, const double* T0, const double* xi, const int32_t* keys,
                                   int64_t nkeys, double delta, double lambda, int coupled, double* loss_kf,
                                   double* dpsi, double* dxi) {
    const size_t npx = (size_t)cam->width * cam->height;
    std::vector<double> T((size_t)12 * K), gl((size_t)6 * K, 0.0);
    for (int i = 0; i < K; ++i) {
        double E[12];
        se3_exp(xi + 6 * i, E);
        std::memcpy(&T[12 * i], T0 + 12 * i, 12 * sizeof(double));
        compose_left(E, &T[12 * i]);
        loss_kf[i] = 0.0;
    }
    if (dpsi) std::fill(dpsi, dpsi + nkeys * kBV, 0.0);
    struct Sample {
        int i;
        PhotoSample S;
        double I[3], dIu[3], dIv[3];
    };
    std::vector<Sample> smp;
    for (int64_t b = 0; b < nkeys; ++b) {
        const Block* B = find_block(M, keys[3 * b], keys[3 * b + 1], keys[3 * b + 2]);
        if (!B) continue;
        for (int c = 0; c < kBV; ++c) {
            const Voxel& V = B->v[c];
            double gh[3];
            if (!photo_surface(V, M->vs, gh)) continue;
            int m[3] = {8 * keys[3 * b] + c % 8, 8 * keys[3 * b + 1] + (c / 8) % 8, 8 * keys[3 * b + 2] + c / 64};
            double p[3];
            for (int k = 0; k < 3; ++k) p[k] = M->vs * m[k] - V.psi * gh[k];
            smp.clear();
            for (int i = 0; i < K; ++i) {
                Sample s;
                s.i = i;
                if (!photo_visible(*cam, depth + i * npx, &T[12 * i], p, gh, M->T, &s.S)) continue;
                bilinear3(rgb + 3 * i * npx, *cam, s.S.u, s.S.v, s.I, s.dIu, s.dIv);
                smp.push_back(s);
            }
            const double N = (double)smp.size();
            if (smp.empty()) continue;
            double mean[3] = {0, 0, 0};
            for (const Sample& s : smp)
                for (int ch = 0; ch < 3; ++ch) mean[ch] += s.I[ch];
            for (int ch = 0; ch < 3; ++ch) mean[ch] /= N;
            double mphi[3] = {0, 0, 0};   // mean of Phi' over the samples, per channel
            for (const Sample& s : smp)
                for (int ch = 0; ch < 3; ++ch) {
                    double r = s.I[ch] - mean[ch];
                    mphi[ch] += huber_weight(r, delta) * r / N;
                }
            for (const Sample& s : smp) {
                double eu = 0, ev = 0;
                for (int ch = 0; ch < 3; ++ch) {
                    double r = s.I[ch] - mean[ch];
                    loss_kf[s.i] += lambda * huber_rho(r, delta);
                    double wgt = lambda * (huber_weight(r, delta) * r - (coupled ? mphi[ch] : 0.0));
                    eu += wgt * s.dIu[ch];
                    ev += wgt * s.dIv[ch];
                }
                const double* Ti = &T[12 * s.i];
                double gx[3] = {eu * cam->fx / s.S.z, ev * cam->fy / s.S.z,
                                -(eu * cam->fx * s.S.x[0] + ev * cam->fy * s.S.x[1]) / (s.S.z * s.S.z)};
                double a[3];
                for (int r = 0; r < 3; ++r) a[r] = Ti[4 * r] * gx[0] + Ti[4 * r + 1] * gx[1] + Ti[4 * r + 2] * gx[2];
                if (dpsi) dpsi[b * kBV + c] -= a[0] * gh[0] + a[1] * gh[1] + a[2] * gh[2];
                double* g6 = &gl[6 * s.i];
                g6[0] -= a[0];
                g6[1] -= a[1];
                g6[2] -= a[2];
                g6[3] += a[1] * p[2] - a[2] * p[1];
                g6[4] += a[2] * p[0] - a[0] * p[2];
                g6[5] += a[0] * p[1] - a[1] * p[0];
            }
        }
    }
    if (dxi) {
        for (int i = 0; i < K; ++i) {
            double Jl[36];
            se3_left_jacobian(xi + 6 * i, Jl);
            for (int q = 0; q < 6; ++q) {
                double s = 0;
                for (int k = 0; k < 6; ++k) s += Jl[6 * k + q] * gl[6 * i + k];
                dxi[6 * i + q] = s;
            }
        }
    }
    double L = 0;
    for (int i = 0; i < K; ++i) L += loss_kf[i];
    return L;
}

// ---------------------------------------------------------------------------
// Oriented point cloud (Sec. 4.3): every observed voxel whose surface point
// lies inside its cell, |psi_j gh_jk| <= v_s/2 for k = x, y, z, gives the
// point v_j - psi_j gh_j with normal -gh_j (outwards: gh points into the
// solid).  Upsampled (level 1): each voxel is split into 2x2x2 subvoxels
// with centres s = v_j + (v_s/4)(+-1, +-1, +-1); the Taylor expansion
// psi(s) = psi_j + gh_j . (s - v_j) gives their distance, and subvoxels with
// |psi(s) gh_jk| <= v_s/4 give s - psi(s) gh_j.  Subvoxel index
// sx + 2 sy + 4 sz (s? = 1 for the + side).  Output in the order of `keys`,
// voxel lx + 8 ly + 64 lz, then subvoxel; returns the count (arrays of
// capacity `cap`; ids: voxel coordinates and subvoxel, 4 int32 each).
// ---------------------------------------------------------------------------
extern "C" int64_t orc_extract_surfels(const OrcMap* M, const int32_t* keys, int64_t nkeys, int level,
                                       double* points, double* normals, int32_t* ids, int64_t cap) {
    int64_t n = 0;
    const double vs = M->vs;
    for (int64_t b = 0; b < nkeys; ++b) {
        const Block* B = find_block(M, keys[3 * b], keys[3 * b + 1], keys[3 * b + 2]);
        if (!B) continue;
        for (int c = 0; c < kBV; ++c) {
            const Voxel& V = B->v[c];
            const double ng = std::sqrt(V.g[0] * V.g[0] + V.g[1] * V.g[1] + V.g[2] * V.g[2]);
            if (!(V.W > 0.0) || !(ng > 0.0)) continue;
            const double gh[3] = {V.g[0] / ng, V.g[1] / ng, V.g[2] / ng};
            const int m[3] = {8 * keys[3 * b] + c % 8, 8 * keys[3 * b + 1] + (c / 8) % 8, 8 * keys[3 * b + 2] + c / 64};
            const double v[3] = {vs * m[0], vs * m[1], vs * m[2]};
            const int nsub = level == 0 ? 1 : 8;
            for (int sub = 0; sub < nsub; ++sub) {
                double s[3], psi = V.psi, half = vs / 2;
                if (level == 0) {
                    for (int k = 0; k < 3; ++k) s[k] = v[k];
                } else {
                    half = vs / 4;
                    for (int k = 0; k < 3; ++k) s[k] = v[k] + ((sub >> k) & 1 ? vs / 4 : -vs / 4);
                    psi = V.psi + gh[0] * (s[0] - v[0]) + gh[1] * (s[1] - v[1]) + gh[2] * (s[2] - v[2]);
                }
                bool inside = true;
                for (int k = 0; k < 3; ++k) inside = inside && std::fabs(psi * gh[k]) <= half;
                if (!inside) continue;
                if (n < cap) {
                    for (int k = 0; k < 3; ++k) {
                        points[3 * n + k] = s[k] - psi * gh[k];
                        normals[3 * n + k] = -gh[k];
                    }
                    ids[4 * n] = m[0];
                    ids[4 * n + 1] = m[1];
                    ids[4 * n + 2] = m[2];
                    ids[4 * n + 3] = level == 0 ? 0 : sub;
                }
                ++n;
            }
        }
    }
    return n;
}

// ---------------------------------------------------------------------------
// Gradient quality (Sec. 5.2, App. A): the stored gradient and finite
// differences of the stored distance, each against the gradient of a known
// union of spheres.
//
// Finite differences of psi at voxel m with step v_s along axis k:
//   forward  (psi(m + e_k) - psi(m)) / v_s
//   backward (psi(m) - psi(m - e_k)) / v_s
//   central  (psi(m + e_k) - psi(m - e_k)) / (2 v_s)
// defined when the voxel and its six face neighbours are observed (W > 0).
// Output per voxel in the order of `keys`, voxel lx + 8 ly + 64 lz: three
// doubles per scheme, valid[i] = 1 where defined (vectors zero elsewhere).
// ---------------------------------------------------------------------------
extern "C" void orc_fd_gradients(const OrcMap* M, const int32_t* keys, int64_t nkeys, double* fwd, double* bwd,
                                 double* cen, uint8_t* valid) {
    const double vs = M->vs;
    for (int64_t b = 0; b < nkeys; ++b) {
        for (int c = 0; c < kBV; ++c) {
            const int64_t i = b * kBV + c;
            const I3 m = {8 * keys[3 * b] + c % 8, 8 * keys[3 * b + 1] + (c / 8) % 8, 8 * keys[3 * b + 2] + c / 64};
            valid[i] = 0;
            for (int k = 0; k < 3; ++k) fwd[3 * i + k] = bwd[3 * i + k] = cen[3 * i + k] = 0.0;
            const Voxel* V = find_voxel(M, m);
            if (!V || !(V->W > 0.0)) continue;
            const Voxel* P[3];
            const Voxel* N[3];
            bool ok = true;
            for (int k = 0; k < 3; ++k) {
                I3 p = m, n = m;
                (k == 0 ? p.x : k == 1 ? p.y : p.z) += 1;
                (k == 0 ? n.x : k == 1 ? n.y : n.z) -= 1;
                P[k] = find_voxel(M, p);
                N[k] = find_voxel(M, n);
                ok = ok && P[k] && P[k]->W > 0.0 && N[k] && N[k]->W > 0.0;
            }
            if (!ok) continue;
            valid[i] = 1;
            for (int k = 0; k < 3; ++k) {
                fwd[3 * i + k] = (P[k]->psi - V->psi) / vs;
                bwd[3 * i + k] = (V->psi - N[k]->psi) / vs;
                cen[3 * i + k] = (P[k]->psi - N[k]->psi) / (2.0 * vs);
            }
        }
    }
}

namespace {

// Angle between two vectors in degrees, atan2(|a x b|, a . b).
double angle_deg(const double a[3], const double b[3]) {
    const double x[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    const double s = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double d = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    return std::atan2(s, d) * (180.0 / M_PI);
}

}  // namespace

// Per observed voxel v (W > 0, g != 0) of the map against spheres
// (cx, cy, cz, r) x ns: the nearest sphere surface is the one minimising
// | |v - c| - r |, the true gradient of the distance (positive inside) is
// (c - v)/|c - v|.  out is 5 planes of nkeys*512 doubles:
//   out[0] distance to that surface, out[1] angle of the stored gradient,
//   out[2..4] angles of the forward, backward and central differences;
// NaN where undefined (unobserved voxel, or a missing neighbour for [2..4]).
extern "C" void orc_gradient_quality(const OrcMap* M, const int32_t* keys, int64_t nkeys, const double* spheres,
                                     int ns, double* out) {
    const int64_t nv = nkeys * kBV;
    std::vector<double> f(3 * nv), bk(3 * nv), ce(3 * nv);
    std::vector<uint8_t> ok(nv);
    orc_fd_gradients(M, keys, nkeys, f.data(), bk.data(), ce.data(), ok.data());
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double vs = M->vs;
    for (int64_t b = 0; b < nkeys; ++b) {
        const Block* B = find_block(M, keys[3 * b], keys[3 * b + 1], keys[3 * b + 2]);
        for (int c = 0; c < kBV; ++c) {
            const int64_t i = b * kBV + c;
            for (int q = 0; q < 5; ++q) out[q * nv + i] = nan;
            if (!B) continue;
            const Voxel& V = B->v[c];
            if (!(V.W > 0.0) || !(V.g[0] != 0.0 || V.g[1] != 0.0 || V.g[2] != 0.0) || ns <= 0) continue;
            const double v[3] = {vs * (8 * keys[3 * b] + c % 8), vs * (8 * keys[3 * b + 1] + (c / 8) % 8),
                                 vs * (8 * keys[3 * b + 2] + c / 64)};
            int best = 0;
            double bd = std::numeric_limits<double>::infinity();
            for (int s = 0; s < ns; ++s) {
                const double* S = spheres + 4 * s;
                const double r = std::sqrt((v[0] - S[0]) * (v[0] - S[0]) + (v[1] - S[1]) * (v[1] - S[1]) +
                                           (v[2] - S[2]) * (v[2] - S[2]));
                if (std::fabs(r - S[3]) < bd) {
                    bd = std::fabs(r - S[3]);
                    best = s;
                }
            }
            const double* S = spheres + 4 * best;
            const double gt[3] = {S[0] - v[0], S[1] - v[1], S[2] - v[2]};
            out[i] = bd;
            out[nv + i] = angle_deg(V.g, gt);
            if (ok[i]) {
                out[2 * nv + i] = angle_deg(&f[3 * i], gt);
                out[3 * nv + i] = angle_deg(&bk[3 * i], gt);
                out[4 * nv + i] = angle_deg(&ce[3 * i], gt);
            }
        }
    }
}
