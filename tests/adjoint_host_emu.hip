// Host build of the adjoint routines (test harness only): the per-face and
// per-cell reverse functions of csrc/swe_adjoint.hip are __host__ __device__;
// this file runs them on the CPU so that tests can compare them with the
// oracle without a GPU.  Nothing here is part of the library.
#include "../paper_1307_4839_amd/csrc/swe_adjoint.hip"  // NOLINT
#include <vector>
extern "C" {
int emu_vjp(const swe_params* prm, const double* z, const double* h, const double* qx,
            const double* qy, const double* mh, const double* mqx, const double* mqy,
            double* oh, double* oqx, double* oqy) {
    KParams p = to_kparams(*prm);
    int nx = p.nx, ny = p.ny;
    size_t px = (size_t)ny * (nx + 1), py = (size_t)(ny + 1) * nx;
    std::vector<double> xc(12 * px), yc(12 * py);
    double out[12];
    const int fl = prm->flux;
    for (int j = 0; j < ny; ++j)
        for (int f = 0; f <= nx; ++f) {
            if (fl == 2) face_contrib<0, 2>(p, z, h, qx, qy, mh, mqx, mqy, f, j, out);
            else if (fl == 1) face_contrib<0, 1>(p, z, h, qx, qy, mh, mqx, mqy, f, j, out);
            else face_contrib<0, 0>(p, z, h, qx, qy, mh, mqx, mqy, f, j, out);
            for (int k = 0; k < 12; ++k) xc[k * px + (size_t)j * (nx + 1) + f] = out[k];
        }
    for (int i = 0; i < nx; ++i)
        for (int f = 0; f <= ny; ++f) {
            if (fl == 2) face_contrib<1, 2>(p, z, h, qx, qy, mh, mqx, mqy, f, i, out);
            else if (fl == 1) face_contrib<1, 1>(p, z, h, qx, qy, mh, mqx, mqy, f, i, out);
            else face_contrib<1, 0>(p, z, h, qx, qy, mh, mqx, mqy, f, i, out);
            for (int k = 0; k < 12; ++k) yc[k * py + (size_t)f * nx + i] = out[k];
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double a, b, c;
            gather_cell(p, xc.data(), yc.data(), i, j, a, b, c);
            oh[j * nx + i] = a; oqx[j * nx + i] = b; oqy[j * nx + i] = c;
        }
    return 0;
}
void emu_face_fwd(double g, const double* in, double* out) {
    FaceOut o = face(g, in[0], in[1], in[2], in[3], in[4], in[5], in[6], in[7]);
    out[0] = o.f0; out[1] = o.fl1; out[2] = o.fr1; out[3] = o.f2;
}
void emu_face_rev(double g, const double* in, const double* bar, double* out) {
    // bar = (F0, F1, F2, sL, sR)
    FaceBar b = face_rev(g, in[0], in[1], in[2], in[3], in[4], in[5], in[6], in[7], bar[0], bar[1], bar[2], bar[3], bar[4]);
    out[0]=b.hm; out[1]=b.zm; out[2]=b.unm; out[3]=b.utm; out[4]=b.hp; out[5]=b.zp; out[6]=b.unp; out[7]=b.utp;
}
void emu_muscl_fwd(const double* a, const double* c, const double* b, double h_eps, double* out) {
    Prim pa{a[0],a[1],a[2],a[3]}, pc{c[0],c[1],c[2],c[3]}, pb{b[0],b[1],b[2],b[3]};
    Rec r = muscl(pa, pc, pb, h_eps);
    double o[8] = {r.h_m, r.h_p, r.z_m, r.z_p, r.un_m, r.un_p, r.ut_m, r.ut_p};
    for (int k = 0; k < 8; ++k) out[k] = o[k];
}
void emu_muscl_rev(const double* a, const double* c, const double* b, double h_eps, const double* rb, double* out) {
    Prim pa{a[0],a[1],a[2],a[3]}, pc{c[0],c[1],c[2],c[3]}, pb{b[0],b[1],b[2],b[3]};
    RecBar R{rb[0],rb[1],rb[2],rb[3],rb[4],rb[5],rb[6],rb[7]};
    PrimBar A, Cc, B; zero(A); zero(Cc); zero(B);
    muscl_rev(pa, pc, pb, h_eps, R, A, Cc, B);
    double o[12] = {A.h,A.un,A.ut,A.eta, Cc.h,Cc.un,Cc.ut,Cc.eta, B.h,B.un,B.ut,B.eta};
    for (int k = 0; k < 12; ++k) out[k] = o[k];
}
void emu_friction_fwd(const swe_params* prm, double coef, const double* in, double dt, double* out) {
    // in = h0 qx0 qy0 h1 qx1 qy1
    KParams p = to_kparams(*prm);
    double qx1 = in[4], qy1 = in[5];
    friction(p, coef, in[0], in[1], in[2], in[3], qx1, qy1, dt);
    out[0] = in[3]; out[1] = qx1; out[2] = qy1;
}
void emu_friction_rev(const swe_params* prm, double coef, const double* in, double dt, const double* bo, double* out) {
    KParams p = to_kparams(*prm);
    double bh1,bqx1,bqy1,bh0,bqx0,bqy0,bc;
    friction_rev(p, coef, in[0], in[1], in[2], in[3], in[4], in[5], dt, bo[0], bo[1], bo[2], bh1,bqx1,bqy1,bh0,bqx0,bqy0,bc);
    out[0]=bh0; out[1]=bqx0; out[2]=bqy0; out[3]=bh1; out[4]=bqx1; out[5]=bqy1; out[6]=bc;
}
}
extern "C" {
void emu_stage_out(const swe_params* prm, const double* fric, const double* h, const double* qx, const double* qy,
                   const double* ph, const double* pqx, const double* pqy, double dt, double* ho, double* qxo, double* qyo) {
    KParams p = to_kparams(*prm);
    size_t n = (size_t)p.nx * p.ny;
    for (size_t i = 0; i < n; ++i) {
        double h1 = h[i] + dt * ph[i], qx1 = qx[i] + dt * pqx[i], qy1 = qy[i] + dt * pqy[i];
        friction(p, fric ? fric[i] : p.coef, h[i], qx[i], qy[i], h1, qx1, qy1, dt);
        ho[i] = h1; qxo[i] = qx1; qyo[i] = qy1;
    }
}
// per-cell reverse of a stage's friction: bo -> lin (set), mu, grad (+=)
void emu_adj_stage(const swe_params* prm, const double* fric, const double* h, const double* qx, const double* qy,
                   const double* ph, const double* pqx, const double* pqy, double dt,
                   const double* boh, const double* boqx, const double* boqy, double scale,
                   double* lh, double* lqx, double* lqy, double* mh, double* mqx, double* mqy, double* grad) {
    KParams p = to_kparams(*prm);
    size_t n = (size_t)p.nx * p.ny;
    for (size_t i = 0; i < n; ++i) {
        double h0 = h[i], qx0 = qx[i], qy0 = qy[i];
        double h1 = h0 + dt * ph[i], qx1 = qx0 + dt * pqx[i], qy1 = qy0 + dt * pqy[i];
        double bh1,bqx1,bqy1,bh0,bqx0,bqy0,bc;
        friction_rev(p, fric ? fric[i] : p.coef, h0, qx0, qy0, h1, qx1, qy1, dt, scale*boh[i], scale*boqx[i], scale*boqy[i], bh1,bqx1,bqy1,bh0,bqx0,bqy0,bc);
        lh[i] = bh1 + bh0; lqx[i] = bqx1 + bqx0; lqy[i] = bqy1 + bqy0;
        mh[i] = dt * bh1; mqx[i] = dt * bqx1; mqy[i] = dt * bqy1;
        grad[i] += bc;
    }
}
}
