/*
 * FP64 serial CPU oracle of the ensemble local-inertial flood model and its
 * particle filter.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  The product
 * library never links, includes or calls it, and it shares no header, helper
 * or constant with the HIP code.
 *
 * Everything is plain IEEE double arithmetic in the order the formulas are
 * written in the paper, one member at a time, one cell or link at a time.
 * Compile with contraction off (-ffp-contract=off) so that every operation is
 * rounded as written.  One option (wet_fp32) takes the links' wet/dry decision
 * in single precision, for comparisons with a single-precision model from the
 * same float state, where the decision is the model's own (see wet_link_f32).
 *
 * Grid and link convention (Sec. 3.1, the link/cell indexing around Fig. 2):
 * cells are row-major h[r*nx + c], r = 0 is the north edge.  x-links are
 * stored as qx[r*(nx+1) + c], c = 0..nx; link c joins cell (r,c-1) and cell
 * (r,c), so link 0 is the west edge and link nx the east edge.  y-links are
 * qy[r*nx + c], r = 0..ny; link r joins (r-1,c) and (r,c).  Positive discharge
 * points toward +c or +r.  Discharge is per unit width (m^2/s).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

enum { EDGE_N = 0, EDGE_E = 1, EDGE_S = 2, EDGE_W = 3 };
enum { EDGE_WALL = 0, EDGE_OPEN = 1 };

typedef struct {
    int32_t ny, nx;
    double dx;                 /* cell size, dx = dy (Sec. 2.1 Cartesian cells) */
    const double* z;           /* bed elevation [ny*nx] */
    const double* n;           /* Manning n per cell [ny*nx] */
    int32_t edge_kind[4];      /* N, E, S, W: wall or open */
    double edge_slope[4];      /* outward water-surface slope of an open edge */
    const double* rain;        /* rain rate per block, m/s [n_rain] */
    int32_t n_rain;
    double rain_interval;      /* block length, s */
    double alpha;              /* Courant coefficient k of Eq. 4 */
    double h_dry;              /* links with flow depth <= h_dry carry no flow */
    double dt_cap;             /* upper bound on the adaptive step */
    double dt_fixed;           /* > 0: fixed step instead of Eq. 4 */
    double g;
    int32_t wet_fp32;          /* 1: take the wet/dry decision of each link in single precision */
    /* land cover (Sec. 4.1, Table 1); cls NULL: no classes (shared field, member scale) */
    const uint8_t* cls;        /* [ny*nx] class of each cell, < n_classes */
    int32_t n_classes;
    const double* class_runoff; /* [n_classes] fraction of the rain that stays on the surface */
    const int32_t* class_drain; /* [n_classes] 1: the member's drainage rate applies to the class */
    /* inflow hydrographs (Sec. 4.1): edge links with a prescribed discharge into
     * the domain, taken from series that are piecewise constant over the rain
     * blocks (zero outside them); an inflow link replaces the edge's wall or open
     * condition on that link */
    int32_t n_inflow;
    const int32_t* inflow;     /* [n_inflow][3]: edge (N, E, S, W), position along it, series index */
    const double* inflow_q;    /* [n_series][n_rain] inward discharge per unit width, m^2/s */
    int32_t n_series;
} orc_model;

typedef struct {
    double* h;                 /* [ny*nx] */
    double* qx;                /* [ny*(nx+1)] */
    double* qy;                /* [(ny+1)*nx] */
    double t;
    double s;                  /* member scale on the Manning field */
    double mu;                 /* member multiplier on the rain series */
    double v_rain, v_out, v_clamp;
    int64_t steps;
    double* hmax;              /* optional [ny*nx]: running maximum of the depth (Sec. 4.4, Figs. 15-16) */
    const double* class_n;     /* land cover: [n_classes] this member's Manning n of each class */
    double drain_rate;         /* land cover: drainage rate of draining classes, m/s */
    double v_drain;            /* drained volume */
    double v_in;               /* volume that entered through inflow links */
} orc_member;

/* ------------------------------------------------------------------------ */
/* rain forcing: piecewise constant over blocks (Sec. 3.1 step I)            */
/* ------------------------------------------------------------------------ */
static double rain_at(const orc_model* m, double t) {
    double jf = floor(t / m->rain_interval);
    if (jf < 0.0 || jf >= (double)m->n_rain) return 0.0;
    return m->rain[(int64_t)jf];
}

static double next_rain_edge(const orc_model* m, double t) {
    double jf = floor(t / m->rain_interval);
    if (jf + 1.0 > (double)m->n_rain) return INFINITY;
    return (jf + 1.0) * m->rain_interval;
}

/* ------------------------------------------------------------------------ */
/* time step: Eq. 4 with the member's own maximum depth                     */
/* ------------------------------------------------------------------------ */
double orc_dt_cfl(const orc_model* m, const double* h) {
    if (m->dt_fixed > 0.0) return m->dt_fixed;
    double H = 0.0;
    int64_t nc = (int64_t)m->ny * m->nx;
    for (int64_t i = 0; i < nc; ++i)
        if (h[i] > H) H = h[i];
    if (H < m->h_dry) H = m->h_dry;
    double dt = m->alpha * m->dx / sqrt(m->g * H);
    if (dt > m->dt_cap) dt = m->dt_cap;
    return dt;
}

/* ------------------------------------------------------------------------ */
/* link discharge: Eq. 3 flow depth, Eq. 2 semi-implicit friction update    */
/* ------------------------------------------------------------------------ */
/* Wet/dry decision of a link in single precision.  A single-precision model
 * decides whether a link carries flow from its own float numbers, so a
 * comparison with it from the same float state takes that decision the same
 * way: Eq. 3's flow depth written as the depth of the higher water surface's
 * cell minus the positive part of the bed step towards the other cell
 * (dz = z2 - z1), every operation rounded to float, compared with h_dry rounded
 * to float.  Only the decision is taken in float; the discharge stays in
 * double.  Edge links compare the inner depth. */
static int wet_link_f32(const orc_model* m, double h1, double z1, double h2, double z2) {
    const float fh1 = (float)h1, fh2 = (float)h2;
    const float dz = (float)z2 - (float)z1;
    const float d = fh1 - fh2;
    const float hf = (d >= dz) ? fh1 - fmaxf(dz, 0.0f) : fh2 - fmaxf(-dz, 0.0f);
    return hf > (float)m->h_dry;
}

static int wet_edge_f32(const orc_model* m, double h) { return (float)h > (float)m->h_dry; }

/* The same decision in double precision: the difference form of the flow depth
 * rounds differently from the literal one only where the flow depth is within
 * a rounding of h_dry.  Used to compare with a double-precision model from the
 * same state. */
static int wet_link_diff64(const orc_model* m, double h1, double z1, double h2, double z2) {
    const double dz = z2 - z1;
    const double d = h1 - h2;
    const double hf = (d >= dz) ? h1 - fmax(dz, 0.0) : h2 - fmax(-dz, 0.0);
    return hf > m->h_dry;
}

/* Interior link between cell 1 (west or north) and cell 2 (east or south).
 * The donor limiter keeps each link from draining more than a quarter of its
 * upwind cell in one step.  force < 0: the link decides wet/dry itself; 0 or 1:
 * the decision is given (replay of another model's decisions, see
 * orc_step_forced); a link given as wet with no flow depth still carries none. */
static double link_interior(const orc_model* m, double s, double q, double h1, double z1, double n1,
                            double h2, double z2, double n2, double dt, int force) {
    double eta1 = h1 + z1;
    double eta2 = h2 + z2;
    double hf = fmax(eta1, eta2) - fmax(z1, z2);
    int wet = force >= 0 ? (force && hf > 0.0) : m->wet_fp32 ? wet_link_f32(m, h1, z1, h2, z2) : hf > m->h_dry;
    if (!wet) return 0.0;
    double S = (eta2 - eta1) / m->dx;
    double nf = s * 0.5 * (n1 + n2);
    double qn = (q - m->g * hf * dt * S) / (1.0 + m->g * nf * nf * fabs(q) * dt / pow(hf, 7.0 / 3.0));
    if (qn > 0.0)
        qn = fmin(qn, h1 * m->dx / (4.0 * dt));
    else
        qn = fmax(qn, -h2 * m->dx / (4.0 * dt));
    return qn;
}

/* Open edge link, outward discharge qo >= 0 driven by a fixed outward
 * water-surface slope Se; the flow depth is the inner cell's depth. */
static double link_open(const orc_model* m, double s, double qo, double hi, double ni, double Se,
                        double dt, int force) {
    double hf = hi;
    int wet = force >= 0 ? (force && hf > 0.0) : m->wet_fp32 ? wet_edge_f32(m, hi) : hf > m->h_dry;
    if (!wet) return 0.0;
    double nf = s * ni;
    double qn = (qo + m->g * hf * dt * Se) / (1.0 + m->g * nf * nf * fabs(qo) * dt / pow(hf, 7.0 / 3.0));
    qn = fmin(qn, hi * m->dx / (4.0 * dt));
    return fmax(qn, 0.0);
}

/* Inward discharge of the edge link at position pos of edge e at time t, or -1
 * when the link is no inflow link (inflow discharges are >= 0). */
static double inflow_at(const orc_model* m, int e, int pos, double t) {
    for (int32_t k = 0; k < m->n_inflow; ++k) {
        const int32_t* f = m->inflow + 3 * (int64_t)k;
        if (f[0] != e || f[1] != pos) continue;
        double jf = floor(t / m->rain_interval);
        if (jf < 0.0 || jf >= (double)m->n_rain) return 0.0;
        return m->inflow_q[(int64_t)f[2] * m->n_rain + (int64_t)jf];
    }
    return -1.0;
}

/* All new link discharges from the old state (h, qx, qy) at time t.  Returns
 * the outflow volume leaving through open edges during dt; the volume entering
 * through inflow links is added to *vin. */
/* Manning n of cell i for one member: the shared field (scaled at the link by
 * the member's factor s) or, with land-cover classes, the member's value for
 * the cell's class (Table 1), unscaled. */
static double cell_rough(const orc_model* m, const double* class_n, int64_t i) {
    return m->cls ? class_n[m->cls[i]] : m->n[i];
}

/* fwx, fwy: optional wet/dry decisions of every link in the x- and y-link
 * layouts (replay); NULL: every link decides itself. */
static double links_all(const orc_model* m, double s, const double* class_n, const double* h, const double* qx,
                        const double* qy, double dt, double t, double* qxn, double* qyn, double* vin,
                        const uint8_t* fwx, const uint8_t* fwy) {
    if (m->cls) s = 1.0;
    const int ny = m->ny, nx = m->nx;
    const double dx = m->dx;
    double vout = 0.0;
    for (int r = 0; r < ny; ++r) {
        for (int c = 0; c <= nx; ++c) {
            int64_t li = (int64_t)r * (nx + 1) + c;
            if ((c == 0 || c == nx) && inflow_at(m, c == 0 ? EDGE_W : EDGE_E, r, t) >= 0.0) {
                double qi = inflow_at(m, c == 0 ? EDGE_W : EDGE_E, r, t);
                qxn[li] = c == 0 ? qi : -qi;
                *vin += qi * dx * dt;
            } else if (c == 0) {
                int64_t i = (int64_t)r * nx;
                double qo = 0.0;
                if (m->edge_kind[EDGE_W] == EDGE_OPEN)
                    qo = link_open(m, s, -qx[li], h[i], cell_rough(m, class_n, i), m->edge_slope[EDGE_W], dt,
                                   fwx ? fwx[li] : -1);
                qxn[li] = -qo;
                vout += qo * dx * dt;
            } else if (c == nx) {
                int64_t i = (int64_t)r * nx + nx - 1;
                double qo = 0.0;
                if (m->edge_kind[EDGE_E] == EDGE_OPEN)
                    qo = link_open(m, s, qx[li], h[i], cell_rough(m, class_n, i), m->edge_slope[EDGE_E], dt,
                                   fwx ? fwx[li] : -1);
                qxn[li] = qo;
                vout += qo * dx * dt;
            } else {
                int64_t i1 = (int64_t)r * nx + c - 1, i2 = i1 + 1;
                qxn[li] = link_interior(m, s, qx[li], h[i1], m->z[i1], cell_rough(m, class_n, i1), h[i2], m->z[i2],
                                        cell_rough(m, class_n, i2), dt, fwx ? fwx[li] : -1);
            }
        }
    }
    for (int r = 0; r <= ny; ++r) {
        for (int c = 0; c < nx; ++c) {
            int64_t li = (int64_t)r * nx + c;
            if ((r == 0 || r == ny) && inflow_at(m, r == 0 ? EDGE_N : EDGE_S, c, t) >= 0.0) {
                double qi = inflow_at(m, r == 0 ? EDGE_N : EDGE_S, c, t);
                qyn[li] = r == 0 ? qi : -qi;
                *vin += qi * dx * dt;
            } else if (r == 0) {
                int64_t i = c;
                double qo = 0.0;
                if (m->edge_kind[EDGE_N] == EDGE_OPEN)
                    qo = link_open(m, s, -qy[li], h[i], cell_rough(m, class_n, i), m->edge_slope[EDGE_N], dt,
                                   fwy ? fwy[li] : -1);
                qyn[li] = -qo;
                vout += qo * dx * dt;
            } else if (r == ny) {
                int64_t i = (int64_t)(ny - 1) * nx + c;
                double qo = 0.0;
                if (m->edge_kind[EDGE_S] == EDGE_OPEN)
                    qo = link_open(m, s, qy[li], h[i], cell_rough(m, class_n, i), m->edge_slope[EDGE_S], dt,
                                   fwy ? fwy[li] : -1);
                qyn[li] = qo;
                vout += qo * dx * dt;
            } else {
                int64_t i1 = (int64_t)(r - 1) * nx + c, i2 = i1 + nx;
                qyn[li] = link_interior(m, s, qy[li], h[i1], m->z[i1], cell_rough(m, class_n, i1), h[i2], m->z[i2],
                                        cell_rough(m, class_n, i2), dt, fwy ? fwy[li] : -1);
            }
        }
    }
    return vout;
}

/* Eq. 1 with the volume change of Eq. 5 taken over the four links of the
 * cell as indexed in Sec. 3.1 (west/east x-links, north/south y-links), using
 * the new discharges, plus the rain depth of this step.  Writes the unclamped
 * depth to hu (may alias nothing). */
/* Rain reaching the surface of cell i: the member's rain depth of the step,
 * times the runoff coefficient of the cell's land-cover class (Sec. 4.1: green
 * land keeps 0.9 of the rain). */
static double cell_rain(const orc_model* m, double rain_depth, int64_t i) {
    return m->cls ? rain_depth * m->class_runoff[m->cls[i]] : rain_depth;
}

static void continuity_unclamped(const orc_model* m, const double* h, const double* qxn,
                                 const double* qyn, double dt, double rain_depth, double* hu) {
    const int ny = m->ny, nx = m->nx;
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            int64_t i = (int64_t)r * nx + c;
            int64_t lx = (int64_t)r * (nx + 1) + c;
            int64_t ly = (int64_t)r * nx + c;
            double dv = qxn[lx] - qxn[lx + 1] + qyn[ly] - qyn[ly + nx];
            hu[i] = h[i] + dt / m->dx * dv + cell_rain(m, rain_depth, i);
        }
}

typedef struct {
    double* qxn;
    double* qyn;
    double* hu;
} orc_scratch;

static int scratch_alloc(const orc_model* m, orc_scratch* w) {
    int64_t nc = (int64_t)m->ny * m->nx;
    w->qxn = (double*)malloc(sizeof(double) * (size_t)(m->ny * (int64_t)(m->nx + 1)));
    w->qyn = (double*)malloc(sizeof(double) * (size_t)((m->ny + 1) * (int64_t)m->nx));
    w->hu = (double*)malloc(sizeof(double) * (size_t)nc);
    if (!w->qxn || !w->qyn || !w->hu) {
        free(w->qxn); free(w->qyn); free(w->hu);
        return ORC_ENOMEM;
    }
    return ORC_OK;
}

static void scratch_free(orc_scratch* w) {
    free(w->qxn); free(w->qyn); free(w->hu);
}

/* One step of length dt starting at st->t (time is not advanced here). */
static void step_core(const orc_model* m, orc_member* st, double dt, orc_scratch* w, const uint8_t* fwx,
                      const uint8_t* fwy) {
    const int64_t nc = (int64_t)m->ny * m->nx;
    const double area = m->dx * m->dx;
    st->v_out += links_all(m, st->s, st->class_n, st->h, st->qx, st->qy, dt, st->t, w->qxn, w->qyn, &st->v_in,
                           fwx, fwy);
    double rain_depth = st->mu * rain_at(m, st->t) * dt;
    continuity_unclamped(m, st->h, w->qxn, w->qyn, dt, rain_depth, w->hu);
    double rain_cells = 0.0;
    for (int64_t i = 0; i < nc; ++i) {
        double hn = w->hu[i];
        if (hn < 0.0) {
            st->v_clamp += -hn * area;
            hn = 0.0;
        }
        /* drainage of the pipe network (Sec. 4.1): a fixed rate on draining
         * classes, limited by the water the cell holds after the step */
        if (m->cls && m->class_drain[m->cls[i]]) {
            double loss = fmin(st->drain_rate * dt, hn);
            hn -= loss;
            st->v_drain += loss * area;
        }
        st->h[i] = hn;
        if (st->hmax && hn > st->hmax[i]) st->hmax[i] = hn;
        rain_cells += m->cls ? m->class_runoff[m->cls[i]] : 1.0;
    }
    st->v_rain += rain_depth * rain_cells * area;
    memcpy(st->qx, w->qxn, sizeof(double) * (size_t)(m->ny * (int64_t)(m->nx + 1)));
    memcpy(st->qy, w->qyn, sizeof(double) * (size_t)((m->ny + 1) * (int64_t)m->nx));
    st->steps += 1;
}

static int model_valid(const orc_model* m) {
    if (!m || m->ny < 1 || m->nx < 1 || !(m->dx > 0.0) || !m->z || !m->n) return 0;
    if (!(m->g > 0.0) || !(m->h_dry >= 0.0) || !(m->rain_interval > 0.0)) return 0;
    if (m->n_rain < 0 || (m->n_rain > 0 && !m->rain)) return 0;
    if (!(m->dt_fixed > 0.0) && (!(m->alpha > 0.0) || !(m->dt_cap > 0.0))) return 0;
    if (m->cls && (m->n_classes < 1 || m->n_classes > 8 || !m->class_runoff || !m->class_drain)) return 0;
    if (m->n_inflow < 0 || (m->n_inflow > 0 && (!m->inflow || !m->inflow_q || m->n_series < 1))) return 0;
    for (int32_t k = 0; k < m->n_inflow; ++k) {
        const int32_t* f = m->inflow + 3 * (int64_t)k;
        const int32_t len = (f[0] == EDGE_N || f[0] == EDGE_S) ? m->nx : m->ny;
        if (f[0] < 0 || f[0] > 3 || f[1] < 0 || f[1] >= len || f[2] < 0 || f[2] >= m->n_series) return 0;
        for (int32_t j = 0; j < k; ++j)
            if (m->inflow[3 * j] == f[0] && m->inflow[3 * j + 1] == f[1]) return 0;
    }
    for (int64_t j = 0; j < (int64_t)m->n_series * m->n_rain; ++j)
        if (!(m->inflow_q[j] >= 0.0)) return 0;
    return 1;
}

/* Single step with a caller-chosen dt (time advances by dt). */
int orc_step(const orc_model* m, orc_member* st, double dt) {
    if (!model_valid(m) || !st || !(dt > 0.0) || (m->cls && !st->class_n)) return ORC_EINVAL;
    orc_scratch w;
    if (scratch_alloc(m, &w)) return ORC_ENOMEM;
    step_core(m, st, dt, &w, NULL, NULL);
    st->t += dt;
    scratch_free(&w);
    return ORC_OK;
}

/* One step of length dt ending at time t_next, with every link's wet/dry
 * decision taken from wet_x [ny*(nx+1)] and wet_y [(ny+1)*nx] (1 wet, 0 dry)
 * instead of from the state.  This replays a trajectory of another model that
 * took its own decisions (a single-precision model near the h_dry threshold):
 * with the same step lengths and the same decisions, the two trajectories
 * differ by rounding only.  Inflow links keep their prescribed discharge. */
int orc_step_forced(const orc_model* m, orc_member* st, double dt, double t_next, const uint8_t* wet_x,
                    const uint8_t* wet_y) {
    if (!model_valid(m) || !st || !(dt > 0.0) || !wet_x || !wet_y || (m->cls && !st->class_n)) return ORC_EINVAL;
    orc_scratch w;
    if (scratch_alloc(m, &w)) return ORC_ENOMEM;
    step_core(m, st, dt, &w, wet_x, wet_y);
    st->t = t_next;
    scratch_free(&w);
    return ORC_OK;
}

/* Flow depth of every link from depths h, as written in Eq. 3: the higher
 * water surface minus the higher bed; an edge link's flow depth is its inner
 * cell's depth.  hx [ny*(nx+1)], hy [(ny+1)*nx]. */
int orc_link_depths(const orc_model* m, const double* h, double* hx, double* hy) {
    if (!m || !h || !hx || !hy) return ORC_EINVAL;
    const int ny = m->ny, nx = m->nx;
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c <= nx; ++c) {
            int64_t li = (int64_t)r * (nx + 1) + c;
            if (c == 0 || c == nx) {
                hx[li] = h[(int64_t)r * nx + (c == 0 ? 0 : nx - 1)];
            } else {
                int64_t i1 = (int64_t)r * nx + c - 1, i2 = i1 + 1;
                hx[li] = fmax(h[i1] + m->z[i1], h[i2] + m->z[i2]) - fmax(m->z[i1], m->z[i2]);
            }
        }
    for (int r = 0; r <= ny; ++r)
        for (int c = 0; c < nx; ++c) {
            int64_t li = (int64_t)r * nx + c;
            if (r == 0 || r == ny) {
                hy[li] = h[(int64_t)(r == 0 ? 0 : ny - 1) * nx + c];
            } else {
                int64_t i1 = (int64_t)(r - 1) * nx + c, i2 = i1 + nx;
                hy[li] = fmax(h[i1] + m->z[i1], h[i2] + m->z[i2]) - fmax(m->z[i1], m->z[i2]);
            }
        }
    return ORC_OK;
}

/* Wet/dry decision of every link from depths h at time t, the one the next
 * step takes: interior links by their flow depth against h_dry, open edge
 * links by the inner depth, walls and inflow links 0 (no decision).  mode 0:
 * in double as Eq. 3 is written; 1: in single precision (wet_link_f32); 2: in
 * double in the difference form (wet_link_diff64). */
int orc_wet_masks(const orc_model* m, const double* h, double t, int32_t mode, uint8_t* wx, uint8_t* wy) {
    if (!model_valid(m) || !h || !wx || !wy || mode < 0 || mode > 2) return ORC_EINVAL;
    const int fp32 = mode == 1;
    const int ny = m->ny, nx = m->nx;
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c <= nx; ++c) {
            int64_t li = (int64_t)r * (nx + 1) + c;
            if (c == 0 || c == nx) {
                int e = c == 0 ? EDGE_W : EDGE_E;
                double hi = h[(int64_t)r * nx + (c == 0 ? 0 : nx - 1)];
                wx[li] = m->edge_kind[e] == EDGE_OPEN && inflow_at(m, e, r, t) < 0.0 &&
                         (fp32 ? wet_edge_f32(m, hi) : hi > m->h_dry);
            } else {
                int64_t i1 = (int64_t)r * nx + c - 1, i2 = i1 + 1;
                double hf = fmax(h[i1] + m->z[i1], h[i2] + m->z[i2]) - fmax(m->z[i1], m->z[i2]);
                wx[li] = fp32        ? wet_link_f32(m, h[i1], m->z[i1], h[i2], m->z[i2])
                         : mode == 2 ? wet_link_diff64(m, h[i1], m->z[i1], h[i2], m->z[i2])
                                     : hf > m->h_dry;
            }
        }
    for (int r = 0; r <= ny; ++r)
        for (int c = 0; c < nx; ++c) {
            int64_t li = (int64_t)r * nx + c;
            if (r == 0 || r == ny) {
                int e = r == 0 ? EDGE_N : EDGE_S;
                double hi = h[(int64_t)(r == 0 ? 0 : ny - 1) * nx + c];
                wy[li] = m->edge_kind[e] == EDGE_OPEN && inflow_at(m, e, c, t) < 0.0 &&
                         (fp32 ? wet_edge_f32(m, hi) : hi > m->h_dry);
            } else {
                int64_t i1 = (int64_t)(r - 1) * nx + c, i2 = i1 + nx;
                double hf = fmax(h[i1] + m->z[i1], h[i2] + m->z[i2]) - fmax(m->z[i1], m->z[i2]);
                wy[li] = fp32        ? wet_link_f32(m, h[i1], m->z[i1], h[i2], m->z[i2])
                         : mode == 2 ? wet_link_diff64(m, h[i1], m->z[i1], h[i2], m->z[i2])
                                     : hf > m->h_dry;
            }
        }
    return ORC_OK;
}

/* Step size and end time of the next step from time t toward t_end.
 * The step is clipped so that it ends exactly on the next event: a rain block
 * edge or t_end. */
static double plan_step(const orc_model* m, const double* h, double t, double t_end, double* t_next) {
    double dt = orc_dt_cfl(m, h);
    double t_ev = next_rain_edge(m, t);
    if (t_end < t_ev) t_ev = t_end;
    if (dt >= t_ev - t) {
        dt = t_ev - t;
        *t_next = t_ev;
    } else {
        *t_next = t + dt;
    }
    return dt;
}

/* Advance one member to t_end.  Optionally logs the step sizes. */
int orc_advance(const orc_model* m, orc_member* st, double t_end, int64_t max_steps, double* dt_log,
                int64_t dt_log_cap, int64_t* n_steps_out) {
    if (!model_valid(m) || !st || (m->cls && !st->class_n)) return ORC_EINVAL;
    orc_scratch w;
    if (scratch_alloc(m, &w)) return ORC_ENOMEM;
    int64_t k = 0;
    while (st->t < t_end && k < max_steps) {
        double t_next;
        double dt = plan_step(m, st->h, st->t, t_end, &t_next);
        step_core(m, st, dt, &w, NULL, NULL);
        st->t = t_next;
        if (dt_log && k < dt_log_cap) dt_log[k] = dt;
        ++k;
    }
    if (n_steps_out) *n_steps_out = k;
    scratch_free(&w);
    return ORC_OK;
}

double orc_storage(const orc_model* m, const double* h) {
    double s = 0.0;
    int64_t nc = (int64_t)m->ny * m->nx;
    for (int64_t i = 0; i < nc; ++i) s += h[i] * m->dx * m->dx;
    return s;
}

/* Streamflow through a section (Sec. 4.4): the discharges of the links that
 * cross it, accumulated with the orientation of each link, times the cell
 * width.  links [n_links][4]: kind (0 x-link, 1 y-link), r, c in the link
 * indexing of this file (x-link (r, c), c = 0..nx; y-link (r, c), r = 0..ny),
 * sign (+1 or -1).  Returns m^3/s. */
int orc_section_flow(const orc_model* m, const double* qx, const double* qy, int32_t n_links, const int32_t* links,
                     double* q_out) {
    if (!m || n_links < 0 || (n_links > 0 && !links) || !q_out) return ORC_EINVAL;
    double acc = 0.0;
    for (int32_t k = 0; k < n_links; ++k) {
        const int32_t* l = links + 4 * (int64_t)k;
        double q;
        if (l[0] == 0 && l[1] >= 0 && l[1] < m->ny && l[2] >= 0 && l[2] <= m->nx)
            q = qx[(int64_t)l[1] * (m->nx + 1) + l[2]];
        else if (l[0] == 1 && l[1] >= 0 && l[1] <= m->ny && l[2] >= 0 && l[2] < m->nx)
            q = qy[(int64_t)l[1] * m->nx + l[2]];
        else
            return ORC_EINVAL;
        if (l[3] != 1 && l[3] != -1) return ORC_EINVAL;
        acc += (double)l[3] * q;
    }
    *q_out = acc * m->dx;
    return ORC_OK;
}

/* Observation standard deviations of Eq. 9's diagonal covariance.  alpha > 0:
 * relative to the observed value (Sec. 4.4 uses 5 % of each observation),
 * sigma_k = alpha |d_k|, bounded below by floor_k so that an observation of zero
 * keeps a finite likelihood; alpha = 0: sigma_k = floor_k. */
int orc_obs_sigma(int32_t K, const double* d, const double* floor_, double alpha, double* sigma) {
    if (K < 0 || !(alpha >= 0.0)) return ORC_EINVAL;
    for (int32_t k = 0; k < K; ++k) {
        double rel = alpha * fabs(d[k]);
        sigma[k] = rel > floor_[k] ? rel : floor_[k];
        if (!(sigma[k] > 0.0)) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* particle filter: Eqs. 9-12 and systematic resampling                     */
/* ------------------------------------------------------------------------ */
/* Gaussian log-likelihood with diagonal covariance (Eq. 9), the constant
 * normaliser dropped because it cancels in Eq. 11. */
static double log_likelihood(int32_t K, const double* y, const double* d, const double* sigma) {
    double acc = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        double e = (y[k] - d[k]) / sigma[k];
        acc += e * e;
    }
    return -0.5 * acc;
}

/* Posterior weights (Eqs. 10-11) in log space and N_eff (Eq. 12).
 * y is [N*K] member-major. */
int orc_pf_weights(int32_t N, int32_t K, const double* y, const double* d, const double* sigma,
                   const double* logw_prior, double* logw_post, double* w, double* neff) {
    if (N < 1 || K < 0) return ORC_EINVAL;
    double* a = (double*)malloc(sizeof(double) * (size_t)N);
    if (!a) return ORC_ENOMEM;
    for (int32_t i = 0; i < N; ++i) a[i] = logw_prior[i] + log_likelihood(K, y + (int64_t)i * K, d, sigma);
    double M = a[0];
    for (int32_t i = 1; i < N; ++i)
        if (a[i] > M) M = a[i];
    double Z = 0.0;
    for (int32_t i = 0; i < N; ++i) Z += exp(a[i] - M);
    double lz = log(Z);
    double s2 = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        w[i] = exp(a[i] - M) / Z;
        logw_post[i] = a[i] - M - lz;
        s2 += w[i] * w[i];
    }
    *neff = 1.0 / s2;
    free(a);
    return ORC_OK;
}

/* Systematic resampling: N ordered positions (u0 + j)/N of the total weight;
 * member j descends from the first particle whose running weight exceeds its
 * position. */
int orc_systematic(int32_t N, const double* w, double u0, int32_t* anc) {
    if (N < 1 || !(u0 >= 0.0) || !(u0 < 1.0)) return ORC_EINVAL;
    double* C = (double*)malloc(sizeof(double) * (size_t)N);
    if (!C) return ORC_ENOMEM;
    double run = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        run += w[i];
        C[i] = run;
    }
    int32_t i = 0;
    for (int32_t j = 0; j < N; ++j) {
        double tj = ((u0 + (double)j) / (double)N) * C[N - 1];
        while (i < N && !(tj < C[i])) ++i;
        anc[j] = i < N ? i : N - 1;
    }
    free(C);
    return ORC_OK;
}

/* Full filter update; logw is the prior on entry and the posterior on exit
 * (reset to -log N when the ensemble is resampled). */
int orc_pf(int32_t N, int32_t K, const double* y, const double* d, const double* sigma, double* logw,
           double neff_frac, double u0, double* neff, int32_t* anc, int32_t* resampled) {
    double* lp = (double*)malloc(sizeof(double) * (size_t)N);
    double* w = (double*)malloc(sizeof(double) * (size_t)N);
    if (!lp || !w) {
        free(lp); free(w);
        return ORC_ENOMEM;
    }
    int rc = orc_pf_weights(N, K, y, d, sigma, logw, lp, w, neff);
    if (rc) {
        free(lp); free(w);
        return rc;
    }
    if (*neff < neff_frac * (double)N) {
        rc = orc_systematic(N, w, u0, anc);
        for (int32_t i = 0; i < N; ++i) logw[i] = -log((double)N);
        *resampled = 1;
    } else {
        for (int32_t i = 0; i < N; ++i) {
            logw[i] = lp[i];
            anc[i] = i;
        }
        *resampled = 0;
    }
    free(lp);
    free(w);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* discrete adjoint of the step (dt and branches frozen from the forward)   */
/* ------------------------------------------------------------------------ */
/* Interior link with partial derivatives of the new discharge with respect to
 * the old discharge q, the two depths and the link roughness nf. */
static double link_interior_d(const orc_model* m, double s, double q, double h1, double z1, double n1,
                              double h2, double z2, double n2, double dt, double* dq, double* dh1,
                              double* dh2, double* dnf) {
    *dq = *dh1 = *dh2 = *dnf = 0.0;
    double eta1 = h1 + z1;
    double eta2 = h2 + z2;
    int up1 = eta1 >= eta2;
    double hf = (up1 ? eta1 : eta2) - fmax(z1, z2);
    if (m->wet_fp32 ? !wet_link_f32(m, h1, z1, h2, z2) : !(hf > m->h_dry)) return 0.0;
    const double g = m->g, dx = m->dx;
    double S = (eta2 - eta1) / dx;
    double nf = s * 0.5 * (n1 + n2);
    double P = pow(hf, 7.0 / 3.0);
    double A = g * nf * nf * dt / P;
    double D = 1.0 + A * fabs(q);
    double F = (q - g * hf * dt * S) / D;
    double sg = (q > 0.0) - (q < 0.0);
    double dF_dq = (1.0 - F * A * sg) / D;
    double dF_dS = -g * hf * dt / D;
    double dD_dhf = -(7.0 / 3.0) * A * fabs(q) / hf;
    double dF_dhf = (-g * dt * S - F * dD_dhf) / D;
    double dF_dnf = -F * (2.0 * g * nf * dt * fabs(q) / P) / D;
    *dq = dF_dq;
    *dh1 = -dF_dS / dx + (up1 ? dF_dhf : 0.0);
    *dh2 = dF_dS / dx + (up1 ? 0.0 : dF_dhf);
    *dnf = dF_dnf;
    if (F > 0.0) {
        double cap = h1 * dx / (4.0 * dt);
        if (cap < F) {
            *dq = 0.0; *dh1 = dx / (4.0 * dt); *dh2 = 0.0; *dnf = 0.0;
            return cap;
        }
    } else {
        double cap = -h2 * dx / (4.0 * dt);
        if (F < cap) {
            *dq = 0.0; *dh1 = 0.0; *dh2 = -dx / (4.0 * dt); *dnf = 0.0;
            return cap;
        }
    }
    return F;
}

static double link_open_d(const orc_model* m, double s, double qo, double hi, double ni, double Se,
                          double dt, double* dq, double* dh, double* dnf) {
    *dq = *dh = *dnf = 0.0;
    double hf = hi;
    if (m->wet_fp32 ? !wet_edge_f32(m, hi) : !(hf > m->h_dry)) return 0.0;
    const double g = m->g, dx = m->dx;
    double nf = s * ni;
    double P = pow(hf, 7.0 / 3.0);
    double A = g * nf * nf * dt / P;
    double D = 1.0 + A * fabs(qo);
    double F = (qo + g * hf * dt * Se) / D;
    double sg = (qo > 0.0) - (qo < 0.0);
    *dq = (1.0 - F * A * sg) / D;
    double dD_dhf = -(7.0 / 3.0) * A * fabs(qo) / hf;
    *dh = (g * dt * Se - F * dD_dhf) / D;
    *dnf = -F * (2.0 * g * nf * dt * fabs(qo) / P) / D;
    double cap = hi * dx / (4.0 * dt);
    if (cap < F) {
        *dq = 0.0; *dh = dx / (4.0 * dt); *dnf = 0.0;
        F = cap;
    }
    if (F < 0.0) {
        *dq = *dh = *dnf = 0.0;
        F = 0.0;
    }
    return F;
}

typedef struct {
    double* lhe;    /* adjoint of the new depth after the clamp branch, [ny*nx] */
    double* lh2;    /* adjoint of the old depth being accumulated, [ny*nx] */
    orc_scratch w;
} adj_scratch;

/* Reverse one step.  On entry lh, lqx, lqy hold the adjoint of the state
 * after the step; on exit the adjoint of the state before it.  The Manning
 * field adjoint is accumulated into gn and the rain multiplier adjoint into
 * *gmu.  h, qx, qy are the state before the step; t its start time. */
static void adj_step(const orc_model* m, double s, double mu, const double* h, const double* qx,
                     const double* qy, double dt, double t, double* lh, double* lqx, double* lqy,
                     double* gn, double* gmu, adj_scratch* a) {
    const int ny = m->ny, nx = m->nx;
    const double dx = m->dx;
    const int64_t nc = (int64_t)ny * nx;
    const double R = rain_at(m, t);
    /* forward recomputation to recover the clamp branch */
    double vin = 0.0;          /* no inflow links here: the adjoint refuses them */
    links_all(m, s, NULL, h, qx, qy, dt, t, a->w.qxn, a->w.qyn, &vin, NULL, NULL);
    continuity_unclamped(m, h, a->w.qxn, a->w.qyn, dt, mu * R * dt, a->w.hu);
    double gm = 0.0;
    for (int64_t i = 0; i < nc; ++i) {
        a->lhe[i] = (a->w.hu[i] < 0.0) ? 0.0 : lh[i];
        gm += a->lhe[i] * R * dt;
        a->lh2[i] = a->lhe[i];
    }
    *gmu += gm;
    const double k = dt / dx;
    /* x-links */
    for (int r = 0; r < ny; ++r) {
        for (int c = 0; c <= nx; ++c) {
            int64_t li = (int64_t)r * (nx + 1) + c;
            double dq, dh1, dh2, dnf;
            if (c == 0) {
                int64_t i = (int64_t)r * nx;
                double lt = lqx[li] + k * a->lhe[i];
                if (m->edge_kind[EDGE_W] == EDGE_OPEN) {
                    link_open_d(m, s, -qx[li], h[i], m->n[i], m->edge_slope[EDGE_W], dt, &dq, &dh1, &dnf);
                    /* stored link value is -qo(-q) */
                    lqx[li] = lt * dq;
                    a->lh2[i] += -lt * dh1;
                    gn[i] += -lt * dnf * s;
                } else {
                    lqx[li] = 0.0;
                }
            } else if (c == nx) {
                int64_t i = (int64_t)r * nx + nx - 1;
                double lt = lqx[li] - k * a->lhe[i];
                if (m->edge_kind[EDGE_E] == EDGE_OPEN) {
                    link_open_d(m, s, qx[li], h[i], m->n[i], m->edge_slope[EDGE_E], dt, &dq, &dh1, &dnf);
                    lqx[li] = lt * dq;
                    a->lh2[i] += lt * dh1;
                    gn[i] += lt * dnf * s;
                } else {
                    lqx[li] = 0.0;
                }
            } else {
                int64_t i1 = (int64_t)r * nx + c - 1, i2 = i1 + 1;
                double lt = lqx[li] + k * (a->lhe[i2] - a->lhe[i1]);
                link_interior_d(m, s, qx[li], h[i1], m->z[i1], m->n[i1], h[i2], m->z[i2], m->n[i2], dt,
                                &dq, &dh1, &dh2, &dnf);
                lqx[li] = lt * dq;
                a->lh2[i1] += lt * dh1;
                a->lh2[i2] += lt * dh2;
                gn[i1] += lt * dnf * s * 0.5;
                gn[i2] += lt * dnf * s * 0.5;
            }
        }
    }
    /* y-links */
    for (int r = 0; r <= ny; ++r) {
        for (int c = 0; c < nx; ++c) {
            int64_t li = (int64_t)r * nx + c;
            double dq, dh1, dh2, dnf;
            if (r == 0) {
                int64_t i = c;
                double lt = lqy[li] + k * a->lhe[i];
                if (m->edge_kind[EDGE_N] == EDGE_OPEN) {
                    link_open_d(m, s, -qy[li], h[i], m->n[i], m->edge_slope[EDGE_N], dt, &dq, &dh1, &dnf);
                    lqy[li] = lt * dq;
                    a->lh2[i] += -lt * dh1;
                    gn[i] += -lt * dnf * s;
                } else {
                    lqy[li] = 0.0;
                }
            } else if (r == ny) {
                int64_t i = (int64_t)(ny - 1) * nx + c;
                double lt = lqy[li] - k * a->lhe[i];
                if (m->edge_kind[EDGE_S] == EDGE_OPEN) {
                    link_open_d(m, s, qy[li], h[i], m->n[i], m->edge_slope[EDGE_S], dt, &dq, &dh1, &dnf);
                    lqy[li] = lt * dq;
                    a->lh2[i] += lt * dh1;
                    gn[i] += lt * dnf * s;
                } else {
                    lqy[li] = 0.0;
                }
            } else {
                int64_t i1 = (int64_t)(r - 1) * nx + c, i2 = i1 + nx;
                double lt = lqy[li] + k * (a->lhe[i2] - a->lhe[i1]);
                link_interior_d(m, s, qy[li], h[i1], m->z[i1], m->n[i1], h[i2], m->z[i2], m->n[i2], dt,
                                &dq, &dh1, &dh2, &dnf);
                lqy[li] = lt * dq;
                a->lh2[i1] += lt * dh1;
                a->lh2[i2] += lt * dh2;
                gn[i1] += lt * dnf * s * 0.5;
                gn[i2] += lt * dnf * s * 0.5;
            }
        }
    }
    memcpy(lh, a->lh2, sizeof(double) * (size_t)nc);
}

/* Record of a forward run used by the adjoint and by frozen-step replays:
 * per step its length, its end time and the index of the sample it ends on
 * (-1 when it ends between samples). */
typedef struct {
    int64_t n_steps;
    int64_t cap;
    double* dt;
    double* t_end;
    int32_t* sample;
} orc_record;

static int rec_push(orc_record* r, double dt, double te, int32_t smp) {
    if (r->n_steps == r->cap) {
        int64_t nc = r->cap ? 2 * r->cap : 1024;
        double* a = (double*)realloc(r->dt, sizeof(double) * (size_t)nc);
        if (!a) return ORC_ENOMEM;
        r->dt = a;
        double* b = (double*)realloc(r->t_end, sizeof(double) * (size_t)nc);
        if (!b) return ORC_ENOMEM;
        r->t_end = b;
        int32_t* c = (int32_t*)realloc(r->sample, sizeof(int32_t) * (size_t)nc);
        if (!c) return ORC_ENOMEM;
        r->sample = c;
        r->cap = nc;
    }
    r->dt[r->n_steps] = dt;
    r->t_end[r->n_steps] = te;
    r->sample[r->n_steps] = smp;
    r->n_steps++;
    return ORC_OK;
}

static double misfit(const orc_model* m, const double* h, int32_t K, const int32_t* grc, const double* d) {
    double L = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        double e = h[(int64_t)grc[2 * k] * m->nx + grc[2 * k + 1]] - d[k];
        L += e * e;
    }
    return L;
}

/* Number of samples at t0 + s*sample_dt, s = 1..S, not beyond t_end. */
static int32_t n_samples(double t0, double t_end, double sample_dt) {
    return (int32_t)floor((t_end - t0) / sample_dt + 1e-9);
}

/* Forward run from the member's state to t_end with steps clipped to the
 * sample times, recording the steps and summing the gauge misfit
 * L = sum over samples and gauges of (h - d)^2.  When `replay` is given its
 * step lengths and end times are used instead of Eq. 4 (frozen-step replay). */
static int forward_loss(const orc_model* m, orc_member* st, double t_end, double sample_dt, int32_t K,
                        const int32_t* grc, const double* obs, const orc_record* replay, orc_record* rec,
                        double* loss, double** ckpt, int32_t ckpt_every, int64_t* n_ckpt) {
    orc_scratch w;
    if (scratch_alloc(m, &w)) return ORC_ENOMEM;
    const double t0 = st->t;
    const int32_t S = n_samples(t0, t_end, sample_dt);
    const int64_t nc = (int64_t)m->ny * m->nx;
    const int64_t nqx = (int64_t)m->ny * (m->nx + 1), nqy = (int64_t)(m->ny + 1) * m->nx;
    double L = 0.0;
    int64_t n = 0;
    int rc = ORC_OK;
    for (int32_t smp = 0; smp < S && rc == ORC_OK; ++smp) {
        double ts = t0 + (double)(smp + 1) * sample_dt;
        while (st->t < ts) {
            if (ckpt && n % ckpt_every == 0) {
                int64_t c = n / ckpt_every;
                double* buf = (double*)malloc(sizeof(double) * (size_t)(nc + nqx + nqy));
                if (!buf) { rc = ORC_ENOMEM; break; }
                memcpy(buf, st->h, sizeof(double) * (size_t)nc);
                memcpy(buf + nc, st->qx, sizeof(double) * (size_t)nqx);
                memcpy(buf + nc + nqx, st->qy, sizeof(double) * (size_t)nqy);
                ckpt[c] = buf;
                *n_ckpt = c + 1;
            }
            double dt, t_next;
            if (replay) {
                if (n >= replay->n_steps) { rc = ORC_EINVAL; break; }
                dt = replay->dt[n];
                t_next = replay->t_end[n];
            } else {
                dt = plan_step(m, st->h, st->t, ts, &t_next);
            }
            step_core(m, st, dt, &w, NULL, NULL);
            st->t = t_next;
            int32_t tag = (st->t >= ts) ? smp : -1;
            if (rec && rec_push(rec, dt, t_next, tag)) { rc = ORC_ENOMEM; break; }
            ++n;
        }
        if (rc) break;
        L += misfit(m, st->h, K, grc, obs + (int64_t)smp * K);
    }
    scratch_free(&w);
    *loss = L;
    return rc;
}

#define ORC_MAX_CKPT 1000000

/* Gauge-misfit loss of one member over samples at t0 + s*sample_dt.  With
 * `replay_dt`/`replay_tend` (length n_replay) the forward reuses those step
 * lengths and end times; otherwise it chooses them by Eq. 4. */
int orc_loss(const orc_model* m, orc_member* st, double t_end, double sample_dt, int32_t K,
             const int32_t* grc, const double* obs, const double* replay_dt, const double* replay_tend,
             int64_t n_replay, double* loss) {
    if (!model_valid(m) || !st || !(sample_dt > 0.0) || m->n_inflow) return ORC_EINVAL;
    orc_record rp = {n_replay, n_replay, (double*)replay_dt, (double*)replay_tend, NULL};
    return forward_loss(m, st, t_end, sample_dt, K, grc, obs, replay_dt ? &rp : NULL, NULL, loss, NULL,
                        1, NULL);
}

/* Gradient of the gauge-misfit loss of one member with respect to the shared
 * Manning field (accumulated into grad_n, [ny*nx]) and the member's rain
 * multiplier (written to *grad_mu).  Forward steps are recorded, the state is
 * checkpointed every ckpt_every steps and each segment is recomputed into a
 * tape before it is reversed.  The member state is advanced to t_end.
 * The step lengths/end times are written to dt_out/tend_out when given
 * (capacity out_cap; *n_steps_out always receives the count). */
int orc_adjoint(const orc_model* m, orc_member* st, double t_end, double sample_dt, int32_t K,
                const int32_t* grc, const double* obs, int32_t ckpt_every, double* loss, double* grad_n,
                double* grad_mu, double* dt_out, double* tend_out, int64_t out_cap, int64_t* n_steps_out) {
    if (!model_valid(m) || !st || !(sample_dt > 0.0) || ckpt_every < 1 || m->cls || m->n_inflow) return ORC_EINVAL;
    const int64_t nc = (int64_t)m->ny * m->nx;
    const int64_t nqx = (int64_t)m->ny * (m->nx + 1), nqy = (int64_t)(m->ny + 1) * m->nx;
    const int64_t nst = nc + nqx + nqy;
    const double t0 = st->t;
    orc_record rec = {0, 0, NULL, NULL, NULL};
    double** ckpt = (double**)calloc(ORC_MAX_CKPT, sizeof(double*));
    if (!ckpt) return ORC_ENOMEM;
    int64_t n_ckpt = 0;
    int rc = forward_loss(m, st, t_end, sample_dt, K, grc, obs, NULL, &rec, loss, ckpt, ckpt_every, &n_ckpt);
    if (n_steps_out) *n_steps_out = rec.n_steps;
    if (rc == ORC_OK && dt_out && tend_out) {
        for (int64_t i = 0; i < rec.n_steps && i < out_cap; ++i) {
            dt_out[i] = rec.dt[i];
            tend_out[i] = rec.t_end[i];
        }
    }
    double* tape = NULL;
    double* lh = (double*)calloc((size_t)nc, sizeof(double));
    double* lqx = (double*)calloc((size_t)nqx, sizeof(double));
    double* lqy = (double*)calloc((size_t)nqy, sizeof(double));
    adj_scratch as;
    as.lhe = (double*)malloc(sizeof(double) * (size_t)nc);
    as.lh2 = (double*)malloc(sizeof(double) * (size_t)nc);
    int sa = scratch_alloc(m, &as.w);
    tape = (double*)malloc(sizeof(double) * (size_t)(nst * (int64_t)(ckpt_every + 1)));
    if (rc == ORC_OK && (!lh || !lqx || !lqy || !as.lhe || !as.lh2 || sa || !tape)) rc = ORC_ENOMEM;
    double gmu = 0.0;
    const int32_t S = n_samples(t0, t_end, sample_dt);
    if (rc == ORC_OK) {
        orc_member tm = *st;
        tm.hmax = NULL;    /* recomputation replays steps already taken */
        for (int64_t c = n_ckpt - 1; c >= 0; --c) {
            int64_t n0 = c * ckpt_every;
            int64_t n1 = n0 + ckpt_every;
            if (n1 > rec.n_steps) n1 = rec.n_steps;
            /* recompute the segment into the tape: tape[j] is the state before step n0+j */
            memcpy(tape, ckpt[c], sizeof(double) * (size_t)nst);
            for (int64_t n = n0; n < n1; ++n) {
                double* cur = tape + (n - n0) * nst;
                double* nxt = cur + nst;
                memcpy(nxt, cur, sizeof(double) * (size_t)nst);
                tm.h = nxt; tm.qx = nxt + nc; tm.qy = nxt + nc + nqx;
                tm.t = (n == 0) ? t0 : rec.t_end[n - 1];
                step_core(m, &tm, rec.dt[n], &as.w, NULL, NULL);
            }
            for (int64_t n = n1 - 1; n >= n0; --n) {
                const double* before = tape + (n - n0) * nst;
                const double* after = before + nst;
                int32_t smp = rec.sample[n];
                if (smp >= 0 && smp < S) {
                    const double* d = obs + (int64_t)smp * K;
                    for (int32_t k = 0; k < K; ++k) {
                        int64_t i = (int64_t)grc[2 * k] * m->nx + grc[2 * k + 1];
                        lh[i] += 2.0 * (after[i] - d[k]);
                    }
                }
                double tn = (n == 0) ? t0 : rec.t_end[n - 1];
                adj_step(m, st->s, st->mu, before, before + nc, before + nc + nqx, rec.dt[n], tn, lh, lqx, lqy,
                         grad_n, &gmu, &as);
            }
        }
    }
    *grad_mu = gmu;
    for (int64_t c = 0; c < n_ckpt; ++c) free(ckpt[c]);
    free(ckpt);
    free(tape);
    free(lh); free(lqx); free(lqy);
    free(as.lhe); free(as.lh2);
    if (!sa) scratch_free(&as.w);
    free(rec.dt); free(rec.t_end); free(rec.sample);
    return rc;
}

/* Adjoint of a single step with a given dt (for transpose checks). */
int orc_adj_step(const orc_model* m, double s, double mu, const double* h, const double* qx, const double* qy,
                 double dt, double t, double* lh, double* lqx, double* lqy, double* grad_n, double* grad_mu) {
    if (!model_valid(m) || !(dt > 0.0) || m->cls || m->n_inflow) return ORC_EINVAL;
    const int64_t nc = (int64_t)m->ny * m->nx;
    adj_scratch as;
    as.lhe = (double*)malloc(sizeof(double) * (size_t)nc);
    as.lh2 = (double*)malloc(sizeof(double) * (size_t)nc);
    if (!as.lhe || !as.lh2 || scratch_alloc(m, &as.w)) {
        free(as.lhe); free(as.lh2);
        return ORC_ENOMEM;
    }
    double gmu = 0.0;
    adj_step(m, s, mu, h, qx, qy, dt, t, lh, lqx, lqy, grad_n, &gmu, &as);
    *grad_mu += gmu;
    free(as.lhe); free(as.lh2);
    scratch_free(&as.w);
    return ORC_OK;
}
