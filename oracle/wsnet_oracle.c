/*
 * FP64 CPU oracle of the learned warm-start network.
 *
 * TEST INFRASTRUCTURE ONLY (called by the tests, never by the GPU library).
 *
 * The network maps the normalised backprojection of a scan, laid out as an
 * image of ny x nx pixels with Q channels (one per spectral bin; NHWC, the
 * voxel order of the reconstruction), to a nonnegative start image:
 *   L layers of 3x3 convolution with zero padding 1, C channels in and out,
 *   weights [co][ky][kx][ci] and a bias per output channel,
 *   ReLU after layers 1..L-1, softplus after layer L.
 * Loss: mean squared error against a target image.  Parameters are stored
 * flat, layer by layer: weights (C*9*C) then bias (C).
 * Plain loops, IEEE double, fixed order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* z[n][y][x][co] = b[co] + sum_{ky,kx,ci} w[co][ky][kx][ci] x[n][y+ky-1][x+kx-1][ci] */
void wn_conv_fwd(int B, int H, int W, int Ci, int Co, const double *x, const double *w,
                 const double *b, double *z)
{
    for (int n = 0; n < B; ++n)
        for (int y = 0; y < H; ++y)
            for (int xx = 0; xx < W; ++xx)
                for (int co = 0; co < Co; ++co) {
                    double acc = b ? b[co] : 0.0;
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int sy = y + ky - 1, sx = xx + kx - 1;
                            if (sy < 0 || sy >= H || sx < 0 || sx >= W)
                                continue;
                            const double *xp = x + (((int64_t)n * H + sy) * W + sx) * Ci;
                            const double *wp = w + (((int64_t)co * 3 + ky) * 3 + kx) * Ci;
                            for (int ci = 0; ci < Ci; ++ci)
                                acc += wp[ci] * xp[ci];
                        }
                    z[(((int64_t)n * H + y) * W + xx) * Co + co] = acc;
                }
}

/* dx = d(loss)/dx given dz: each output position scatters dz * w back to
 * the inputs it read. */
void wn_conv_bwd_data(int B, int H, int W, int Ci, int Co, const double *dz, const double *w,
                      double *dx)
{
    memset(dx, 0, sizeof(double) * (size_t)B * H * W * Ci);
    for (int n = 0; n < B; ++n)
        for (int y = 0; y < H; ++y)
            for (int xx = 0; xx < W; ++xx)
                for (int co = 0; co < Co; ++co) {
                    double g = dz[(((int64_t)n * H + y) * W + xx) * Co + co];
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int sy = y + ky - 1, sx = xx + kx - 1;
                            if (sy < 0 || sy >= H || sx < 0 || sx >= W)
                                continue;
                            double *xp = dx + (((int64_t)n * H + sy) * W + sx) * Ci;
                            const double *wp = w + (((int64_t)co * 3 + ky) * 3 + kx) * Ci;
                            for (int ci = 0; ci < Ci; ++ci)
                                xp[ci] += g * wp[ci];
                        }
                }
}

/* dw[co][ky][kx][ci] = sum over positions of dz * x(shifted); db[co] = sum dz */
void wn_conv_bwd_weight(int B, int H, int W, int Ci, int Co, const double *x, const double *dz,
                        double *dw, double *db)
{
    memset(dw, 0, sizeof(double) * (size_t)Co * 9 * Ci);
    if (db)
        memset(db, 0, sizeof(double) * (size_t)Co);
    for (int n = 0; n < B; ++n)
        for (int y = 0; y < H; ++y)
            for (int xx = 0; xx < W; ++xx)
                for (int co = 0; co < Co; ++co) {
                    double g = dz[(((int64_t)n * H + y) * W + xx) * Co + co];
                    if (db)
                        db[co] += g;
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int sy = y + ky - 1, sx = xx + kx - 1;
                            if (sy < 0 || sy >= H || sx < 0 || sx >= W)
                                continue;
                            const double *xp = x + (((int64_t)n * H + sy) * W + sx) * Ci;
                            double *wp = dw + (((int64_t)co * 3 + ky) * 3 + kx) * Ci;
                            for (int ci = 0; ci < Ci; ++ci)
                                wp[ci] += g * xp[ci];
                        }
                }
}

/* softplus(z) = log(1 + e^z), written without overflow */
static double softplus(double z) { return (z > 0 ? z : 0.0) + log1p(exp(-fabs(z))); }
static double sigmoid(double z) { return z >= 0 ? 1.0 / (1.0 + exp(-z)) : exp(z) / (1.0 + exp(z)); }

static int64_t layer_params(int C) { return (int64_t)C * 9 * C + C; }

/*
 * Forward pass of the L-layer network on B images; out receives the start
 * images.  If acts is not NULL it receives the input of every layer
 * (L blocks of B*H*W*C) and zs the pre-activations (L blocks).
 */
void wn_forward(int L, int B, int H, int W, int C, const double *params, const double *x_in,
                double *out, double *acts, double *zs)
{
    size_t n = (size_t)B * H * W * C;
    double *cur = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    memcpy(cur, x_in, sizeof(double) * n);
    for (int l = 0; l < L; ++l) {
        const double *w = params + l * layer_params(C);
        const double *b = w + (int64_t)C * 9 * C;
        if (acts)
            memcpy(acts + l * n, cur, sizeof(double) * n);
        wn_conv_fwd(B, H, W, C, C, cur, w, b, z);
        if (zs)
            memcpy(zs + l * n, z, sizeof(double) * n);
        for (size_t i = 0; i < n; ++i)
            cur[i] = l + 1 < L ? (z[i] > 0 ? z[i] : 0.0) : softplus(z[i]);
    }
    memcpy(out, cur, sizeof(double) * n);
    free(cur);
    free(z);
}

/* Loss = mean over all outputs of (out - target)^2 and its gradient with
 * respect to every parameter (grad laid out like params).  Returns the loss. */
double wn_loss_grad(int L, int B, int H, int W, int C, const double *params, const double *x_in,
                    const double *target, double *grad)
{
    size_t n = (size_t)B * H * W * C;
    double *acts = malloc(sizeof(double) * n * L), *zs = malloc(sizeof(double) * n * L);
    double *out = malloc(sizeof(double) * n), *dz = malloc(sizeof(double) * n);
    double *da = malloc(sizeof(double) * n);
    wn_forward(L, B, H, W, C, params, x_in, out, acts, zs);
    double loss = 0.0;
    for (size_t i = 0; i < n; ++i)
        loss += (out[i] - target[i]) * (out[i] - target[i]);
    loss /= (double)n;
    /* d loss / d z_L = 2 (out - target) / n * softplus'(z_L) */
    for (size_t i = 0; i < n; ++i)
        dz[i] = 2.0 * (out[i] - target[i]) / (double)n * sigmoid(zs[(L - 1) * n + i]);
    for (int l = L - 1; l >= 0; --l) {
        const double *w = params + l * layer_params(C);
        double *gw = grad + l * layer_params(C);
        wn_conv_bwd_weight(B, H, W, C, C, acts + l * n, dz, gw, gw + (int64_t)C * 9 * C);
        if (l == 0)
            break;
        wn_conv_bwd_data(B, H, W, C, C, dz, w, da);
        /* through the ReLU of layer l-1: its output is the input of layer l */
        for (size_t i = 0; i < n; ++i)
            dz[i] = zs[(l - 1) * n + i] > 0 ? da[i] : 0.0;
    }
    free(acts);
    free(zs);
    free(out);
    free(dz);
    free(da);
    return loss;
}

/* One Adam step (Kingma and Ba) on n parameters; t is the 1-based step count. */
void wn_adam(int64_t n, double *p, const double *g, double *m, double *v, int64_t t, double lr,
             double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
