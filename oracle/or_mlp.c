/* Oracle of the learned page-prefetch network (test infrastructure only).
 *
 * A multilayer perceptron with ReLU hidden layers and one logit per page
 * cluster, trained with the mean binary cross-entropy of the logits and Adam.
 * The method's own visibility pass alone decides what renders: the network only adds
 * lowest-priority prefetch requests (the "prefetching" the paper leaves to
 * future work, Sec. 6).  Everything here is plain double-precision loops.
 *
 * With bf16 != 0 the operands of every matrix product are rounded to bf16 at
 * the points where the GPU kernels hold them in bf16: the weights, the input
 * features, each hidden activation after its ReLU, and each layer's output
 * gradient before it enters the two products of the backward pass.  Sums are
 * exact-ish (double); biases and the loss are double.
 *
 * Parameter layout (floats): for each layer l, W_l [d_l][d_{l+1}] row-major
 * (input index major) followed by b_l [d_{l+1}].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define MAXL 8

static double rnd(double x, int bf16) { return bf16 ? (double)or_round_bf16((float)x) : x; }

static int64_t n_params(int n_layers, const int* dims)
{
    int64_t n = 0;
    for (int l = 0; l < n_layers; l++) n += (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
    return n;
}

/* forward pass; acts[l] = operand of layer l ([B][d_l], rounded as used),
 * z = logits [B][d_L] */
static void forward(int B, int nl, const int* dims, const float* params, const float* x, int bf16,
                    double** acts, double* z)
{
    for (int64_t i = 0; i < (int64_t)B * dims[0]; i++) acts[0][i] = rnd(x[i], bf16);
    const float* p = params;
    for (int l = 0; l < nl; l++) {
        int din = dims[l], dout = dims[l + 1];
        const float* W = p;
        const float* b = p + (int64_t)din * dout;
        double* out = l + 1 < nl ? acts[l + 1] : z;
        for (int r = 0; r < B; r++)
            for (int j = 0; j < dout; j++) {
                double s = 0.0;
                for (int k = 0; k < din; k++) s += acts[l][(int64_t)r * din + k] * rnd(W[(int64_t)k * dout + j], bf16);
                s += (double)b[j];
                if (l + 1 < nl) s = rnd(s > 0.0 ? s : 0.0, bf16);   /* ReLU, then the bf16 operand */
                out[(int64_t)r * dout + j] = s;
            }
        p = b + dout;
    }
}

static double** alloc_acts(int B, int nl, const int* dims)
{
    double** a = calloc(MAXL, sizeof(double*));
    for (int l = 0; l < nl; l++) a[l] = malloc(sizeof(double) * (size_t)B * dims[l]);
    return a;
}

static void free_acts(double** a, int nl)
{
    for (int l = 0; l < nl; l++) free(a[l]);
    free(a);
}

/* logits of a batch: z [B][d_L] */
int or_mlp_forward(int B, int n_layers, const int* dims, const float* params, const float* x, int bf16, double* z)
{
    if (n_layers < 1 || n_layers > MAXL) return -1;
    double** acts = alloc_acts(B, n_layers, dims);
    forward(B, n_layers, dims, params, x, bf16, acts, z);
    free_acts(acts, n_layers);
    return 0;
}

/* loss = mean over the B x d_L outputs of softplus(z) - y z (binary
 * cross-entropy of sigmoid(z) against y); grad has the parameter layout.
 * Returns the loss. */
double or_mlp_backward(int B, int n_layers, const int* dims, const float* params, const float* x, const float* y,
                       int bf16, double* grad, double* z)
{
    if (n_layers < 1 || n_layers > MAXL) return NAN;
    int nl = n_layers;
    double** acts = alloc_acts(B, nl, dims);
    forward(B, nl, dims, params, x, bf16, acts, z);
    int dL = dims[nl];
    double inv = 1.0 / ((double)B * dL);
    double loss = 0.0;
    double* dz = malloc(sizeof(double) * (size_t)B * dL);
    for (int64_t i = 0; i < (int64_t)B * dL; i++) {
        double zi = z[i], yi = y[i];
        loss += (zi > 0.0 ? zi : 0.0) + log1p(exp(-fabs(zi))) - yi * zi;
        double s = 1.0 / (1.0 + exp(-zi));
        dz[i] = rnd((s - yi) * inv, bf16);
    }
    loss *= inv;
    /* parameter offsets */
    int64_t off[MAXL + 1];
    off[0] = 0;
    for (int l = 0; l < nl; l++) off[l + 1] = off[l] + (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
    for (int l = nl - 1; l >= 0; l--) {
        int din = dims[l], dout = dims[l + 1];
        const float* W = params + off[l];
        double* gW = grad + off[l];
        double* gb = gW + (int64_t)din * dout;
        /* dW = X^T dZ, db = sum over the batch of dZ */
        for (int k = 0; k < din; k++)
            for (int j = 0; j < dout; j++) {
                double s = 0.0;
                for (int r = 0; r < B; r++) s += acts[l][(int64_t)r * din + k] * dz[(int64_t)r * dout + j];
                gW[(int64_t)k * dout + j] = s;
            }
        for (int j = 0; j < dout; j++) {
            double s = 0.0;
            for (int r = 0; r < B; r++) s += dz[(int64_t)r * dout + j];
            gb[j] = s;
        }
        if (l == 0) break;
        /* dX = dZ W^T, through the ReLU of the layer below */
        double* dx = malloc(sizeof(double) * (size_t)B * din);
        for (int r = 0; r < B; r++)
            for (int k = 0; k < din; k++) {
                double s = 0.0;
                for (int j = 0; j < dout; j++) s += dz[(int64_t)r * dout + j] * rnd(W[(int64_t)k * dout + j], bf16);
                dx[(int64_t)r * din + k] = acts[l][(int64_t)r * din + k] > 0.0 ? rnd(s, bf16) : 0.0;
            }
        free(dz);
        dz = dx;
    }
    free(dz);
    free_acts(acts, nl);
    return loss;
}

/* One Adam step (Kingma and Ba) on float state: m, v moments, step t >= 1. */
void or_adam(int64_t n, float* w, float* m, float* v, const double* g, double lr, double b1, double b2, double eps,
             int t)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int64_t i = 0; i < n; i++) {
        double mi = b1 * m[i] + (1.0 - b1) * g[i];
        double vi = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        m[i] = (float)mi;
        v[i] = (float)vi;
        w[i] = (float)(w[i] - lr * (mi / c1) / (sqrt(vi / c2) + eps));
    }
}

int64_t or_mlp_n_params(int n_layers, const int* dims) { return n_params(n_layers, dims); }
