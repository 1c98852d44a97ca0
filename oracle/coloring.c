/*
 * ORACLE (test infrastructure only; never linked by the product library).
 *
 * Greedy graph coloring of a sparse matrix's off-diagonal structure, following
 * the paper's Alg. "Graph Coloring" and App. A: nodes are visited in
 * descending degree (ties: ascending index); each node takes the first palette
 * entry not used by an already-painted neighbour, which is then moved to the
 * back of the palette; if none fits a new color is created and appended.
 * Colors are numbered in order of creation.
 *
 * rowptr/cols: CSR pattern (diagonal entries, if present, are ignored).
 * color: output, one color id per node.  Returns the number of colors.
 */
#include <stdlib.h>

int oracle_color(int n, const int *rowptr, const int *cols, int *color) {
    int *deg = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *order = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int maxdeg = 0;
    for (int i = 0; i < n; ++i) {
        int d = 0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) if (cols[p] != i) d++;
        deg[i] = d;
        if (d > maxdeg) maxdeg = d;
        color[i] = -1;
    }
    /* stable counting sort by descending degree */
    int *bucket = (int *)calloc((size_t)maxdeg + 2, sizeof(int));
    for (int i = 0; i < n; ++i) bucket[maxdeg - deg[i] + 1]++;
    for (int d = 1; d <= maxdeg + 1; ++d) bucket[d] += bucket[d - 1];
    for (int i = 0; i < n; ++i) order[bucket[maxdeg - deg[i]]++] = i;

    int cap = maxdeg + 2;
    int *palette = (int *)malloc(sizeof(int) * (size_t)cap);
    int *seen = (int *)malloc(sizeof(int) * (size_t)cap);
    int npal = 0, ncolors = 0;
    for (int t = 0; t < n; ++t) {
        int i = order[t];
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = cols[p];
            if (j != i && color[j] >= 0) seen[color[j]] = i + 1;  /* stamp */
        }
        int pos = -1;
        for (int s = 0; s < npal; ++s)
            if (seen[palette[s]] != i + 1) { pos = s; break; }
        int c;
        if (pos < 0) {
            c = ncolors++;
            seen[c] = 0;
            palette[npal++] = c;
        } else {
            c = palette[pos];
            for (int s = pos; s + 1 < npal; ++s) palette[s] = palette[s + 1];
            palette[npal - 1] = c;
        }
        color[i] = c;
    }
    free(deg); free(order); free(bucket); free(palette); free(seen);
    return ncolors;
}
